// Device helpers shared by the SOAR kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace soar {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr float kInf = __builtin_inff();
constexpr float kU32 = 5.9604644775390625e-08f;   // 2^-24, unit roundoff of float32

// Counters kept in device memory by every assignment call.
enum Counter : int {
  CNT_FULLSCAN = 0,   // rows sent to the exact full scan
  CNT_NONFINITE = 1,  // set when a NaN/Inf was read from X or C
  CNT_FP64 = 2,       // rows whose decision was taken in FP64
  CNT_CMAX2 = 3,      // max_j ||c_j||^2 as float bits (non-negative floats order like uints)
  CNT_BOUNDED = 5,    // rows whose spill candidates came from the spill bound (no sweep)
  CNT_WORDS = 8,      // words of one call's counters (cleared by every call)
  // status record of enqueue-only calls, kept across calls (see async_note_kernel)
  CNT_ASYNC_M0 = 8,
  CNT_ASYNC_M1 = 9,
  CNT_ASYNC_FLAGS = 10,
  CNT_ALLOC_WORDS = 16
};
constexpr unsigned kAsyncMagic0 = 0x534f4152u, kAsyncMagic1 = 0x41535943u;
// Counters cleared at the start of every assignment (the codebook's CNT_CMAX2 is kept).
constexpr int CNT_STEP_WORDS = 3;

// Finiteness by the exponent bits, so that no floating-point mode or flag can fold it away.
__device__ __forceinline__ bool is_finite_bits(float v) {
  return (__builtin_bit_cast(unsigned, v) & 0x7f800000u) != 0x7f800000u;
}
__device__ __forceinline__ bool all_finite4(v4f v) {
  return is_finite_bits(v.x) && is_finite_bits(v.y) && is_finite_bits(v.z) && is_finite_bits(v.w);
}

// Rows to process: the launch capacity, or fewer when a device-side live count is given (graph
// replays of serving steps read the batch size from device memory).
__device__ __forceinline__ int64_t live_rows(int64_t cap, const int64_t* live) {
  if (!live) return cap;
  const int64_t l = *live;
  return l < cap ? (l < 0 ? 0 : l) : cap;
}

// Sum over the 4 lanes that share (lane & 15): lanes l, l^16, l^32, l^48.
__device__ __forceinline__ float sum_quad_f(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
__device__ __forceinline__ double sum_quad_d(double v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// (value, index) lexicographic minimum over the 16 lanes of a lane group (lane >> 4 fixed).
__device__ __forceinline__ void argmin16(float& v, int& j) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) {
    float ov = __shfl_xor(v, off);
    int oj = __shfl_xor(j, off);
    if (ov < v || (ov == v && oj < j)) { v = ov; j = oj; }
  }
}

__device__ __forceinline__ void argmin_d(double& v, int& j, double ov, int oj) {
  if (ov < v || (ov == v && oj < j)) { v = ov; j = oj; }
}

// s_waitcnt on the vector-memory counter alone (gfx9 encoding: vmcnt in bits [3:0] and [15:14];
// expcnt [6:4] and lgkmcnt [11:8] left at their maxima, i.e. not waited on).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Direct global->LDS copies (gfx950 global_load_lds, 16 bytes per lane).
#define LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

// Copy record t into ring stage t % STG with direct global->LDS loads: every wave issues exactly
// NI copies of 64 x 16 bytes (source addresses past the record end are clamped to its last
// chunk), so the number of outstanding copies is the same in every wave.
// The wave index and the LDS destination are wave-uniform (scalar registers); the per-lane source
// offset is a 32-bit unsigned value added to a scalar base.
// record_offsets: the per-lane source offsets of a record copy (the same for every record), so that
// a loop can compute them once and issue each record with issue_record_at.
// NWG: waves of the workgroup that share the copies (each copy round moves NWG x 1 KiB).
template <int BYTES, int NI, int NWG = 4>
__device__ __forceinline__ void record_offsets(int w, int lane, unsigned* offs) {
  const int wu = __builtin_amdgcn_readfirstlane(w);
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    const unsigned c = (unsigned)((k * NWG * 64 + wu * 64) * 16 + lane * 16);
    // only the last copy round can reach past the record end
    offs[k] = (k < NI - 1 || c < (unsigned)BYTES) ? c : (unsigned)BYTES - 16u;
  }
}
template <int BYTES, int STAGE, int NI, int STG, int NWG = 4>
__device__ __forceinline__ void issue_record_at(const char* recs, char* ring, int t, int w,
                                                const unsigned* offs) {
  const char* src = recs + (int64_t)t * BYTES;
  char* dst = ring + (t % STG) * STAGE;
  const int wu = __builtin_amdgcn_readfirstlane(w);
#pragma unroll
  for (int k = 0; k < NI; ++k)
    __builtin_amdgcn_global_load_lds(src + offs[k], LDS_PTR(dst + (k * NWG * 64 + wu * 64) * 16),
                                     16, 0, 0);
}
template <int BYTES, int STAGE, int NI, int STG, int NWG = 4>
__device__ __forceinline__ void issue_record(const char* recs, char* ring, int t, int w,
                                             int lane) {
  const char* src = recs + (int64_t)t * BYTES;
  char* dst = ring + (t % STG) * STAGE;
  const int wu = __builtin_amdgcn_readfirstlane(w);
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    const int off = (k * NWG * 64 + wu * 64) * 16;
    const unsigned c = (unsigned)(off + lane * 16);
    // only the last copy round can reach past the record end
    __builtin_amdgcn_global_load_lds(
        src + ((k < NI - 1 || c < (unsigned)BYTES) ? c : (unsigned)BYTES - 16u),
        LDS_PTR(dst + off), 16, 0, 0);
  }
}

}  // namespace soar
