// Codebook training on gfx950: k-means++ seeding and Lloyd updates (the VQ index the paper
// trains before spilling, Section 3.5; Lloyd's assignment step is the primary assignment of
// Section 2.2).
//
// Lloyd update (segmented centroid reduction).  Rows are grouped by label with a counting sort
// (histogram, exclusive scan, scatter), then one workgroup per cluster sums its rows.  The sums
// are taken in 64-bit fixed point (x * 2^F rounded to an integer, F chosen from max|x| and n so
// that no sum can overflow), which makes them exact and independent of the order the scatter
// produced; the mean is rounded to float once at the end.  An empty cluster keeps its centroid.
//
// k-means++ (HBM-bound, one pass over X per round).  Round m draws w from Philox4x32-10
// (Salmon et al., SC 2011) with counter (m, 0, 0, 0) and key (seed lo, seed hi).  Round 0 takes
// row (w * n) >> 32; later rounds take the smallest row i whose prefix sum of D^2 exceeds
// u * sum(D^2) with u = (w >> 8) * 2^-24 (D = distance to the nearest chosen centre, FP32 direct
// differences).  Prefix sums use fixed-order per-block partials.
#include <cmath>
#include <vector>

#include "../../include/soar.h"
#include "common.h"
#include "kernels.h"
#include "train.h"

namespace soar {

// ---------------------------------------------------------------------------------------------
// Philox4x32-10, from the published round function and key schedule.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t philox_word0(uint32_t ctr0, uint64_t seed) {
  uint32_t c0 = ctr0, c1 = 0u, c2 = 0u, c3 = 0u;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return c0;
}

// ---------------------------------------------------------------------------------------------
// Small utilities
// ---------------------------------------------------------------------------------------------
__global__ void fill_i32_kernel(int32_t* p, int64_t count, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// max |x| over X (float bits of a non-negative float order like unsigned ints)
__global__ __launch_bounds__(256) void maxabs_kernel(const float* __restrict__ X, int64_t count,
                                                     unsigned* out) {
  float m = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = fabsf(X[i]);
    m = (v > m || v != v) ? v : m;   // NaN propagates (its bits exceed every finite value)
  }
  unsigned u = __float_as_uint(m);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) u = max(u, (unsigned)__shfl_xor((int)u, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out, u);
}

// Fixed-order partial sums of v[0..n) per block of SUM_CHUNK elements.
constexpr int SUM_CHUNK = 4096;
__global__ __launch_bounds__(256) void block_sums_kernel(const float* __restrict__ v, int64_t n,
                                                         float* __restrict__ partial) {
  __shared__ float red[256];
  const int64_t base = (int64_t)blockIdx.x * SUM_CHUNK;
  float acc = 0.f;
  for (int k = threadIdx.x; k < SUM_CHUNK; k += 256) {
    const int64_t i = base + k;
    if (i < n) acc += v[i];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------------------------
// Lloyd update
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void label_hist_kernel(const int32_t* __restrict__ labels,
                                                         int64_t n, int K, int32_t* counts,
                                                         unsigned* bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int l = labels[i];
    if (l >= 0 && l < K) atomicAdd(&counts[l], 1);
    else atomicOr(bad, 1u);
  }
}

// Exclusive scan of counts[0..K) into offsets[0..K], and cursor = offsets (one workgroup).
__global__ __launch_bounds__(1024) void scan_counts_kernel(const int32_t* __restrict__ counts,
                                                           int K, int32_t* offsets,
                                                           int32_t* cursor) {
  __shared__ int32_t s[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < K; base += 1024) {
    const int j = base + threadIdx.x;
    const int32_t v = j < K ? counts[j] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // Hillis-Steele inclusive scan
      const int32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    const int32_t excl = carry + s[threadIdx.x] - v;
    if (j < K) { offsets[j] = excl; cursor[j] = excl; }
    __syncthreads();
    if (threadIdx.x == 1023) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) offsets[K] = carry;
}

__global__ __launch_bounds__(256) void scatter_rows_kernel(const int32_t* __restrict__ labels,
                                                           int64_t n, int K, int32_t* cursor,
                                                           int32_t* __restrict__ members) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int l = labels[i];
    if (l >= 0 && l < K) members[atomicAdd(&cursor[l], 1)] = (int32_t)i;
  }
}

// One workgroup per cluster: exact fixed-point sums of its member rows, then the mean.  Threads
// take 4 consecutive dimensions each (float4 loads when the
// rows allow), `slots` member rows are summed side by side and every thread keeps four rows'
// loads in flight; the int64 fixed-point sums make the result independent of that order.
__global__ __launch_bounds__(256) void segment_mean_kernel(
    const float* __restrict__ X, int d, const int32_t* __restrict__ offsets,
    const int32_t* __restrict__ members, const float* C_prev, float* C_out, int32_t* counts_out,
    int fbits, bool vec) {
  __shared__ long long part[256][4];
  const int j = blockIdx.x;
  const int beg = offsets[j], end = offsets[j + 1];
  const int cnt = end - beg;
  const int q4 = (d + 3) / 4;                    // 4-dimension groups per row
  const int tpr = q4 < 256 ? q4 : 256;           // threads per row
  const int slots = 256 / tpr;                   // rows summed side by side
  const int t = threadIdx.x, slot = t / tpr, kk = t % tpr;
  const bool active = slot < slots;
  if (t == 0 && counts_out) counts_out[j] = cnt;
  for (int g0 = 0; g0 < q4; g0 += tpr) {
    const int k = (g0 + kk) * 4;
    long long acc[4] = {0, 0, 0, 0};
    if (active && k < d && cnt > 0) {
      auto add_row = [&](int m) {
        const float* xr = X + (int64_t)members[m] * d + k;
        float v[4];
        if (vec) {
          const v4f t4 = *reinterpret_cast<const v4f*>(xr);
          v[0] = t4.x; v[1] = t4.y; v[2] = t4.z; v[3] = t4.w;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = k + e < d ? xr[e] : 0.f;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] += __float2ll_rn(ldexpf(v[e], fbits));
      };
      int m = beg + slot;
      for (; m + 3 * slots < end; m += 4 * slots) {
        add_row(m); add_row(m + slots); add_row(m + 2 * slots); add_row(m + 3 * slots);
      }
      for (; m < end; m += slots) add_row(m);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) part[t][e] = acc[e];
    __syncthreads();
    if (active && slot == 0 && k < d) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (k + e >= d) break;
        long long s = 0;
        for (int sl = 0; sl < slots; ++sl) s += part[sl * tpr + kk][e];
        const float c = cnt > 0 ? ldexpf(__ll2float_rn(s) / (float)cnt, -fbits)
                                : C_prev[(int64_t)j * d + k + e];
        C_out[(int64_t)j * d + k + e] = c;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// k-means++
// ---------------------------------------------------------------------------------------------
constexpr int KPP_ROWS = 1024;     // rows per block in the D^2 update / prefix search
constexpr int kMaxTrainD = 1024;   // widest rows k-means++ takes (its chosen row sits in LDS)

// D2[i] = min(D2[i], ||x_i - x_c||^2) (or = when first) for the row chosen last, and per-block partial sums of D^2 (fixed order: each
// thread adds its rows grp, grp + 16, ... in turn, then a tree over the block).  A 16-lane group
// takes a row with its lanes across the dimensions (float4 loads when the rows allow) and keeps
// four rows in flight; the chosen row sits in LDS.
__global__ __launch_bounds__(256) void kpp_update_kernel(const float* __restrict__ X, int64_t n,
                                                         int d, const int32_t* cur, bool first,
                                                         float* __restrict__ D2,
                                                         float* __restrict__ partial, bool vec) {
  __shared__ float red[256];
  __shared__ __attribute__((aligned(16))) float sxc[kMaxTrainD];
  const int c = *cur;
  for (int k = threadIdx.x; k < d; k += 256) sxc[k] = X[(int64_t)c * d + k];
  __syncthreads();
  const int lane16 = threadIdx.x & 15, grp = threadIdx.x >> 4;   // 16 row groups per block
  const int64_t base = (int64_t)blockIdx.x * KPP_ROWS;
  auto row_d2 = [&](int64_t i) -> float {
    float a0 = 0.f, a1 = 0.f;
    if (i < n) {
      const float* xi = X + i * d;
      if (vec) {
        for (int k = 4 * lane16; k < d; k += 64) {
          const v4f xv = *reinterpret_cast<const v4f*>(xi + k);
          const v4f cv = *reinterpret_cast<const v4f*>(sxc + k);
          const float e0 = xv.x - cv.x, e1 = xv.y - cv.y, e2 = xv.z - cv.z, e3 = xv.w - cv.w;
          a0 = fmaf(e0, e0, a0); a1 = fmaf(e1, e1, a1);
          a0 = fmaf(e2, e2, a0); a1 = fmaf(e3, e3, a1);
        }
      } else {
        for (int k = lane16; k < d; k += 16) {
          const float e0 = xi[k] - sxc[k];
          a0 = fmaf(e0, e0, a0);
        }
      }
    }
    float s = a0 + a1;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off);
    return s;
  };
  float local = 0.f;
  for (int r0 = grp; r0 < KPP_ROWS; r0 += 64) {
    float sv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) sv[u] = row_d2(base + r0 + 16 * u);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = base + r0 + 16 * u;
      if (i < n && lane16 == 0) {
        const float v = first ? sv[u] : fminf(D2[i], sv[u]);
        D2[i] = v;
        local += v;
      }
    }
  }
  red[threadIdx.x] = local;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Inclusive scan of s[0..1024) in place (one workgroup of 1024 threads, fixed order).
__device__ __forceinline__ void scan1024(float* s, int t) {
  for (int off = 1; off < 1024; off <<= 1) {
    const float u = t >= off ? s[t - off] : 0.f;
    __syncthreads();
    s[t] += u;
    __syncthreads();
  }
}

// Pick round m's row; writes rows_out[m], *cur, chosen[], and C_out[m] = X[row].
// Blocks own [prefix of earlier partials, + own partial); the target is u * (sum of partials).
__global__ __launch_bounds__(1024) void kpp_select_kernel(
    const float* __restrict__ X, int64_t n, int d, const float* __restrict__ D2,
    const float* __restrict__ partial, int nblocks, int m, uint64_t seed, int32_t* cur,
    uint8_t* chosen, float* C_out, int32_t* rows_out) {
  __shared__ float s[1024];
  __shared__ float carry, total;
  __shared__ int pick_block, pick_row, last_pos_block;
  const int t = threadIdx.x;
  const uint32_t w = philox_word0((uint32_t)m, seed);
  if (t == 0) { pick_block = 0x7fffffff; pick_row = 0x7fffffff; last_pos_block = -1; }
  __syncthreads();
  if (m == 0) {
    if (t == 0) pick_row = (int)(((uint64_t)w * (uint64_t)n) >> 32);
  } else {
    // total = prefix of all block partials, scanned in chunks of 1024 in a fixed order
    if (t == 0) total = 0.f;
    __syncthreads();
    for (int base = 0; base < nblocks; base += 1024) {
      const float v = base + t < nblocks ? partial[base + t] : 0.f;
      s[t] = v;
      if (v > 0.f) atomicMax(&last_pos_block, base + t);
      __syncthreads();
      scan1024(s, t);
      if (t == 1023) total += s[1023];
      __syncthreads();
    }
    const float S = total;
    if (S > 0.f) {
      const float target = (float)(w >> 8) * 5.9604644775390625e-08f * S;
      if (t == 0) carry = 0.f;
      __syncthreads();
      for (int base = 0; base < nblocks; base += 1024) {
        const float v = base + t < nblocks ? partial[base + t] : 0.f;
        s[t] = v;
        __syncthreads();
        scan1024(s, t);
        if (v > 0.f && carry + s[t] > target) atomicMin(&pick_block, base + t);
        __syncthreads();
        if (pick_block != 0x7fffffff) break;
        if (t == 1023) carry += s[1023];
        __syncthreads();
      }
      // rounding can put the target past the last prefix: take the last block with weight
      const int b = pick_block != 0x7fffffff ? pick_block : last_pos_block;
      __syncthreads();
      // carry before block b, recomputed in the same chunked order
      if (t == 0) carry = 0.f;
      __syncthreads();
      for (int base = 0; base < b; base += 1024) {
        const float v = base + t < b ? partial[base + t] : 0.f;
        s[t] = v;
        __syncthreads();
        scan1024(s, t);
        if (t == 1023) carry += s[1023];
        __syncthreads();
      }
      const int64_t base_row = (int64_t)b * KPP_ROWS;
      const int64_t i = base_row + t;
      const float v = i < n ? D2[i] : 0.f;
      s[t] = v;
      __syncthreads();
      scan1024(s, t);
      if (v > 0.f && carry + s[t] > target) atomicMin(&pick_row, (int)i);
      __syncthreads();
      if (pick_row == 0x7fffffff) {   // same rounding case inside the block: last row with weight
        if (t == 0) {
          for (int r = KPP_ROWS - 1; r >= 0; --r) {
            const int64_t ii = base_row + r;
            if (ii < n && D2[ii] > 0.f) { pick_row = (int)ii; break; }
          }
        }
      }
    }
    __syncthreads();
    if (pick_row == 0x7fffffff) {
      // sum(D^2) = 0: the lowest-index row not chosen yet
      for (int64_t i = t; i < n; i += 1024)
        if (!chosen[i]) { atomicMin(&pick_row, (int)i); break; }
      __syncthreads();
      if (t == 0 && pick_row == 0x7fffffff) pick_row = -1;
    }
  }
  __syncthreads();
  const int row = pick_row;
  if (t == 0) {
    *cur = row < 0 ? 0 : row;
    rows_out[m] = row;
    if (row >= 0) chosen[row] = 1;
  }
  if (row >= 0)
    for (int k = t; k < d; k += 1024) C_out[(int64_t)m * d + k] = X[(int64_t)row * d + k];
}

// ---------------------------------------------------------------------------------------------
// Workspace layout of the training calls
// ---------------------------------------------------------------------------------------------
namespace {
constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

struct TrainLayout {
  void* assign_ws;      // workspace of the primary-assignment pass
  int32_t* labels;      // [n]
  float* dist;          // [n] (also D^2 of k-means++)
  int32_t* counts;      // [K]
  int32_t* offsets;     // [K + 1]
  int32_t* cursor;      // [K]
  int32_t* members;     // [n]
  float* partial;       // [n / SUM_CHUNK + n / KPP_ROWS + 2]
  unsigned* flags;      // [8]: 0 max|x| bits, 1 bad label
  int32_t* cur;         // [1]
  uint8_t* chosen;      // [n]
  int32_t* rows;        // [K]
  float* Ctmp;          // [K x d]
  size_t bytes;
};

TrainLayout layout_train(void* ws, int64_t n, int d, int K) {
  char* b = static_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? b + off : nullptr;
    off = al(off + bytes);
    return p;
  };
  TrainLayout L;
  const size_t aws = assign_workspace_bytes(n, d, K);
  L.assign_ws = take(aws);
  L.labels = (int32_t*)take(n * 4);
  L.dist = (float*)take(n * 4);
  L.counts = (int32_t*)take((size_t)K * 4);
  L.offsets = (int32_t*)take((size_t)(K + 1) * 4);
  L.cursor = (int32_t*)take((size_t)K * 4);
  L.members = (int32_t*)take(n * 4);
  L.partial = (float*)take((size_t)(n / SUM_CHUNK + n / KPP_ROWS + 4) * 4);
  L.flags = (unsigned*)take(8 * 4);
  L.cur = (int32_t*)take(4);
  L.chosen = (uint8_t*)take(n);
  L.rows = (int32_t*)take((size_t)K * 4);
  L.Ctmp = (float*)take((size_t)K * d * 4);
  L.bytes = off;
  return L;
}

inline unsigned grid_for(int64_t work, int per_block, unsigned cap = 65535u) {
  const int64_t g = (work + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

// F such that sum of n values of magnitude <= maxabs, times 2^F, stays below 2^62.
int fixed_point_bits(float maxabs, int64_t n) {
  if (!(maxabs > 0.f)) return 40;
  const int e = (int)std::ceil(std::log2((double)maxabs));
  const int en = (int)std::ceil(std::log2((double)(n > 1 ? n : 2)));
  int f = 61 - e - en;
  if (f > 100) f = 100;
  return f;
}
}  // namespace

static soar_status lloyd_update_impl(const float* X, int64_t n, int d, const int32_t* labels,
                                     int K, const float* C_prev, float* C_out, int32_t* counts,
                                     const TrainLayout& L, int fbits, hipStream_t st) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(K, 256)), dim3(256), 0, st, L.counts,
                     (int64_t)K, 0);
  hipLaunchKernelGGL(label_hist_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, labels,
                     n, K, L.counts, L.flags + 1);
  hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(1024), 0, st, L.counts, K, L.offsets,
                     L.cursor);
  hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, labels,
                     n, K, L.cursor, L.members);
  const bool vec = d % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0;
  hipLaunchKernelGGL(segment_mean_kernel, dim3((unsigned)K), dim3(256), 0, st, X, d, L.offsets,
                     L.members, C_prev, C_out, counts, fbits, vec);
  return hipGetLastError() == hipSuccess ? SOAR_OK : SOAR_E_DEVICE;
}

static soar_status maxabs_bits(const float* X, int64_t n, int d, const TrainLayout& L,
                               hipStream_t st, int* fbits, bool* nonfinite) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, st, (int32_t*)L.flags, (int64_t)8, 0);
  hipLaunchKernelGGL(maxabs_kernel, dim3(grid_for(n * d, 256, 2048)), dim3(256), 0, st, X,
                     n * (int64_t)d, L.flags);
  unsigned bits = 0;
  if (hipMemcpyAsync(&bits, L.flags, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SOAR_E_DEVICE;
  const float m = __builtin_bit_cast(float, bits);
  *nonfinite = !std::isfinite(m);
  *fbits = fixed_point_bits(m, n);
  return SOAR_OK;
}

static soar_status kmeanspp_impl(const float* X, int64_t n, int d, int K, uint64_t seed,
                                 float* C_out, int32_t* rows_out, const TrainLayout& L,
                                 hipStream_t st) {
  const int nblocks = (int)((n + KPP_ROWS - 1) / KPP_ROWS);
  const bool vec = d % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0;
  float* partial = L.partial;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n, 1024, 4096)), dim3(256), 0, st,
                     (int32_t*)L.chosen, (int64_t)((n + 3) / 4), 0);
  int32_t* rows = rows_out ? rows_out : L.rows;
  for (int m = 0; m < K; ++m) {
    if (m > 0)
      hipLaunchKernelGGL(kpp_update_kernel, dim3((unsigned)nblocks), dim3(256), 0, st, X, n, d,
                         L.cur, m == 1, L.dist, partial, vec);
    hipLaunchKernelGGL(kpp_select_kernel, dim3(1), dim3(1024), 0, st, X, n, d, L.dist, partial,
                       nblocks, m, seed, L.cur, L.chosen, C_out, rows);
  }
  return hipGetLastError() == hipSuccess ? SOAR_OK : SOAR_E_DEVICE;
}

static soar_status reduce_sum_host(const float* v, int64_t n, const TrainLayout& L, hipStream_t st,
                                   double* out) {
  const int nb = (int)((n + SUM_CHUNK - 1) / SUM_CHUNK);
  hipLaunchKernelGGL(block_sums_kernel, dim3((unsigned)nb), dim3(256), 0, st, v, n, L.partial);
  std::vector<float> h(nb);
  if (hipMemcpyAsync(h.data(), L.partial, nb * sizeof(float), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SOAR_E_DEVICE;
  double s = 0.0;
  for (float x : h) s += x;
  *out = s;
  return SOAR_OK;
}

size_t train_workspace_bytes(int64_t n, int d, int K) { return layout_train(nullptr, n, d, K).bytes; }

}  // namespace soar

using namespace soar;

namespace {
soar_status check_train_args(const float* X, int64_t n, int32_t d, int32_t K, void* ws,
                             size_t ws_bytes, bool k_may_exceed_n) {
  if (!X || !ws || n < 1 || n > INT32_MAX || d < 1 || K < 1) return SOAR_E_INVAL;
  if (K > n && !k_may_exceed_n) return SOAR_E_INVAL;
  if ((reinterpret_cast<uintptr_t>(X) % 4) != 0 || (reinterpret_cast<uintptr_t>(ws) % 256) != 0)
    return SOAR_E_INVAL;
  if (ws_bytes < train_workspace_bytes(n, d, K)) return SOAR_E_INVAL;
  return SOAR_OK;
}
}  // namespace

extern "C" {

soar_status soar_train_workspace_size(int64_t n, int32_t d, int32_t K, size_t* bytes) {
  if (!bytes || n < 1 || n > INT32_MAX || d < 1 || K < 1) return SOAR_E_INVAL;
  *bytes = train_workspace_bytes(n, d, K);
  return SOAR_OK;
}

soar_status soar_kmeanspp(const float* X, int64_t n, int32_t d, int32_t K, uint64_t seed,
                          float* C_out, int32_t* rows_out, void* workspace, size_t ws_bytes,
                          void* stream) {
  soar_status s = check_train_args(X, n, d, K, workspace, ws_bytes, false);
  if (s != SOAR_OK) return s;
  if (!C_out) return SOAR_E_INVAL;
  if (d > kMaxTrainD) return SOAR_E_UNSUPPORTED;   // the chosen row is staged in LDS
  hipStream_t st = static_cast<hipStream_t>(stream);
  TrainLayout L = layout_train(workspace, n, d, K);
  int fb;
  bool nonfinite;
  s = maxabs_bits(X, n, d, L, st, &fb, &nonfinite);
  if (s != SOAR_OK) return s;
  if (nonfinite) return SOAR_E_NONFINITE;
  s = kmeanspp_impl(X, n, d, K, seed, C_out, rows_out, L, st);
  if (s != SOAR_OK) return s;
  return hipStreamSynchronize(st) == hipSuccess ? SOAR_OK : SOAR_E_DEVICE;
}

soar_status soar_lloyd_update(const float* X, int64_t n, int32_t d, const int32_t* labels,
                              int32_t K, const float* C_prev, float* C_out, int32_t* counts,
                              void* workspace, size_t ws_bytes, void* stream) {
  soar_status s = check_train_args(X, n, d, K, workspace, ws_bytes, true);
  if (s != SOAR_OK) return s;
  if (!labels || !C_prev || !C_out) return SOAR_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  TrainLayout L = layout_train(workspace, n, d, K);
  int fb;
  bool nonfinite;
  s = maxabs_bits(X, n, d, L, st, &fb, &nonfinite);
  if (s != SOAR_OK) return s;
  if (nonfinite) return SOAR_E_NONFINITE;
  s = lloyd_update_impl(X, n, d, labels, K, C_prev, C_out, counts, L, fb, st);
  if (s != SOAR_OK) return s;
  unsigned bad = 0;
  if (hipMemcpyAsync(&bad, L.flags + 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SOAR_E_DEVICE;
  return bad ? SOAR_E_INVAL : SOAR_OK;
}

soar_status soar_train_codebook(const float* X, int64_t n, int32_t d, int32_t K, int32_t iters,
                                uint64_t seed, const float* C_init, float* C_out, int32_t* labels,
                                double* inertia, void* workspace, size_t ws_bytes, void* stream) {
  soar_status s = check_train_args(X, n, d, K, workspace, ws_bytes, false);
  if (s != SOAR_OK) return s;
  if (!C_out || iters < 0 || fp32_padded_dim(d) < 0) return d > 1024 ? SOAR_E_UNSUPPORTED
                                                                    : SOAR_E_INVAL;
  if (K < 2 && iters > 0) return SOAR_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  TrainLayout L = layout_train(workspace, n, d, K);
  int fb;
  bool nonfinite;
  s = maxabs_bits(X, n, d, L, st, &fb, &nonfinite);
  if (s != SOAR_OK) return s;
  if (nonfinite) return SOAR_E_NONFINITE;
  if (C_init) {
    if (hipMemcpyAsync(C_out, C_init, (size_t)K * d * 4, hipMemcpyDeviceToDevice, st) !=
        hipSuccess)
      return SOAR_E_DEVICE;
  } else {
    s = kmeanspp_impl(X, n, d, K, seed, C_out, nullptr, L, st);
    if (s != SOAR_OK) return s;
  }
  int32_t* lab = labels ? labels : L.labels;
  unsigned cnt[CNT_WORDS];
  for (int t = 0; t <= iters; ++t) {
    s = run_assign_fp32(X, n, d, C_out, K, 0.f, 0.f, false, lab, nullptr, L.dist, nullptr,
                        L.assign_ws, st, cnt);
    if (s != SOAR_OK) return s;
    if (inertia) {
      s = reduce_sum_host(L.dist, n, L, st, &inertia[t]);
      if (s != SOAR_OK) return s;
    }
    if (t == iters) break;
    s = lloyd_update_impl(X, n, d, lab, K, C_out, C_out, nullptr, L, fb, st);
    if (s != SOAR_OK) return s;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return SOAR_E_DEVICE;
  return cnt[CNT_NONFINITE] ? SOAR_E_NONFINITE : SOAR_OK;
}

}  // extern "C"
