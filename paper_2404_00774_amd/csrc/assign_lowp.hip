// Low-precision SOAR assignment on gfx950: the two contractions X C^T and R C^T in BF16
// (v_mfma_f32_16x16x32_bf16) or OCP FP8-e4m3 (v_mfma_scale_f32_16x16x128_f8f6f4, unit block
// scales) with FP32 accumulation, followed by an FP32 re-score of a few candidates per row by
// direct differences and an FP64 decision among near-ties.  Same loss as the FP32 path:
//     primary  argmin_j ||x - c_j||^2                               (Section 2.2)
//     spill    argmin_{j != pi} ||x - c_j||^2 + lambda <r, x - c_j>^2 / ||r||^2
//                                                                  (Section 3.4, Theorem 3.1)
//
// Pipeline (all on the caller's stream):
//   quantize  X -> Xq, C -> Cq (rows padded to DP elements with zeros; FP8 rows carry a
//             power-of-two scale so that max|row| * scale lies in [128, 256))
//   sweep     primary: ranking value ||c||^2 - 2<x,c>; candidates per row -> cand
//   rescore   exact FP32 over the candidates, FP64 among near-ties -> pi, ||x - c_pi||^2;
//             residual r = x - c_pi in FP32, quantized -> Rq, and the row constants
//   sweep     spill: ||c||^2 - 2<x,c> + lambda/||r||^2 (<r,c> - <r,x>)^2, pi masked -> cand
//   rescore   exact FP32 SOAR loss over the candidates, FP64 among near-ties -> pi', loss
//
// Candidates.  In the 16x16 MFMA result a lane sees one column of every 16-column block, so per
// row the 16 lanes of a lane group see the 16 residues j mod 16.  Each lane splits its columns
// once more by the parity of the block within the tile, so a row's columns fall into 32 classes
// (16 lanes x 2), and a lane keeps, per row and class, the smallest ranking value (BF16) or the
// two smallest (FP8, whose coarser rounding moves the true best further down the approximate
// order).  The global 16-column block index j / 16 is packed into the low mantissa bits of the
// value (12 bits up to K = 65,536: a relative perturbation below 2^-11, against the 2^-8 of a
// BF16 operand; with the mask held in a register, packing is one v_and_or), so a kept value
// carries its column.  The topk (<= 16) smallest kept values of a row, ranked across its 16
// lanes, are re-scored.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace soar {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr float kBig = 3.0e38f;       // finite sentinel: never a candidate, survives the packing
constexpr int kMaxTopk = 16;          // candidates re-scored per row

template <int FMT>
struct FmtTraits;
template <>
struct FmtTraits<LOWP_BF16> {
  static constexpr int BYTES = 2;    // bytes per element
  static constexpr int KSTEP = 32;   // contraction length of one MFMA
  static constexpr int LANE_B = 16;  // bytes one lane supplies per MFMA
};
template <>
struct FmtTraits<LOWP_FP8> {
  static constexpr int BYTES = 1;
  static constexpr int KSTEP = 128;
  static constexpr int LANE_B = 32;
};

// Rotations within a DPP row (16 lanes: 16k .. 16k + 15) by N lanes, on the VALU.
template <int N>
__device__ __forceinline__ int row_ror(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x120 + N, 0xf, 0xf, false);
}
template <int N>
__device__ __forceinline__ float row_ror(float v) {
  return __builtin_bit_cast(float, row_ror<N>(__builtin_bit_cast(int, v)));
}
template <int N>
__device__ __forceinline__ double row_ror(double v) {
  const auto w = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, int2{row_ror<N>(w.x), row_ror<N>(w.y)});
}
#ifndef SOAR_CAND_BF16
#define SOAR_CAND_BF16 1
#endif
#ifndef SOAR_CAND_FP8
#define SOAR_CAND_FP8 2
#endif

// The low cbits mantissa bits carry the global block index j / 16 (cbits: enough bits for every
// block of the codebook).  The mask sits in a VGPR (the block code takes the one scalar operand
// a VALU instruction may read), so packing stays one v_and_or.
__device__ __forceinline__ int code_bits(int K) {
  const unsigned nblk = (unsigned)(K + 15) >> 4;
  return nblk <= 2u ? 1 : 32 - __builtin_clz(nblk - 1u);
}
__device__ __forceinline__ unsigned code_mask(int cbits) {
  const unsigned m = ~((1u << cbits) - 1u);
  unsigned v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(m));
  return v;
}
__device__ __forceinline__ float pack_code(float v, unsigned mask, unsigned c) {
  return __builtin_bit_cast(float, (__builtin_bit_cast(unsigned, v) & mask) | c);
}

// ------------------------------------------------------------------------------------------------
// Quantization of rows (X or C): FP32 -> padded BF16 / FP8 rows, plus per-row inverse scales.
// One 16-lane group per row.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned char fp8_of(float v) {
  v = fminf(fmaxf(v, -448.f), 448.f);
  return (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0u, false) & 0xFFu);
}

template <int FMT, bool V4 = false>
__global__ __launch_bounds__(256) void quantize_rows_kernel(const float* __restrict__ A,
                                                            int64_t rows, int d, int dp,
                                                            float mult, void* __restrict__ out,
                                                            float* __restrict__ inv_scale,
                                                            unsigned* counters,
                                                            const int64_t* live_n) {
  const int l16 = threadIdx.x & 15;
  const int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  if (row >= live_rows(rows, live_n)) return;
  const float* a = A + row * d;
  float scale = 1.f;
  bool fin = true;
  if constexpr (FMT == LOWP_FP8 && V4) {
    // rows of whole float4 chunks: 16-byte loads, 4 codes per 4-byte store (the same scale and
    // codes as the scalar form below; the second pass reads the row again from cache)
    float m = 0.f;
    for (int k = 4 * l16; k < d; k += 64) {
      const v4f v = *reinterpret_cast<const v4f*>(a + k);
      fin = fin && all_finite4(v);
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (m > 0.f && is_finite_bits(m)) {
      int e;
      (void)frexpf(m, &e);
      scale = ldexpf(1.f, 8 - e);
    }
    unsigned* o = reinterpret_cast<unsigned*>(static_cast<unsigned char*>(out) + row * dp);
    for (int k = 4 * l16; k < dp; k += 64) {
      v4f v = {0.f, 0.f, 0.f, 0.f};
      if (k < d) v = *reinterpret_cast<const v4f*>(a + k);
      o[k / 4] = (unsigned)fp8_of(v.x * scale) | ((unsigned)fp8_of(v.y * scale) << 8) |
                 ((unsigned)fp8_of(v.z * scale) << 16) | ((unsigned)fp8_of(v.w * scale) << 24);
    }
    if (l16 == 0) inv_scale[row] = 1.f / scale;
  } else if constexpr (FMT == LOWP_FP8) {
    float m = 0.f;
    for (int k = l16; k < d; k += 16) {
      const float v = a[k];
      fin = fin && is_finite_bits(v);
      m = fmaxf(m, fabsf(v));
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (m > 0.f && is_finite_bits(m)) {
      int e;
      (void)frexpf(m, &e);              // m = f * 2^e with f in [0.5, 1)
      scale = ldexpf(1.f, 8 - e);        // m * scale in [128, 256)
    }
    unsigned char* o = static_cast<unsigned char*>(out) + row * dp;
    for (int k = l16; k < dp; k += 16) o[k] = k < d ? fp8_of(a[k] * scale) : (unsigned char)0;
    if (l16 == 0) inv_scale[row] = 1.f / scale;
  } else if constexpr (V4) {
    // rows of whole float4 chunks: 16-byte loads, 8-byte stores
    __bf16* o = static_cast<__bf16*>(out) + row * dp;
    for (int k = 4 * l16; k < dp; k += 64) {
      v4f v = {0.f, 0.f, 0.f, 0.f};
      if (k < d) v = *reinterpret_cast<const v4f*>(a + k);
      fin = fin && all_finite4(v);
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      const bf16x4 b = {(__bf16)(v.x * mult), (__bf16)(v.y * mult), (__bf16)(v.z * mult),
                        (__bf16)(v.w * mult)};
      *reinterpret_cast<bf16x4*>(o + k) = b;
    }
    if (inv_scale && l16 == 0) inv_scale[row] = 1.f;
  } else {
    __bf16* o = static_cast<__bf16*>(out) + row * dp;
    for (int k = l16; k < dp; k += 16) {
      const float v = k < d ? a[k] : 0.f;
      fin = fin && is_finite_bits(v);
      o[k] = (__bf16)(v * mult);   // mult is a power of two: exact
    }
    if (inv_scale && l16 == 0) inv_scale[row] = 1.f;
  }
  if (!fin) atomicOr(&counters[CNT_NONFINITE], 1u);
}

// ------------------------------------------------------------------------------------------------
// The sweep: one workgroup = 4 waves x SPW stripes x 16 rows; C streamed through LDS tiles.
// ------------------------------------------------------------------------------------------------
template <int FMT, int DP>
struct OperandRegs {
  static constexpr int NSTEP = DP / FmtTraits<FMT>::KSTEP;
  static constexpr int W4 = FmtTraits<FMT>::LANE_B / 16;   // u32x4 per lane per step
  u32x4 v[NSTEP][W4];
};

template <int FMT, int DP>
__device__ __forceinline__ void load_operand(const void* __restrict__ base, int64_t row,
                                             bool ok, int q, OperandRegs<FMT, DP>& r) {
  using T = FmtTraits<FMT>;
  constexpr int NSTEP = OperandRegs<FMT, DP>::NSTEP, W4 = OperandRegs<FMT, DP>::W4;
  const char* p = static_cast<const char*>(base) + (row * DP + q * (DP / 4)) * T::BYTES;
#pragma unroll
  for (int s = 0; s < NSTEP; ++s)
#pragma unroll
    for (int w = 0; w < W4; ++w)
      r.v[s][w] = ok ? *reinterpret_cast<const u32x4*>(p + s * T::LANE_B + w * 16)
                     : u32x4{0u, 0u, 0u, 0u};
}

// FP8: sa and sb are E8M0 block scales (the factor 2^(s - 127)) of the lane's A row and B column.
// Lane (q, c) supplies the scales of row c and of column c for contraction block q; every block
// of a row (column) carries the same one, so the MFMA applies the per-row and per-column
// power-of-two scales of the quantized operands itself.
template <int FMT>
__device__ __forceinline__ v4f mfma_step(const u32x4* a, const u32x4* b, v4f acc, int sa, int sb) {
  if constexpr (FMT == LOWP_BF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[0]),
                                                   __builtin_bit_cast(bf16x8, b[0]), acc, 0, 0, 0);
  } else {
    const i32x8 av = {(int)a[0].x, (int)a[0].y, (int)a[0].z, (int)a[0].w,
                      (int)a[1].x, (int)a[1].y, (int)a[1].z, (int)a[1].w};
    const i32x8 bv = {(int)b[0].x, (int)b[0].y, (int)b[0].z, (int)b[0].w,
                      (int)b[1].x, (int)b[1].y, (int)b[1].z, (int)b[1].w};
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc, 0, 0, 0, sa, 0, sb);
  }
}

// E8M0 code of a power of two: its biased exponent field.
__device__ __forceinline__ int e8m0_of(float pow2) {
  return (int)((__builtin_bit_cast(unsigned, pow2) >> 23) & 0xffu);
}

// ------------------------------------------------------------------------------------------------
// Packed codebook: the sweep streams the codebook in tiles of BN centroids, and each tile is one
// contiguous record in HBM so that the waves can copy it to LDS with direct global->LDS loads:
//   [BN quantized rows, row stride DP*BYTES + 16 (padding keeps the B reads conflict-free)]
//   [BN x float4: ||c_j||^2 four times (a finite 3e38 beyond K)]
//   [BN x 4 bytes: FP8: E8M0 block scale of the row, 2 / its quantization scale; BF16: 1.f]
// Rows beyond K are zero.  A record is read with NI whole 4 KiB wave-group copies.
// ------------------------------------------------------------------------------------------------
template <int FMT, int DP, int BN>
struct TileRec {
  static constexpr int ROWB = DP * FmtTraits<FMT>::BYTES;
  static constexpr int LDWB = ROWB + 16;
  static constexpr int CN_OFF = BN * LDWB;
  static constexpr int CS_OFF = CN_OFF + BN * 16;
  static constexpr int BYTES = CS_OFF + BN * 4;
  static constexpr int NI = (BYTES + 4095) / 4096;     // copies per wave (4 waves x 64 lanes x 16 B)
  static constexpr int STAGE = NI * 4096;              // LDS bytes per ring stage
};

template <int FMT, int DP, int BN>
__global__ __launch_bounds__(256) void pack_codebook_kernel(const float* __restrict__ C, int K,
                                                            int d, const float* __restrict__ cnorm,
                                                            char* __restrict__ rec,
                                                            unsigned* counters) {
  using R = TileRec<FMT, DP, BN>;
  const int l16 = threadIdx.x & 15;
  const int j = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int t = j / BN, jl = j % BN;
  char* base = rec + (int64_t)t * R::BYTES;
  const bool ok = j < K;
  const float* c = C + (int64_t)(ok ? j : 0) * d;
  float scale = 1.f;
  bool fin = true;
  if constexpr (FMT == LOWP_FP8) {
    float m = 0.f;
    if (ok)
      for (int k = l16; k < d; k += 16) {
        fin = fin && is_finite_bits(c[k]);
        m = fmaxf(m, fabsf(c[k]));
      }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (m > 0.f && is_finite_bits(m)) {
      int e;
      (void)frexpf(m, &e);
      scale = ldexpf(1.f, 8 - e);
    }
    // -c (a sign flip, exact); the column's block scale carries 2 / scale, so the MFMA
    // accumulates -2 <x, c> onto ||c||^2 as in BF16
    unsigned char* o = reinterpret_cast<unsigned char*>(base + jl * R::LDWB);
    for (int k = l16; k < R::LDWB; k += 16)
      o[k] = (ok && k < d) ? fp8_of(-c[k] * scale) : (unsigned char)0;
  } else {
    __bf16* o = reinterpret_cast<__bf16*>(base + jl * R::LDWB);
    for (int k = l16; k < R::LDWB / 2; k += 16) {
      const float v = (ok && k < d) ? c[k] : 0.f;
      fin = fin && is_finite_bits(v);
      o[k] = (__bf16)(-2.f * v);   // exact: the accumulator then holds ||c||^2 - 2 <x, c>
    }
  }
  if (l16 == 0) {
    const float cn = ok ? cnorm[j] : kBig;
    *reinterpret_cast<v4f*>(base + R::CN_OFF + jl * 16) = v4f{cn, cn, cn, cn};
    if constexpr (FMT == LOWP_FP8)
      *reinterpret_cast<int*>(base + R::CS_OFF + jl * 4) = e8m0_of(2.f / scale);
    else
      *reinterpret_cast<float*>(base + R::CS_OFF + jl * 4) = 1.f;
  }
  if (!fin) atomicOr(&counters[CNT_NONFINITE], 1u);
}

// Ranking values in the epilogue (row constants of the loss dropped): the record holds -2 c
// (BF16: exact; FP8: -c with the factor 2 in the column's block scale, and every FP8 row's
// power-of-two scale applied by the MFMA) and the residual rows are stored pre-scaled by
// sigma = sqrt(lambda) / (2 ||r||); the S accumulator starts at ||c_j||^2 and the T
// accumulator at 2 sigma <r_i, x_i>, so S = ||c||^2 - 2<x,c>, T = -2 sigma (<r,c> - <r,x>) and
// the spill value is S + T^2 (one fma).  Both formats share this epilogue.
// The codebook records flow through an LDS ring of STG stages filled STG-1 tiles ahead.
// GPD (grouped spill form): each 16-row stripe holds up to 15 rows sharing the primary p and, as
// row 15, c_p quantized like the rows; with S the rescaled ||c||^2 - 2<., c> of a row,
// <r_i, c_j> - <r_i, x_i> = (S_pj - S_ij) / 2 - <r_i, x_i>, so one MFMA stream serves the spill:
// T = sigma (S_pj - S_ij) - 2 sigma <r_i, x_i> and the value is S_ij + T^2.
// GR (grouped form over residual rows, BF16, lambda > 0): the stripe rows are the pre-scaled
// residuals sigma r_i instead of x_i, and row 15 is c_p with ||c_j||^2 added after the MFMA, so
// row 15 gives D_j = ||c_j||^2 - 2<c_p, c_j>.  With m = -2 sigma <r, c_j> from the MFMA,
// ||x - c_j||^2 = ||x||^2 + D_j + m / sigma and lambda <r, x - c_j>^2 / ||r||^2 =
// (m + 2 sigma <r, x>)^2; completing the square in m leaves, up to row constants,
// D_j + z^2 with z = m + 2 sigma <r, x> + 1 / (2 sigma): the accumulator starts at the row
// constant beta = 2 sigma <r, x> + 1 / (2 sigma), and the value is one fma, as in the direct
// form, from one MFMA stream.  The dropped row constant 1 / (4 sigma^2) = ||r||^2 / lambda stays
// within a few powers of two of the loss for lambda >= kGroupedResidualMinLam.
// Waves per workgroup of the sweep: WPE workgroups of 4 waves share a CU.  (One workgroup of
// 4 WPE waves per CU, which copies each record once instead of WPE times, measured no faster at
// BF16 and slower at FP8: its waves meet at every barrier together.)
constexpr int lowp_wg_waves(int) { return 4; }

template <int FMT, int DP, int SPW, int BN, int STG, int WPE, bool SP, bool GPD = false,
          bool GR = false, bool KS = false>
__global__ __launch_bounds__(64 * lowp_wg_waves(WPE))
__attribute__((amdgpu_waves_per_eu(WPE, WPE > 2 ? WPE : 2)))
void lowp_sweep_kernel(LowpParams P) {
  using T = FmtTraits<FMT>;
  using R = TileRec<FMT, DP, BN>;
  constexpr bool BF = FMT == LOWP_BF16;
  constexpr int NB = BN / 16;                      // 16-column blocks per tile
  static_assert(NB <= 8 && (NB == 1 || NB % 2 == 0), "tile of 1, 2, 4 or 8 blocks");
  constexpr int NSTEP = OperandRegs<FMT, DP>::NSTEP, W4 = OperandRegs<FMT, DP>::W4;
  constexpr int NR = SPW * 4;                      // rows per lane in the output layout
  constexpr int NW = lowp_wg_waves(WPE);            // waves of the workgroup
  constexpr int NI = (R::BYTES + NW * 1024 - 1) / (NW * 1024);   // record copies per wave
  constexpr int STAGE = NI * NW * 1024;            // LDS bytes per ring stage
  __shared__ __attribute__((aligned(16))) char s_ring[STG * STAGE];

  static_assert(!GPD || SP, "the grouped form is a spill sweep");
  static_assert(!GR || GPD, "residual rows: a grouped form");
  static_assert(!(KS && GPD), "codebook splits: direct sweeps only");
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, q = lane >> 4, c16 = lane & 15;
  const int64_t n = live_rows(P.n, P.live_n);
  // GPD: stripes (blockIdx.x * NW + w) * SPW + st; each is {p, first in perm, rows}
  const int ns = GPD ? *P.nstripes : 0;
  if (GPD ? (int64_t)blockIdx.x * NW * SPW >= ns : (int64_t)blockIdx.x * 16 * NW * SPW >= n)
    return;
  const int64_t row0 = ((int64_t)blockIdx.x * NW + w) * (16 * SPW);
  // KS: codebook split blockIdx.y of gridDim.y (at most one split per tile): tiles
  // [t0, t0 + ntiles).  (A separate instantiation: the split bookkeeping costs registers.)
  const int ntiles_all = (P.K + BN - 1) / BN;
  const int t0 = KS ? (int)((int64_t)ntiles_all * blockIdx.y / gridDim.y) : 0;
  const int ntiles =
      KS ? (int)((int64_t)ntiles_all * (blockIdx.y + 1) / gridDim.y) - t0 : ntiles_all;
  const int kbase = t0 * BN;                       // first column of the split
  const char* recs = static_cast<const char*>(P.Cq) + (size_t)t0 * R::BYTES;
  int4 sd[GPD ? SPW : 1];
  if constexpr (GPD) {
#pragma unroll
    for (int st = 0; st < SPW; ++st) {
      const int sidx = (blockIdx.x * NW + w) * SPW + st;
      sd[st] = sidx < ns ? P.stripes[sidx] : int4{0, 0, 0, 0};
    }
  }
  // row id of stripe-row lr of stripe st (-1: no data row there)
  auto row_of = [&](int st, int lr) -> int64_t {
    if constexpr (GPD) return lr < sd[st].z ? (int64_t)P.perm[sd[st].y + lr] : -1;
    else { const int64_t r = row0 + st * 16 + lr; return r < n ? r : -1; }
  };

  // copies of record t into its ring stage; short records keep their per-lane source offsets in
  // registers, long ones (many copies per wave) recompute them
  constexpr bool KEEP_OFF = NI <= 4;
  unsigned roff[KEEP_OFF ? NI : 1];
  if constexpr (KEEP_OFF) record_offsets<R::BYTES, NI, NW>(w, lane, roff);
  auto issue = [&](int t) __attribute__((always_inline)) {
    if constexpr (KEEP_OFF)
      issue_record_at<R::BYTES, STAGE, NI, STG, NW>(recs, s_ring, t, w, roff);
    else
      issue_record<R::BYTES, STAGE, NI, STG, NW>(recs, s_ring, t, w, lane);
  };
  // prologue: records 0 .. STG - 2 in flight
#pragma unroll
  for (int k = 0; k < STG - 1; ++k)
    if (k < ntiles) issue(k);

  // A operands (A layout: lane (q, c16) holds row c16 of each stripe, quarter q of the dims)
  OperandRegs<FMT, DP> xa[SPW];
  OperandRegs<FMT, DP> ra[SP && !GPD ? SPW : 1];
  // FP8: E8M0 scales of the lane's A rows (row c16 of each stripe) for xa and ra
  int xsc[SPW], rsc[SP && !GPD ? SPW : 1];
#pragma unroll
  for (int st = 0; st < SPW; ++st) {
    const int64_t r = row_of(st, c16);
    const bool ok = r >= 0;
    if (GPD && c16 == 15) load_operand<FMT, DP>(P.Cp, sd[st].x, true, q, xa[st]);   // c_p
    else load_operand<FMT, DP>(GR ? P.Rq : P.Xq, r, ok, q, xa[st]);
    if constexpr (SP && !GPD) load_operand<FMT, DP>(P.Rq, r, ok, q, ra[st]);
    if constexpr (BF) {
      xsc[st] = 127;
      if constexpr (SP && !GPD) rsc[st] = 127;
    } else {
      // inverse row scales: x (xs), the centroid row (cps), residual rows (rowc.x)
      if (GPD && c16 == 15) xsc[st] = e8m0_of(P.cps[sd[st].x]);
      else xsc[st] = ok ? e8m0_of(GR ? P.rowc[r].x : P.xs[r]) : 127;
      if constexpr (SP && !GPD) rsc[st] = ok ? e8m0_of(P.rowc[r].x) : 127;
    }
  }
  // row constants in the output layout: row (st, 4q + v)
  constexpr int NRS = SP ? NR : 1;                 // spill-only row constants
  float gs[GPD && !GR ? NR : 1], gm[GPD && !GR ? NR : 1];   // GPD: sigma, -2 sigma <r, x>
  int kp[NRS];
  v4f a2[SP ? SPW : 1];
#pragma unroll
  for (int st = 0; st < SPW; ++st)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = st * 4 + v;
      const int64_t r = row_of(st, 4 * q + v);
      const bool ok = r >= 0;
      if constexpr (GPD) {
        const float4 rc = ok ? P.rowc[r] : float4{0.f, 0.f, 0.f, 0.f};
        if constexpr (GR) {
          // beta; zero for rows without a residual term (their operand row is zero too, so
          // their value is D_j, the distance ranking), for empty rows and for row 15
          a2[st][v] = rc.w > 0.f ? fmaf(2.f * rc.w, rc.y, 0.5f / rc.w) : 0.f;
        } else {
          gs[i] = rc.w;
          gm[i] = -2.f * rc.w * rc.y;
        }
        kp[i] = sd[st].x;
      } else if constexpr (SP) {
        const float4 rc = ok ? P.rowc[r] : float4{0.f, 0.f, 0.f, 0.f};
        kp[i] = ok ? P.primary[r] : -1;
        a2[st][v] = 2.f * rc.w * rc.y;       // 2 sigma <r, x>
      }
    }
  // primaries relative to the split (a row without one stays negative and matches no column)
  if constexpr (KS) {
#pragma unroll
    for (int i = 0; i < NRS; ++i) kp[i] -= kbase;
  }
  // kept values per row: NCLS classes (block parity) x CAND smallest, packed with their block
  constexpr int NCLS = NB >= 2 ? 2 : 1;
  constexpr int CAND = BF ? SOAR_CAND_BF16 : SOAR_CAND_FP8;
  static_assert(CAND == 1 || CAND == 2, "one or two kept values per class");
  constexpr int NS = NCLS * CAND;
  const int cbits = code_bits(P.K);
  const unsigned cmask = code_mask(cbits);
  float kept[NR][NS];
#pragma unroll
  for (int i = 0; i < NR; ++i)
#pragma unroll
    for (int k = 0; k < NS; ++k) kept[i][k] = kBig;
  // lane's base addresses inside a ring stage: B operand rows and the norms
  const int lane_b = c16 * R::LDWB + (q * (DP / 4)) * T::BYTES;
  const int lane_cn = R::CN_OFF + c16 * 16;

  // Software pipeline over units of GU blocks (two units per tile, or one tile per unit when the
  // tile has a single block).  The MFMAs of unit u run interleaved with the epilogue of unit u - 1,
  // whose results are complete by then, so the matrix core and the VALU work side by side instead
  // of the epilogue waiting on the last MFMAs of its own unit.  Units alternate between two
  // accumulator sets; an epilogue reads registers only (FP8 column scales and norms are copied out
  // of LDS with the unit's operands), so the ring stage of a finished tile can be refilled while
  // its last epilogue is still pending.
  constexpr bool ST2 = SP && !GPD;                 // second MFMA stream (residual rows)
  // The pipeline keeps two accumulator sets live; a direct spill over long rows (whose X and R
  // operands fill most of the registers) runs each unit's epilogue right after its MFMAs instead.
  constexpr bool PIPE = !(ST2 && DP * T::BYTES > 512);
  constexpr int GU = PIPE ? (NB >= 2 ? NB / 2 : 1) : NB;   // blocks per unit
  static_assert(PIPE || NB <= 4, "one unit per tile without the pipeline");
  constexpr int NU = NB / GU;                      // units per tile
  static_assert(NU == 1 || NU == 2, "one or two units per tile");
  // block b of unit g: g + NU b, so with two units each unit's blocks share one parity class
  v4f accS[2][SPW][GU], accT[2][ST2 ? SPW : 1][GU];
  // GR: ||c_j||^2 for row 15; FP8: E8M0 scale of the lane's column (2 / its quantization scale)
  float ucn[2][GR ? GU : 1];
  int usc[2][GU];

  auto mfma_unit = [&](auto set, const char* tile, int g) __attribute__((always_inline)) {
    constexpr int S = decltype(set)::value;
    const char* tb = tile + lane_b;
#pragma unroll
    for (int b = 0; b < GU; ++b) {
      const int blk = g + NU * b;
      v4f init = v4f{0.f, 0.f, 0.f, 0.f};
      if constexpr (GR) ucn[S][b] = *reinterpret_cast<const float*>(tile + lane_cn + blk * 256);
      else init = *reinterpret_cast<const v4f*>(tile + lane_cn + blk * 256);
      usc[S][b] = BF ? 127 : *reinterpret_cast<const int*>(tile + R::CS_OFF + (blk * 16 + c16) * 4);
#pragma unroll
      for (int st = 0; st < SPW; ++st) {
        accS[S][st][b] = GR ? a2[st] : init;
        if constexpr (ST2) accT[S][st][b] = a2[st];
      }
    }
#pragma unroll
    for (int s = 0; s < NSTEP; ++s) {
      u32x4 bv[GU][W4];
#pragma unroll
      for (int b = 0; b < GU; ++b)
#pragma unroll
        for (int ww = 0; ww < W4; ++ww)
          bv[b][ww] = *reinterpret_cast<const u32x4*>(tb + (g + NU * b) * 16 * R::LDWB +
                                                      s * T::LANE_B + ww * 16);
#pragma unroll
      for (int b = 0; b < GU; ++b)
#pragma unroll
        for (int st = 0; st < SPW; ++st) {
          accS[S][st][b] =
              mfma_step<FMT>(xa[st].v[s], bv[b], accS[S][st][b], xsc[st], usc[S][b]);
          if constexpr (ST2)
            accT[S][st][b] =
                mfma_step<FMT>(ra[st].v[s], bv[b], accT[S][st][b], rsc[st], usc[S][b]);
        }
    }
  };

  // Epilogue of unit (ts, g) from accumulator set S: ranking values, class minima (block index
  // packed in the low mantissa bits); with_mask compares the columns against each row's primary
  // and only runs for tiles that hold one.  It is split into a preparation and one slot per row
  // of the lane (i = st * 4 + v), so that the slots can be spread between MFMAs.
  unsigned etc[GU];                               // the unit's block codes (wave-uniform)
  float espv[GPD ? SPW : 1][GU];                  // GPD: S of each stripe's centroid row
  // GR: do all stripes of the wave share their primary?  (Stripes are ordered by primary, so
  // most waves' stripes do.)  Wave-uniform.
  // If not, do they hold only the primaries of the first and the last stripe (a wave across one
  // partition boundary)?  Then two broadcasts serve them, and psel picks each stripe's.
  bool samep = false, twop = false;
  const int plane = GR ? sd[0].x - c16 : 0;       // GR: first column of a block whose lane c16 is p
  bool psel[GR ? SPW : 1];
  if constexpr (GR && SPW > 1) {
    bool same = true, two = true;
#pragma unroll
    for (int st = 0; st < SPW; ++st) {
      const bool first = sd[st].x == sd[0].x;
      same = same && first;
      two = two && (first || sd[st].x == sd[SPW - 1].x);
      psel[st] = __builtin_amdgcn_readfirstlane((int)first) != 0;
    }
    samep = __builtin_amdgcn_readfirstlane((int)same) != 0;
    twop = __builtin_amdgcn_readfirstlane((int)two) != 0;
  }
  // em (wave-uniform, fixed for the wave's lifetime): 1 when every stripe shares its primary
  // (GR); the sweep loop is instantiated once per value, so that a shared broadcast is one
  // register per block in the epilogue rather than a copy per stripe.
  auto epi_prep = [&](auto set, auto em, int ts, int g) __attribute__((always_inline)) {
    constexpr int S = decltype(set)::value;
    // each packing is then one v_and_or with an SGPR
#pragma unroll
    for (int b = 0; b < GU; ++b)
      etc[b] = (unsigned)__builtin_amdgcn_readfirstlane((t0 + ts) * NB + g + NU * b);
    // GPD: stripe row 15 is lane group 3 (lanes 48..63), register 3.  It is broadcast to every
    // lane group with two lane swaps instead of an LDS permute: after the 32-lane swap of a
    // register with itself the second result holds lanes 32..63 in both halves, and after the
    // 16-lane swap of that with itself the second result holds lanes 48..63 in all four groups.
    if constexpr (GPD) {
      auto row15 = [&](int st, int b) __attribute__((always_inline)) -> unsigned {
        const float v3 = GR ? accS[S][st][b][3] + ucn[S][b] : accS[S][st][b][3];
        return __builtin_bit_cast(unsigned, v3);
      };
      auto bcast = [&](int st, int b) __attribute__((always_inline)) -> float {
        const unsigned u3 = row15(st, b);
        const auto h32 = __builtin_amdgcn_permlane32_swap(u3, u3, false, false);
        const auto h16 = __builtin_amdgcn_permlane16_swap(h32[1], h32[1], false, false);
        return __builtin_bit_cast(float, (unsigned)h16[1]);
      };
      // both blocks of a two-block unit at once: with lane groups [x0 x1 x2 x3], the 32-lane
      // swap of (a, b) leaves [a2 a3 b2 b3] second, the 16-lane swap of that with itself
      // [a3 a3 b3 b3] second, and the 32-lane swap of that with itself [a3 a3 a3 a3] first and
      // [b3 b3 b3 b3] second: three swaps for two broadcasts instead of four
      auto bcast2 = [&](int st, float& e0, float& e1) __attribute__((always_inline)) {
        const auto h32 = __builtin_amdgcn_permlane32_swap(row15(st, 0), row15(st, 1), false, false);
        const auto h16 = __builtin_amdgcn_permlane16_swap(h32[1], h32[1], false, false);
        const auto g32 = __builtin_amdgcn_permlane32_swap(h16[1], h16[1], false, false);
        e0 = __builtin_bit_cast(float, (unsigned)g32[0]);
        e1 = __builtin_bit_cast(float, (unsigned)g32[1]);
      };
      if (GR && decltype(em)::value == 1) {
        // every stripe of the wave has the same centroid row: one broadcast serves them all.
        // The shared primary's column is masked here, once per block: its D_j becomes kBig, so
        // its value z^2 + kBig never leads a class (the sweep takes no masked epilogue).
        float e[GU];
        if constexpr (GU == 2) {
          bcast2(0, e[0], e[1]);
        } else {
#pragma unroll
          for (int b = 0; b < GU; ++b) e[b] = bcast(0, b);
        }
#pragma unroll
        for (int b = 0; b < GU; ++b) {
          e[b] = ts * BN + (g + NU * b) * 16 == plane ? kBig : e[b];
#pragma unroll
          for (int st = 0; st < SPW; ++st) espv[st][b] = e[b];
        }
      } else if (GR && SPW > 2 && twop) {
        if constexpr (GU == 2) {
          float f0, f1, l0, l1;
          bcast2(0, f0, f1);
          bcast2(SPW - 1, l0, l1);
#pragma unroll
          for (int st = 0; st < SPW; ++st) {
            espv[st][0] = psel[st] ? f0 : l0;
            espv[st][1] = psel[st] ? f1 : l1;
          }
        } else {
#pragma unroll
          for (int b = 0; b < GU; ++b) {
            const float e0 = bcast(0, b), e1 = bcast(SPW - 1, b);
#pragma unroll
            for (int st = 0; st < SPW; ++st) espv[st][b] = psel[st] ? e0 : e1;
          }
        }
      } else {
#pragma unroll
        for (int st = 0; st < SPW; ++st) {
          if constexpr (GU == 2) {
            bcast2(st, espv[st][0], espv[st][1]);
          } else {
#pragma unroll
            for (int b = 0; b < GU; ++b) espv[st][b] = bcast(st, b);
          }
        }
      }
    }
  };
  auto epi_slot = [&](auto set, auto with_mask, int i, int ts, int g)
                      __attribute__((always_inline)) {
    constexpr int S = decltype(set)::value;
    const int st = i / 4, v = i % 4;
    float pv[GU];
#pragma unroll
    for (int b = 0; b < GU; ++b) {
      // S = ||c_j||^2 - 2 <row, c_j>: the accumulator itself
      float val = accS[S][st][b][v];
      if constexpr (GR) {
        val = fmaf(val, val, espv[st][b]);             // D_j + z^2
      } else if constexpr (GPD) {
        const float tt = fmaf(gs[i], espv[st][b] - val, gm[i]);
        val = fmaf(tt, tt, val);
      } else if constexpr (SP) {
        val = fmaf(accT[S][st][b][v], accT[S][st][b][v], val);
      }
      if constexpr (SP && decltype(with_mask)::value)
        val = (ts * BN + (g + NU * b) * 16 + c16 == kp[i]) ? kBig : val;
      pv[b] = pack_code(val, cmask, etc[b]);
    }
    // block g + NU b has class (g + NU b) % NCLS: one class for the whole unit when NU == 2
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
      if constexpr (CAND == 1) {
        float m = kept[i][c];
#pragma unroll
        for (int b = 0; b < GU; ++b)
          if ((NU == 2 ? g % NCLS : b % NCLS) == c) m = fminf(m, pv[b]);
        kept[i][c] = m;
      } else {
#pragma unroll
        for (int b = 0; b < GU; ++b)
          if ((NU == 2 ? g % NCLS : b % NCLS) == c) {
            // two smallest: the new second is the median of (first, second, new)
            kept[i][2 * c + 1] = __builtin_amdgcn_fmed3f(kept[i][2 * c], kept[i][2 * c + 1], pv[b]);
            kept[i][2 * c] = fminf(kept[i][2 * c], pv[b]);
          }
      }
    }
  };
  auto epi_unit = [&](auto set, auto em, auto with_mask, int ts, int g)
                      __attribute__((always_inline)) {
    epi_prep(set, em, ts, g);
#pragma unroll
    for (int i = 0; i < NR; ++i) epi_slot(set, with_mask, i, ts, g);
  };

  // The MFMAs of unit (t, g) into set S with the epilogue of the previous unit (set 1 - S) placed
  // by hand between them: a few row slots while the first operands arrive from LDS, the rest
  // spread evenly after the MFMAs; scheduling barriers keep that order, so the wave always has
  // independent VALU work to issue while the matrix core runs.
  auto fused_unit = [&](auto set, auto em, const char* tile, int g, int tsp, int gp)
                        __attribute__((always_inline)) {
    constexpr int S = decltype(set)::value;
    const auto pset = std::integral_constant<int, 1 - S>{};
    constexpr int NMI = NSTEP * GU * SPW * (ST2 ? 2 : 1);   // MFMAs of the unit
    constexpr int PRE = NR / 4;                              // slots before the first MFMA
    const char* tb = tile + lane_b;
    v4f init[GU];
#pragma unroll
    for (int b = 0; b < GU; ++b) {
      const int blk = g + NU * b;
      if constexpr (GR) {
        init[b] = v4f{0.f, 0.f, 0.f, 0.f};
        ucn[S][b] = *reinterpret_cast<const float*>(tile + lane_cn + blk * 256);
      } else {
        init[b] = *reinterpret_cast<const v4f*>(tile + lane_cn + blk * 256);
      }
      usc[S][b] = BF ? 127 : *reinterpret_cast<const int*>(tile + R::CS_OFF + (blk * 16 + c16) * 4);
    }
    u32x4 bv[2][GU][W4];
    auto read_step = [&](int s, int k) __attribute__((always_inline)) {
#pragma unroll
      for (int b = 0; b < GU; ++b)
#pragma unroll
        for (int ww = 0; ww < W4; ++ww)
          bv[k][b][ww] = *reinterpret_cast<const u32x4*>(tb + (g + NU * b) * 16 * R::LDWB +
                                                         s * T::LANE_B + ww * 16);
    };
    read_step(0, 0);
    if constexpr (NSTEP > 1) read_step(1, 1);
    epi_prep(pset, em, tsp, gp);
#pragma unroll
    for (int i = 0; i < PRE; ++i) epi_slot(pset, std::false_type{}, i, tsp, gp);
    __builtin_amdgcn_sched_barrier(0);
    int mi = 0;                                    // MFMAs issued so far (compile-time)
#pragma unroll
    for (int s = 0; s < NSTEP; ++s) {
#pragma unroll
      for (int b = 0; b < GU; ++b)
#pragma unroll
        for (int st = 0; st < SPW; ++st)
#pragma unroll
          for (int x = 0; x < (ST2 ? 2 : 1); ++x) {
            if (x == 0) {
              accS[S][st][b] = mfma_step<FMT>(xa[st].v[s], bv[s & 1][b],
                                              s == 0 ? (GR ? a2[st] : init[b])
                                                     : accS[S][st][b],
                                              xsc[st], usc[S][b]);
            } else {
              accT[S][st][b] = mfma_step<FMT>(ra[st].v[s], bv[s & 1][b],
                                              s == 0 ? a2[st] : accT[S][st][b],
                                              rsc[st], usc[S][b]);
            }
            // row slots [lo, hi) follow MFMA mi
            const int lo = PRE + mi * (NR - PRE) / NMI, hi = PRE + (mi + 1) * (NR - PRE) / NMI;
#pragma unroll
            for (int i = PRE; i < NR; ++i)
              if (i >= lo && i < hi) epi_slot(pset, std::false_type{}, i, tsp, gp);
            ++mi;
            __builtin_amdgcn_sched_barrier(0);
          }
      if (s + 2 < NSTEP) read_step(s + 2, s & 1);
    }
  };

  // does tile t hold the primary of any row of the wave? (wave-uniform)
  auto tile_masked = [&](int t) __attribute__((always_inline)) -> bool {
    if constexpr (!SP) {
      return false;
    } else {
      bool hit = false;
#pragma unroll
      for (int i = 0; i < NRS; ++i) hit |= (unsigned)(kp[i] - t * BN) < (unsigned)BN;
      return __builtin_amdgcn_readfirstlane((int)__any(hit)) != 0;
    }
  };

  const char* tile = s_ring;
  int stage = 0;
  bool m_cur = false, m_last = false;             // masks of the current and the previous tile
  // Start of tile t: its record is in LDS for every wave, and a later record is issued.
  auto begin_tile = [&](int t) __attribute__((always_inline)) {
    // record t has landed in LDS for this wave (later records may still be in flight) ...
    // (vmcnt counts VMEM operations of this wave in order: with later records in flight,
    // leaving at most the last record's NI copies outstanding means record t is complete)
    if (STG > 2 && t + 1 < ntiles)
      wait_vmcnt<NI>();
    else
      wait_vmcnt<0>();
    // ... and for every wave; every wave is also done reading the stage refilled next (its
    // last reads were the B operands of tile t - 1, issued before this barrier)
    __builtin_amdgcn_s_barrier();
    if (t + STG - 1 < ntiles)
      issue(t + STG - 1);
    tile = s_ring + stage * STAGE;
    stage = stage + 1 == STG ? 0 : stage + 1;
    m_last = m_cur;
    m_cur = tile_masked(t);
  };
  const auto s0 = std::integral_constant<int, 0>{};
  const auto s1 = std::integral_constant<int, 1>{};
  // One pipeline step: unit (current tile, g) into set S, and the epilogue of the previous unit
  // (tp, gp) from set 1 - S, masked when that unit's tile holds a primary (mp).
  auto step = [&](auto set, auto em, int g, int tp, int gp, bool mp)
                  __attribute__((always_inline)) {
    const auto prev = std::integral_constant<int, 1 - decltype(set)::value>{};
    if (decltype(em)::value != 1 && __builtin_expect(mp, 0)) {
      epi_unit(prev, em, std::true_type{}, tp, gp);
      mfma_unit(set, tile, g);
    } else {
      fused_unit(set, em, tile, g, tp, gp);
    }
  };
  auto drain = [&](auto set, auto em, int tp, int gp) __attribute__((always_inline)) {
    if (decltype(em)::value != 1 && m_cur) epi_unit(set, em, std::true_type{}, tp, gp);
    else epi_unit(set, em, std::false_type{}, tp, gp);
  };
  // The tile loop, with the first unit peeled and the sets fixed per position, so that no
  // accumulator changes registers between iterations.
  auto run = [&](auto em) __attribute__((always_inline)) {
    if constexpr (!PIPE) {
      for (int t = 0; t < ntiles; ++t) {
        begin_tile(t);
        mfma_unit(s0, tile, 0);
        drain(s0, em, t, 0);
      }
    } else if constexpr (NU == 2) {
      // units (t, 0) in set 0 and (t, 1) in set 1
      begin_tile(0);
      mfma_unit(s0, tile, 0);
      step(s1, em, 1, 0, 0, m_cur);
      for (int t = 1; t < ntiles; ++t) {
        begin_tile(t);
        step(s0, em, 0, t - 1, 1, m_last);
        step(s1, em, 1, t, 0, m_cur);
      }
      drain(s1, em, ntiles - 1, 1);
    } else {
      // one unit per tile: even tiles in set 0, odd tiles in set 1
      begin_tile(0);
      mfma_unit(s0, tile, 0);
      int t = 1;
      for (; t + 1 < ntiles; t += 2) {
        begin_tile(t);
        step(s1, em, 0, t - 1, 0, m_last);
        begin_tile(t + 1);
        step(s0, em, 0, t, 0, m_last);
      }
      if (t < ntiles) {
        begin_tile(t);
        step(s1, em, 0, t - 1, 0, m_last);
        drain(s1, em, t, 0);
      } else {
        drain(s0, em, t - 1, 0);
      }
    }
  };
  if constexpr (GR && SPW > 1) {
    if (samep) run(std::integral_constant<int, 1>{});
    else run(std::integral_constant<int, 0>{});
  } else {
    run(std::integral_constant<int, 0>{});
  }

  // candidates: the topk smallest kept values of every row across its 16 lanes (value, then
  // column), by repeated extraction: each lane orders its NS keys, the row takes the least head
  // of its lanes (DPP minima, so all 16 lanes agree), and the lane that held it moves on
  const int topk = P.topk;
  const unsigned cfield = (1u << cbits) - 1u;
#pragma unroll
  for (int st = 0; st < SPW; ++st)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = st * 4 + v;
      const int64_t r = row_of(st, 4 * q + v);
      float kv[NS];
      int kj[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        kv[k] = kept[i][k];
        const bool valid = kv[k] < 1.0e38f;
        // (slots without a value get distinct keys past every column, so every one of the topk
        // places is written, with -1)
        kj[k] = valid ? (int)((__builtin_bit_cast(unsigned, kv[k]) & cfield) * 16u) + c16
                      : 0x7fffff00 + c16 * NS + k;
        if (!valid) kv[k] = kInf;
      }
      // order the lane's keys (a small exchange network)
#pragma unroll
      for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int b = 0; b + 1 < NS - a; ++b) {
          const bool sw = kv[b + 1] < kv[b] || (kv[b + 1] == kv[b] && kj[b + 1] < kj[b]);
          const float tv = sw ? kv[b + 1] : kv[b];
          const int tj = sw ? kj[b + 1] : kj[b];
          kv[b + 1] = sw ? kv[b] : kv[b + 1];
          kj[b + 1] = sw ? kj[b] : kj[b + 1];
          kv[b] = tv;
          kj[b] = tj;
        }
      int head = 0;
      for (int k = 0; k < topk; ++k) {
        float h = kInf;
        int hj = 0x7ffffff0 + c16;
#pragma unroll
        for (int a = 0; a < NS; ++a)
          if (head == a) { h = kv[a]; hj = kj[a]; }
        float m = fminf(h, row_ror<8>(h));
        m = fminf(m, row_ror<4>(m));
        m = fminf(m, row_ror<2>(m));
        m = fminf(m, row_ror<1>(m));
        int cj = h == m ? hj : 0x7fffffff;
        cj = min(cj, row_ror<8>(cj));
        cj = min(cj, row_ror<4>(cj));
        cj = min(cj, row_ror<2>(cj));
        cj = min(cj, row_ror<1>(cj));
        const bool win = h == m && hj == cj;
        if (win && r >= 0) {
          const int jj = (m < kInf && cj < P.K) ? cj : -1;
          if constexpr (!KS) {
            P.cand[r * topk + k] = jj;
          } else {                                 // per split, with values, for the merge
            const int64_t o = (r * gridDim.y + blockIdx.y) * topk + k;
            P.cand_split[o] = jj;
            P.cand_val[o] = jj >= 0 ? m : kInf;
          }
        }
        head += win ? 1 : 0;
      }
    }
}

// Candidates of a codebook swept in S splits: per row, the topk smallest (value, column) pairs
// of the S * topk the splits kept, in order.  The splits partition the columns, so every column
// appears at most once.
// Eight lanes per row: lane g holds the row's split candidates g, g + 8, ... (S topk <= 128 of
// them, so at most 16 per lane, loaded once); each of the topk rounds takes every lane's best
// candidate after the previous pick, and the row's best of those by three lane swaps.
constexpr int kMergeLanes = 8;
constexpr int kMergeMax = 128 / kMergeLanes;

__global__ __launch_bounds__(256) void lowp_merge_kernel(LowpParams P, int S) {
  const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kMergeLanes;
  const int g = threadIdx.x % kMergeLanes;
  const bool live = r < live_rows(P.n, P.live_n);
  const int topk = P.topk, m = S * topk;
  int j[kMergeMax];
  float v[kMergeMax];
#pragma unroll
  for (int e = 0; e < kMergeMax; ++e) {
    const int idx = g + kMergeLanes * e;
    const bool ok = live && idx < m;
    j[e] = ok ? P.cand_split[r * m + idx] : -1;
    v[e] = ok ? P.cand_val[r * m + idx] : kInf;
  }
  float pv = -kInf;                                // the previous pick: (pv, pj)
  int pj = -1;
  for (int k = 0; k < topk; ++k) {
    float bv = kInf;
    int bj = -1;
#pragma unroll
    for (int e = 0; e < kMergeMax; ++e) {
      const bool after = v[e] > pv || (v[e] == pv && j[e] > pj);
      const bool better = bj < 0 || v[e] < bv || (v[e] == bv && j[e] < bj);
      if (j[e] >= 0 && after && better) { bv = v[e]; bj = j[e]; }
    }
#pragma unroll
    for (int off = kMergeLanes / 2; off >= 1; off >>= 1) {
      const float ov = __shfl_xor(bv, off);
      const int oj = __shfl_xor(bj, off);
      if (oj >= 0 && (bj < 0 || ov < bv || (ov == bv && oj < bj))) { bv = ov; bj = oj; }
    }
    if (live && g == 0) P.cand[r * topk + k] = bj;
    if (bj >= 0) { pv = bv; pj = bj; }
  }
}

hipError_t launch_lowp_merge(const LowpParams& P, hipStream_t st) {
  if (P.ksplit <= 1) return hipSuccess;
  if (!P.cand_split || !P.cand_val || P.ksplit * P.topk > kMergeLanes * kMergeMax)
    return hipErrorInvalidValue;
  const int64_t threads = P.n * kMergeLanes;
  hipLaunchKernelGGL(lowp_merge_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st,
                     P, P.ksplit);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Re-score: 16 lanes per row (4 rows per wave), FP32 direct differences, FP64 among near-ties.
// ------------------------------------------------------------------------------------------------
// A row's 16 lanes are one DPP row, so its sums and maxima take four rotate-and-combine steps
// (row_ror by 8, 4, 2, 1) instead of chains of LDS permutes.  Each step combines the same two
// partial results in both lanes of a pair, so all 16 lanes end with the bitwise-same value.
__device__ __forceinline__ float sum16(float v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  return v + row_ror<1>(v);
}
__device__ __forceinline__ double sum16d(double v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  return v + row_ror<1>(v);
}
__device__ __forceinline__ float max16(float v) {
  v = fmaxf(v, row_ror<8>(v));
  v = fmaxf(v, row_ror<4>(v));
  v = fmaxf(v, row_ror<2>(v));
  return fmaxf(v, row_ror<1>(v));
}

// RS_MAXD: dimensions held per lane.  Scalar layout: lane l16 holds l16, l16 + 16, ...
// (d <= 16 RS_MAXD).  V4 layout (d % 4 == 0, 16-byte aligned rows): lane l16 holds the float4
// chunks 4 l16 + 64 m (d <= 16 RS_MAXD), so every load is a 16-byte vector load.  Values past d
// are zero in both layouts, so the loops need no guards.
template <bool V4>
__device__ __forceinline__ int rs_dim(int l16, int m) {
  return V4 ? 4 * l16 + 64 * (m >> 2) + (m & 3) : l16 + 16 * m;
}
template <bool V4, int RS_MAXD>
__device__ __forceinline__ void rs_load(const float* __restrict__ p, int d, int l16,
                                        float (&v)[RS_MAXD]) {
  if constexpr (V4) {
#pragma unroll
    for (int m = 0; m < RS_MAXD; m += 4) {
      const int k = 4 * l16 + 16 * m;
      v4f t = {0.f, 0.f, 0.f, 0.f};
      if (k < d) t = *reinterpret_cast<const v4f*>(p + k);
      v[m] = t.x; v[m + 1] = t.y; v[m + 2] = t.z; v[m + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int m = 0; m < RS_MAXD; ++m) {
      const int k = l16 + 16 * m;
      v[m] = k < d ? p[k] : 0.f;
    }
  }
}

// DX > 0: the row length is DX (= P.d), known at compile time, so the row loads need no
// run-time bounds and the row addresses fold.
// Short float4 rows (at most 8 dimensions per lane) ask for 8 waves per SIMD: the re-score waits
// on gathered candidate rows, and more waves in flight hide that (n=1M, d=128: 334 -> 308 us).
// (The scalar layout would spill registers at that occupancy.)
template <int FMT, bool SP, int RS_MAXD, bool V4, int DX = 0>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(V4 && RS_MAXD <= 8 ? 8 : 1, 8)))
void lowp_rescore_kernel(LowpParams P) {
  static_assert(!V4 || RS_MAXD % 4 == 0, "V4 layout holds whole float4 chunks");
  static_assert(DX <= 16 * RS_MAXD, "a lane holds at most RS_MAXD dimensions");
  const int l16 = threadIdx.x & 15;
  const int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  if (row >= live_rows(P.n, P.live_n)) return;
  const int d = DX > 0 ? DX : P.d, topk = P.topk;
  float x[RS_MAXD], r[RS_MAXD];
  rs_load<V4, RS_MAXD>(P.X + row * d, d, l16, x);
  int pi = -1;
  float rr = 0.f, lr = 0.f;                       // ||r||^2 and lambda / ||r||^2
  if constexpr (SP) {
    pi = P.primary[row];
    if (pi < 0 || pi >= P.K) {   // no primary: nothing to spill
      if (l16 == 0) { P.spill[row] = -1; if (P.sloss) P.sloss[row] = kInf; }
      return;
    }
    rs_load<V4, RS_MAXD>(P.C + (int64_t)pi * d, d, l16, r);
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int m = 0; m < RS_MAXD; ++m) {
      r[m] = x[m] - r[m];
      if (m & 1) a1 = fmaf(r[m], r[m], a1); else a0 = fmaf(r[m], r[m], a0);
    }
    rr = sum16(a0 + a1);
    lr = rr > 0.f ? P.lam / rr : 0.f;             // one division per row, not per candidate
  }
  // FP32 pass
  float best = kInf;
  int bj = 0x7fffffff;
  float vals[kMaxTopk];
#pragma unroll
  for (int c = 0; c < kMaxTopk; ++c) {
    vals[c] = kInf;
    if (c >= topk) continue;
    const int j = P.cand[row * topk + c];
    if (j < 0 || j >= P.K || (SP && j == pi)) continue;
    float cv[RS_MAXD];
    rs_load<V4, RS_MAXD>(P.C + (int64_t)j * d, d, l16, cv);
    float s0 = 0.f, s1 = 0.f, p0 = 0.f, p1 = 0.f;
#pragma unroll
    for (int m = 0; m < RS_MAXD; ++m) {
      const float e = x[m] - cv[m];
      if (m & 1) { s1 = fmaf(e, e, s1); if (SP) p1 = fmaf(r[m], e, p1); }
      else { s0 = fmaf(e, e, s0); if (SP) p0 = fmaf(r[m], e, p0); }
    }
    const float sq = sum16(s0 + s1);
    float val = sq;
    if constexpr (SP) {
      const float pj = sum16(p0 + p1);
      val = fmaf(lr, pj * pj, sq);
    }
    vals[c] = val;
    if (val < best || (val == best && j < bj)) { best = val; bj = j; }
  }
  if (bj == 0x7fffffff) {
    if (l16 == 0) {
      if (SP) { P.spill[row] = -1; if (P.sloss) P.sloss[row] = kInf; }
      else {
        P.primary[row] = -1;
        if (P.pdist) P.pdist[row] = kInf;
        if (P.radius) P.radius[row] = kInf;      // no primary: no spill, no bound
      }
    }
    return;
  }
  // FP64 among near-ties
  const float lim = best + best * P.tie_rel;
  int ntie = 0;
#pragma unroll
  for (int c = 0; c < kMaxTopk; ++c) ntie += vals[c] <= lim;
  if (ntie >= 2) {
    double bd = __builtin_inf();
    int bdj = 0x7fffffff;
    float cpv[SP ? RS_MAXD : 1];
    if constexpr (SP) rs_load<V4, RS_MAXD>(P.C + (int64_t)pi * d, d, l16, cpv);
#pragma unroll
    for (int c = 0; c < kMaxTopk; ++c) {
      if (!(vals[c] <= lim)) continue;
      const int j = P.cand[row * topk + c];
      float cv[RS_MAXD];
      rs_load<V4, RS_MAXD>(P.C + (int64_t)j * d, d, l16, cv);
      double sq = 0.0, pj = 0.0, r2 = 0.0;
#pragma unroll
      for (int m = 0; m < RS_MAXD; ++m) {
        const double e = (double)x[m] - (double)cv[m];
        sq = fma(e, e, sq);
        if constexpr (SP) {
          const double rk = (double)x[m] - (double)cpv[m];
          pj = fma(rk, e, pj);
          r2 = fma(rk, rk, r2);
        }
      }
      sq = sum16d(sq);
      double val = sq;
      if constexpr (SP) {
        pj = sum16d(pj);
        r2 = sum16d(r2);
        if (r2 > 0.0) val = sq + (double)P.lam * (pj * pj) / r2;
      }
      argmin_d(bd, bdj, val, j);
    }
    best = (float)bd;
    bj = bdj;
    if (l16 == 0) atomicAdd(&P.counters[CNT_FP64], 1u);
  }
  if constexpr (SP) {
    if (l16 == 0) { P.spill[row] = bj; if (P.sloss) P.sloss[row] = best; }
    return;
  }
  if (l16 == 0) { P.primary[row] = bj; if (P.pdist) P.pdist[row] = best; }
  // residual of the chosen primary, quantized for the spill sweep, and its row constants
  rs_load<V4, RS_MAXD>(P.C + (int64_t)bj * d, d, l16, r);
  float a0 = 0.f, r0 = 0.f, m0 = 0.f;
#pragma unroll
  for (int m = 0; m < RS_MAXD; ++m) {
    r[m] = x[m] - r[m];
    a0 = fmaf(r[m], x[m], a0);
    r0 = fmaf(r[m], r[m], r0);
    m0 = fmaxf(m0, fabsf(r[m]));
  }
  const float a = sum16(a0), r2 = sum16(r0);
  // sigma = sqrt(lambda) / (2 ||r||): the residual rows are stored pre-scaled by it, FP8 ones
  // with a power-of-two scale of their own
  const float rn = sqrtf(r2);
  if (P.radius) {
    // Spill bound: U = (1 + lambda) ||x - c_j2||^2 for the nearest other candidate j2 bounds the
    // spill's loss, so the spill lies within ||r|| + sqrt(U) of c_pi (raised by a margin for the
    // FP32 rounding of both terms); launch_bound_decide compares it with c_pi's table entry.
    float second = kInf;
#pragma unroll
    for (int c = 0; c < kMaxTopk; ++c) {
      if (c >= topk) continue;
      if (P.cand[row * topk + c] != bj) second = fminf(second, vals[c]);
    }
    const float rad = (rn + sqrtf((1.f + P.lam) * second)) * (1.f + 4.f * (float)(d + 8) * kU32);
    if (l16 == 0) P.radius[row] = rad;
  }
  const float sigma = rn > 0.f ? 0.5f * sqrtf(P.lam) / rn : 0.f;
  float inv = 1.f, scale = 1.f;
  if constexpr (FMT == LOWP_FP8) {
    const float mx = max16(m0) * sigma;
    if (mx > 0.f) {
      int e;
      (void)frexpf(mx, &e);
      scale = ldexpf(1.f, 8 - e);
      inv = 1.f / scale;
    }
  }
  if (l16 == 0) P.rowc_out[row] = float4{inv, a, r2 > 0.f ? P.lam / r2 : 0.f, sigma};
  if (!P.Rq_out) return;   // grouped form over X rows: no residual rows
  // the whole padded row is written: the padding must hold zeros, not old workspace bytes
  const int dp = P.dp;
  if constexpr (FMT == LOWP_FP8) {
    unsigned char* o = static_cast<unsigned char*>(P.Rq_out) + row * dp;
#pragma unroll
    for (int m = 0; m < RS_MAXD; ++m) {
      const int k = rs_dim<V4>(l16, m);
      if (k < d) o[k] = fp8_of(sigma * r[m] * scale);
    }
    for (int k = d + l16; k < dp; k += 16) o[k] = (unsigned char)0;
  } else {
    __bf16* o = static_cast<__bf16*>(P.Rq_out) + row * dp;
#pragma unroll
    for (int m = 0; m < RS_MAXD; ++m) {
      const int k = rs_dim<V4>(l16, m);
      if (k < d) o[k] = (__bf16)(sigma * r[m]);
    }
    for (int k = d + l16; k < dp; k += 16) o[k] = (__bf16)0.f;
  }
}

// ------------------------------------------------------------------------------------------------
// Host-side launchers
// ------------------------------------------------------------------------------------------------
int lowp_padded_dim(int fmt, int d) {
  static const int bf[] = {32, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
  static const int f8[] = {128, 256, 384, 512, 768, 1024};
  if (fmt == LOWP_BF16) {
    for (int v : bf) if (d <= v) return v;
  } else {
    for (int v : f8) if (d <= v) return v;
  }
  return -1;
}

hipError_t launch_lowp_quantize(int fmt, const float* A, int64_t rows, int d, int dp,
                                bool codebook, void* out, float* inv_scale, unsigned* counters,
                                hipStream_t st, const int64_t* live_n) {
  const dim3 grid((unsigned)((rows + 15) / 16)), block(256);
  const bool v4 = d % 4 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0;
  if (fmt == LOWP_BF16 && v4)
    hipLaunchKernelGGL((quantize_rows_kernel<LOWP_BF16, true>), grid, block, 0, st, A, rows, d, dp,
                       codebook ? -2.f : 1.f, out, inv_scale, counters, live_n);
  else if (fmt == LOWP_BF16)
    hipLaunchKernelGGL(quantize_rows_kernel<LOWP_BF16>, grid, block, 0, st, A, rows, d, dp,
                       codebook ? -2.f : 1.f, out, inv_scale, counters, live_n);
  else if (v4)
    hipLaunchKernelGGL((quantize_rows_kernel<LOWP_FP8, true>), grid, block, 0, st, A, rows, d, dp,
                       1.f, out, inv_scale, counters, live_n);
  else
    hipLaunchKernelGGL(quantize_rows_kernel<LOWP_FP8>, grid, block, 0, st, A, rows, d, dp, 1.f,
                       out, inv_scale, counters, live_n);
  return hipGetLastError();
}

// Tile shapes per padded width: SPW stripes of 16 rows per wave in the primary / spill sweep,
// BN centroids per tile, STG ring stages.
template <int FMT, int DP>
struct SweepShape;
#define SOAR_SHAPE(F, D, SP_P, W_P, SP_S, W_S, B, S)                                \
  template <>                                                                       \
  struct SweepShape<F, D> {                                                         \
    static constexpr int SPW_P = SP_P, WPE_P = W_P, SPW_S = SP_S, WPE_S = W_S;      \
    static constexpr int BN = B, STG = S;                                           \
  };
#define SOAR_SHAPE_X(...) SOAR_SHAPE(__VA_ARGS__)
// (the most used widths can be set at build time, e.g. -DSOAR_SHAPE_BF16_96=4,2,2,2,64,3)
#ifndef SOAR_SHAPE_BF16_96
#define SOAR_SHAPE_BF16_96 4, 2, 2, 2, 64, 3
#endif
#ifndef SOAR_SHAPE_BF16_128
#define SOAR_SHAPE_BF16_128 4, 2, 2, 1, 64, 3
#endif
#ifndef SOAR_SHAPE_BF16_768
#define SOAR_SHAPE_BF16_768 4, 1, 2, 1, 32, 2
#endif
#ifndef SOAR_SHAPE_FP8_768
#define SOAR_SHAPE_FP8_768 2, 1, 2, 1, 32, 2
#endif
//         format     DP  primary  spill   BN  stages   (SPW stripes, waves per SIMD)
SOAR_SHAPE(LOWP_BF16, 32, 4, 2, 2, 2, 64, 3)
SOAR_SHAPE(LOWP_BF16, 64, 4, 2, 2, 2, 64, 3)
SOAR_SHAPE_X(LOWP_BF16, 96, SOAR_SHAPE_BF16_96)
SOAR_SHAPE_X(LOWP_BF16, 128, SOAR_SHAPE_BF16_128)
SOAR_SHAPE(LOWP_BF16, 192, 2, 1, 2, 1, 64, 3)
SOAR_SHAPE(LOWP_BF16, 256, 2, 1, 1, 1, 64, 3)
SOAR_SHAPE(LOWP_BF16, 384, 1, 1, 1, 1, 64, 2)
SOAR_SHAPE(LOWP_BF16, 512, 1, 2, 1, 1, 32, 2)
SOAR_SHAPE_X(LOWP_BF16, 768, SOAR_SHAPE_BF16_768)
SOAR_SHAPE(LOWP_BF16, 1024, 1, 1, 1, 1, 16, 2)
SOAR_SHAPE(LOWP_FP8, 128, 2, 2, 2, 2, 64, 3)
SOAR_SHAPE(LOWP_FP8, 256, 2, 2, 2, 1, 64, 3)
SOAR_SHAPE(LOWP_FP8, 384, 2, 1, 1, 1, 64, 3)
SOAR_SHAPE(LOWP_FP8, 512, 2, 2, 1, 2, 64, 2)
SOAR_SHAPE_X(LOWP_FP8, 768, SOAR_SHAPE_FP8_768)
SOAR_SHAPE(LOWP_FP8, 1024, 1, 2, 1, 2, 32, 2)
#undef SOAR_SHAPE

// Codebook splits of a sweep: P.ksplit (launch_lowp_sweep checks P.ksplit <= K / 64; every tile
// holds at most 64 columns, so each split gets at least one tile and the merge's S matches).
template <int FMT, int DP>
static int ksplit_tiles(const LowpParams& P) {
  static_assert(SweepShape<FMT, DP>::BN <= 64, "a split per 64 columns covers a tile");
  return P.ksplit < 1 ? 1 : P.ksplit;
}

template <int FMT, int DP>
static void sweep_dp(const LowpParams& P, bool spill, hipStream_t st) {
  using S = SweepShape<FMT, DP>;
  if (spill) {
    constexpr int NW = lowp_wg_waves(S::WPE_S);
    const int ks = ksplit_tiles<FMT, DP>(P);
    const dim3 grid((unsigned)((P.n + 16 * NW * S::SPW_S - 1) / (16 * NW * S::SPW_S)),
                    (unsigned)ks);
    if (ks > 1)
      hipLaunchKernelGGL(
          (lowp_sweep_kernel<FMT, DP, S::SPW_S, S::BN, S::STG, S::WPE_S, true, false, false, true>),
          grid, dim3(64 * NW), 0, st, P);
    else
      hipLaunchKernelGGL((lowp_sweep_kernel<FMT, DP, S::SPW_S, S::BN, S::STG, S::WPE_S, true>),
                         grid, dim3(64 * NW), 0, st, P);
  } else {
    constexpr int NW = lowp_wg_waves(S::WPE_P);
    const int ks = ksplit_tiles<FMT, DP>(P);
    const dim3 grid((unsigned)((P.n + 16 * NW * S::SPW_P - 1) / (16 * NW * S::SPW_P)),
                    (unsigned)ks);
    if (ks > 1)
      hipLaunchKernelGGL(
          (lowp_sweep_kernel<FMT, DP, S::SPW_P, S::BN, S::STG, S::WPE_P, false, false, false, true>),
          grid, dim3(64 * NW), 0, st, P);
    else
      hipLaunchKernelGGL((lowp_sweep_kernel<FMT, DP, S::SPW_P, S::BN, S::STG, S::WPE_P, false>),
                         grid, dim3(64 * NW), 0, st, P);
  }
}

// The grouped spill runs one MFMA stream at the primary's waves per SIMD.  Over X rows it keeps
// two more row constants than the primary sweep and takes the spill's stripes per wave; over
// residual rows (GR) it keeps one, and takes the primary's up to 96 dimensions and at 768.  At
// 128 the primary's four stripes would spill registers; three measured 5% faster than two
// (BF16, n=1M, K=2000: 1.42 vs 1.50 ms).  At 768 (one wave per SIMD) four BF16 stripes per wave
// read each B operand from LDS for four MFMAs instead of two: 20.2 -> 16.1 ms at n=500K,
// K=10,000 (three stripes measured far slower, and FP8 gained nothing from three or four).
template <int FMT, int DP, bool GR>
static void sweep_grouped_dp(const LowpParams& P, hipStream_t st) {
  using S = SweepShape<FMT, DP>;
  constexpr int SPW = !GR                      ? S::SPW_S
                      : DP <= 96 || DP == 768 ? S::SPW_P
                      : DP == 128             ? 3
                                              : S::SPW_S;
  const int64_t ms = group_max_stripes(P.n, P.K);
  constexpr int NW = lowp_wg_waves(S::WPE_P);
  const dim3 grid((unsigned)((ms + NW * SPW - 1) / (NW * SPW)));
  hipLaunchKernelGGL((lowp_sweep_kernel<FMT, DP, SPW, S::BN, S::STG, S::WPE_P, true, true, GR>),
                     grid, dim3(64 * NW), 0, st, P);
}

template <int FMT, int DP>
static void pack_dp(const float* C, int K, int d, const float* cnorm, void* rec,
                    unsigned* counters, hipStream_t st) {
  constexpr int BN = SweepShape<FMT, DP>::BN;
  const int kpad = (K + BN - 1) / BN * BN;
  hipLaunchKernelGGL((pack_codebook_kernel<FMT, DP, BN>), dim3((unsigned)(kpad / 16)), dim3(256),
                     0, st, C, K, d, cnorm, static_cast<char*>(rec), counters);
}

template <int FMT, int DP>
static size_t rec_bytes_dp(int K) {
  using S = SweepShape<FMT, DP>;
  return (size_t)((K + S::BN - 1) / S::BN) * TileRec<FMT, DP, S::BN>::BYTES;
}

// Dispatch on the padded width with plain switches (kernel templates instantiated from generic
// lambdas did not get their host launch stubs emitted).
#define SOAR_DP_CASES(FMT, X)                                        \
  case 32: if constexpr (FMT == LOWP_BF16) { X(32); } break;         \
  case 64: if constexpr (FMT == LOWP_BF16) { X(64); } break;         \
  case 96: if constexpr (FMT == LOWP_BF16) { X(96); } break;         \
  case 128: X(128); break;                                           \
  case 192: if constexpr (FMT == LOWP_BF16) { X(192); } break;       \
  case 256: X(256); break;                                           \
  case 384: X(384); break;                                           \
  case 512: X(512); break;                                           \
  case 768: X(768); break;                                           \
  case 1024: X(1024); break;                                         \
  default: break;

template <int FMT>
static void sweep_fmt(const LowpParams& P, bool spill, hipStream_t st) {
#define X(D) sweep_dp<FMT, D>(P, spill, st)
  switch (P.dp) { SOAR_DP_CASES(FMT, X) }
#undef X
}

hipError_t launch_lowp_sweep(int fmt, const LowpParams& P, bool spill, hipStream_t st) {
  if (P.ksplit > 1 && ((int64_t)P.ksplit * 64 > P.K || !P.cand_split || !P.cand_val))
    return hipErrorInvalidValue;
  if (fmt == LOWP_BF16) sweep_fmt<LOWP_BF16>(P, spill, st);
  else sweep_fmt<LOWP_FP8>(P, spill, st);
  return hipGetLastError();
}

template <int FMT>
static void sweep_grouped_fmt(const LowpParams& P, hipStream_t st) {
  if (grouped_residual_rows(FMT, P.lam)) {
#define X(D) sweep_grouped_dp<FMT, D, true>(P, st)
    switch (P.dp) { SOAR_DP_CASES(FMT, X) }
#undef X
    return;
  }
#define X(D) sweep_grouped_dp<FMT, D, false>(P, st)
  switch (P.dp) { SOAR_DP_CASES(FMT, X) }
#undef X
}

hipError_t launch_lowp_sweep_grouped(int fmt, const LowpParams& P, hipStream_t st) {
  if (!P.perm || !P.stripes || !P.nstripes || !P.Cp) return hipErrorInvalidValue;
  if (fmt == LOWP_BF16) sweep_grouped_fmt<LOWP_BF16>(P, st);
  else sweep_grouped_fmt<LOWP_FP8>(P, st);
  return hipGetLastError();
}

template <int FMT>
static size_t rec_bytes_fmt(int dp, int K) {
  size_t b = 0;
#define X(D) b = rec_bytes_dp<FMT, D>(K)
  switch (dp) { SOAR_DP_CASES(FMT, X) }
#undef X
  return b;
}

size_t lowp_codebook_bytes(int fmt, int d, int K) {
  const int dp = lowp_padded_dim(fmt, d);
  return fmt == LOWP_BF16 ? rec_bytes_fmt<LOWP_BF16>(dp, K) : rec_bytes_fmt<LOWP_FP8>(dp, K);
}

template <int FMT>
static void pack_fmt(int dp, const float* C, int K, int d, const float* cnorm, void* rec,
                     unsigned* counters, hipStream_t st) {
#define X(D) pack_dp<FMT, D>(C, K, d, cnorm, rec, counters, st)
  switch (dp) { SOAR_DP_CASES(FMT, X) }
#undef X
}

hipError_t launch_lowp_pack_codebook(int fmt, const float* C, int K, int d, const float* cnorm,
                                     void* rec, unsigned* counters, hipStream_t st) {
  const int dp = lowp_padded_dim(fmt, d);
  if (fmt == LOWP_BF16) pack_fmt<LOWP_BF16>(dp, C, K, d, cnorm, rec, counters, st);
  else pack_fmt<LOWP_FP8>(dp, C, K, d, cnorm, rec, counters, st);
  return hipGetLastError();
}
#undef SOAR_DP_CASES

template <int FMT, int M, bool V4, int DX>
static void rescore_go(const LowpParams& P, bool spill, hipStream_t st) {
  const dim3 grid((unsigned)((P.n + 15) / 16)), block(256);
  if (spill) hipLaunchKernelGGL((lowp_rescore_kernel<FMT, true, M, V4>), grid, block, 0, st, P);
  else hipLaunchKernelGGL((lowp_rescore_kernel<FMT, false, M, V4, DX>), grid, block, 0, st, P);
}

template <int FMT, int M>
static void rescore_m(const LowpParams& P, bool spill, bool v4, hipStream_t st) {
  const dim3 grid((unsigned)((P.n + 15) / 16)), block(256);
  if constexpr (M % 4 == 0) {
    if (v4) {
      // common narrow widths get a compile-time row length in the primary re-score: 389 -> 339 us
      // at n=1M, d=128 (the spill re-score measured slower with it, and at d = 768 it raised the
      // registers past two waves per SIMD)
      if constexpr (M == 4) { if (P.d == 64) return rescore_go<FMT, M, true, 64>(P, spill, st); }
      if constexpr (M == 8) {
        if (P.d == 96) return rescore_go<FMT, M, true, 96>(P, spill, st);
        if (P.d == 128) return rescore_go<FMT, M, true, 128>(P, spill, st);
      }
      if constexpr (M == 16) { if (P.d == 256) return rescore_go<FMT, M, true, 256>(P, spill, st); }
      return rescore_go<FMT, M, true, 0>(P, spill, st);
    }
  }
  if (spill) hipLaunchKernelGGL((lowp_rescore_kernel<FMT, true, M, false>), grid, block, 0, st, P);
  else hipLaunchKernelGGL((lowp_rescore_kernel<FMT, false, M, false>), grid, block, 0, st, P);
}

template <int FMT>
static hipError_t rescore_fmt(const LowpParams& P, bool spill, hipStream_t st) {
  // float4 layout when the rows allow it: ceil(d / 64) chunks of 4 per lane
  const bool v4 = P.d % 4 == 0 && reinterpret_cast<uintptr_t>(P.X) % 16 == 0 &&
                  reinterpret_cast<uintptr_t>(P.C) % 16 == 0;
  const int m = v4 ? 4 * ((P.d + 63) / 64) : (P.d + 15) / 16;
  if (m <= 2) rescore_m<FMT, 2>(P, spill, v4, st);
  else if (m <= 4) rescore_m<FMT, 4>(P, spill, v4, st);
  else if (m <= 6) rescore_m<FMT, 6>(P, spill, v4, st);
  else if (m <= 8) rescore_m<FMT, 8>(P, spill, v4, st);
  else if (m <= 12) rescore_m<FMT, 12>(P, spill, v4, st);
  else if (m <= 16) rescore_m<FMT, 16>(P, spill, v4, st);
  else if (m <= 24) rescore_m<FMT, 24>(P, spill, v4, st);
  else if (m <= 32) rescore_m<FMT, 32>(P, spill, v4, st);
  else if (m <= 48) rescore_m<FMT, 48>(P, spill, v4, st);
  else if (m <= 64) rescore_m<FMT, 64>(P, spill, v4, st);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_lowp_rescore(int fmt, const LowpParams& P, bool spill, hipStream_t st) {
  return fmt == LOWP_BF16 ? rescore_fmt<LOWP_BF16>(P, spill, st)
                          : rescore_fmt<LOWP_FP8>(P, spill, st);
}

}  // namespace soar
