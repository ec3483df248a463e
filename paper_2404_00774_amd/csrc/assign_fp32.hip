// FP32 SOAR assignment on gfx950: primary (Section 2.2) and spill (Section 3.4, Eq. 2 via
// Theorem 3.1) for a block of rows in one kernel.
//
// Layout of the work.  A workgroup of 4 waves owns 64 consecutive rows (16 per wave).  Each wave
// keeps its 16 rows of X -- and, for the spill, of R = X - C[pi] -- resident in VGPRs in the
// A-operand layout of v_mfma_f32_16x16x4_f32, and the workgroup streams the codebook through
// double-buffered LDS tiles of BN centroids.  The contraction dimension is permuted so that lane
// group q = lane/16 holds the contiguous quarter [q*DP/4, (q+1)*DP/4) of every row: at MFMA step
// s lane (q, i) supplies X[i][q*DP/4 + s] and C[j][q*DP/4 + s], so both operands load as float4.
//
// Exactness.  The tile epilogue ranks centroids by the expanded value (constants of the row
// dropped)
//     primary: ||c||^2 - 2<x,c>
//     spill:   ||c||^2 - 2<x,c> + lambda/||r||^2 * (<r,c> - <r,x>)^2,  masked at j = pi
// and every lane keeps, per row, its two best values with their indices and its third-best value
// over the columns it sees.  With delta a proven bound on the expansion's rounding error, every
// centroid whose value lies within 2*delta of the row minimum is a candidate for the exact
// arg-min; the lanes' two bests cover all of them unless some lane's third best is itself inside
// that band, in which case the row is handed to the exact full scan.  Candidates are re-scored by direct differences
// in FP32 (16 partial sums per row), and candidates within the near-tie gap of the best are
// re-decided in FP64.  Ties go to the lowest index.
#include "common.h"
#include "kernels.h"

namespace soar {

template <int KS, bool VEC>
__device__ __forceinline__ void load_quarter(const float* __restrict__ base, int64_t row, int d,
                                             int q, bool ok, float (&v)[KS]) {
  const int k0 = q * KS;
  const float* p = base + row * (int64_t)d + k0;
  if constexpr (VEC) {
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      v4f t = {0.f, 0.f, 0.f, 0.f};
      if (ok && k0 + s < d) t = *reinterpret_cast<const v4f*>(p + s);
      v[s] = t.x; v[s + 1] = t.y; v[s + 2] = t.z; v[s + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int s = 0; s < KS; ++s) v[s] = (ok && k0 + s < d) ? p[s] : 0.f;
  }
}

// Direct ||x - c_j||^2 (and <r, x - c_j>) over this lane's quarter, 4 partial sums per lane.
template <int KS, bool VEC, bool SP>
__device__ __forceinline__ void direct32(const float* __restrict__ C, int d, int j, int q,
                                         const float (&xa)[KS], const float (&ra)[KS], float& sq,
                                         float& pj) {
  float c[KS];
  load_quarter<KS, VEC>(C, j, d, q, true, c);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
  for (int s = 0; s < KS; s += 4) {
    const float e0 = xa[s] - c[s], e1 = xa[s + 1] - c[s + 1];
    const float e2 = xa[s + 2] - c[s + 2], e3 = xa[s + 3] - c[s + 3];
    s0 = fmaf(e0, e0, s0); s1 = fmaf(e1, e1, s1); s2 = fmaf(e2, e2, s2); s3 = fmaf(e3, e3, s3);
    if constexpr (SP) {
      p0 = fmaf(ra[s], e0, p0); p1 = fmaf(ra[s + 1], e1, p1);
      p2 = fmaf(ra[s + 2], e2, p2); p3 = fmaf(ra[s + 3], e3, p3);
    }
  }
  sq = sum_quad_f((s0 + s1) + (s2 + s3));
  pj = SP ? sum_quad_f((p0 + p1) + (p2 + p3)) : 0.f;
}

// The same in FP64 with the residual formed exactly from C[pi] (near-tie decisions only).
template <int KS, bool VEC, bool SP>
__device__ __forceinline__ double direct64(const float* __restrict__ C, int d, int j, int pi,
                                           int q, const float (&xa)[KS], float lam) {
  float c[KS], cp[KS];
  load_quarter<KS, VEC>(C, j, d, q, true, c);
  if constexpr (SP) load_quarter<KS, VEC>(C, pi, d, q, true, cp);
  double sq0 = 0.0, sq1 = 0.0, pj0 = 0.0, pj1 = 0.0, rr0 = 0.0, rr1 = 0.0;
#pragma unroll
  for (int s = 0; s < KS; s += 2) {
    const double e0 = (double)xa[s] - (double)c[s], e1 = (double)xa[s + 1] - (double)c[s + 1];
    sq0 = fma(e0, e0, sq0); sq1 = fma(e1, e1, sq1);
    if constexpr (SP) {
      const double r0 = (double)xa[s] - (double)cp[s], r1 = (double)xa[s + 1] - (double)cp[s + 1];
      pj0 = fma(r0, e0, pj0); pj1 = fma(r1, e1, pj1);
      rr0 = fma(r0, r0, rr0); rr1 = fma(r1, r1, rr1);
    }
  }
  const double sq = sum_quad_d(sq0 + sq1);
  if constexpr (!SP) return sq;
  const double pj = sum_quad_d(pj0 + pj1);
  const double rr = sum_quad_d(rr0 + rr1);
  return rr > 0.0 ? sq + (double)lam * (pj * pj) / rr : sq;
}

template <int DP, int BN, bool VEC>
struct TileLoader {
  static constexpr int KS = DP / 4;
  static constexpr int LDW = DP + 4;
  static constexpr int F4_PER_ROW = DP / 4;
  static constexpr int NLD = (BN * DP / 4) / 256;
  static_assert((BN * DP / 4) % 256 == 0, "tile must split evenly over 256 threads");
  v4f reg[NLD];
  float cn;

  __device__ __forceinline__ void load(const float* __restrict__ C, const float* __restrict__ cnorm,
                                       int K, int d, int t, int tid) {
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int f = tid + i * 256;
      const int row = f / F4_PER_ROW, k = (f % F4_PER_ROW) * 4;
      const int j = t * BN + row;
      v4f v = {0.f, 0.f, 0.f, 0.f};
      if (j < K) {
        const float* p = C + (int64_t)j * d + k;
        if constexpr (VEC) {
          if (k < d) v = *reinterpret_cast<const v4f*>(p);
        } else {
          if (k + 0 < d) v.x = p[0];
          if (k + 1 < d) v.y = p[1];
          if (k + 2 < d) v.z = p[2];
          if (k + 3 < d) v.w = p[3];
        }
      }
      reg[i] = v;
    }
    if (tid < BN) cn = (t * BN + tid < K) ? cnorm[t * BN + tid] : kInf;
  }
  __device__ __forceinline__ void store(float* s_c, float* s_cn, int tid) const {
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int f = tid + i * 256;
      const int row = f / F4_PER_ROW, k = (f % F4_PER_ROW) * 4;
      *reinterpret_cast<v4f*>(s_c + row * LDW + k) = reg[i];
    }
    if (tid < BN) s_cn[tid] = cn;
  }
};

// One sweep over all K centroids for the wave's 16 rows.  Output-layout lane (q, c16) sees rows
// 4q+v (v = 0..3) at column c16 of every 16-column block.
template <int DP, int BN, bool VEC, bool SP>
__device__ __forceinline__ void sweep(const AssignParams& P, float* s_c, float* s_cn, int tid,
                                      const float (&xa)[DP / 4], const float (&ra)[DP / 4],
                                      const float (&lp)[4], const float (&av)[4],
                                      const int (&pr)[4], float (&b1)[4], int (&i1)[4],
                                      float (&b2)[4], int (&i2)[4], float (&b3)[4]) {
  constexpr int KS = DP / 4, LDW = DP + 4, NB = BN / 16;
  const int lane = tid & 63, q = lane >> 4, c16 = lane & 15;
  const int ntiles = (P.K + BN - 1) / BN;
  TileLoader<DP, BN, VEC> ld;
  ld.load(P.C, P.cnorm, P.K, P.d, 0, tid);
  ld.store(s_c, s_cn, tid);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    const int buf = t & 1;
    const float* sb = s_c + buf * (BN * LDW);
    if (t + 1 < ntiles) ld.load(P.C, P.cnorm, P.K, P.d, t + 1, tid);
    v4f accS[NB], accT[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      accS[b] = v4f{0.f, 0.f, 0.f, 0.f};
      accT[b] = v4f{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      v4f bv[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b)
        bv[b] = *reinterpret_cast<const v4f*>(sb + (b * 16 + c16) * LDW + q * KS + s);
      // consecutive MFMAs write different accumulators so none waits on the one before
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          accS[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[s + e], bv[b][e], accS[b], 0, 0, 0);
          if constexpr (SP)
            accT[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[s + e], bv[b][e], accT[b], 0, 0, 0);
        }
      }
    }
    const float* scn = s_cn + buf * BN;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = t * BN + b * 16 + c16;
      const float cn = scn[b * 16 + c16];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float val;
        if constexpr (SP) {
          const float e = accT[b][v] - av[v];
          const float w = fmaf(-2.f, accS[b][v], cn);
          val = fmaf(lp[v] * e, e, w);
          if (j == pr[v]) val = kInf;
        } else {
          val = fmaf(-2.f, accS[b][v], cn);
        }
        // keep (b1, i1) <= (b2, i2) <= b3 over the columns seen so far
        const bool lt1 = val < b1[v], lt2 = val < b2[v];
        b3[v] = fminf(b3[v], fmaxf(b2[v], val));
        i2[v] = lt1 ? i1[v] : (lt2 ? j : i2[v]);
        b2[v] = fminf(b2[v], fmaxf(b1[v], val));
        i1[v] = lt1 ? j : i1[v];
        b1[v] = fminf(b1[v], val);
      }
    }
    if (t + 1 < ntiles) ld.store(s_c + (buf ^ 1) * (BN * LDW), s_cn + (buf ^ 1) * BN, tid);
    __syncthreads();
  }
}

struct RowShared {
  float band[4][16];   // per wave, per row: 2*delta for the current pass
  float lp[4][16];     // lambda / ||r||^2 (0 when r = 0)
  float av[4][16];     // <r, x>
  int pi[4][16];       // primary (-1: the row went to the full scan)
  int nc[4][16];       // number of candidates
  int sat[4][16];      // candidate set not proven complete
  int cand[4][16][32];
  float cv[4][16][32];
};

// Reduce the lane-level state to per-row candidate lists in LDS (output layout -> LDS).
__device__ __forceinline__ void publish_candidates(RowShared& S, int w, int lane,
                                                   const float (&b1)[4], const int (&i1)[4],
                                                   const float (&b2)[4], const int (&i2)[4],
                                                   const float (&b3)[4]) {
  const int q = lane >> 4, c16 = lane & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * q + v;
    float m = b1[v];
    int mj = i1[v];
    argmin16(m, mj);
    const float thr = m + S.band[w][r];
    const bool finite_min = m < kInf;
    const bool sat = b3[v] <= thr;
    const bool c1 = finite_min && b1[v] <= thr;
    const bool c2 = finite_min && b2[v] <= thr;   // implies c1
    const unsigned sg = (unsigned)(__ballot(sat) >> (16 * q)) & 0xFFFFu;
    const unsigned g1 = (unsigned)(__ballot(c1) >> (16 * q)) & 0xFFFFu;
    const unsigned g2 = (unsigned)(__ballot(c2) >> (16 * q)) & 0xFFFFu;
    if (c16 == 0) {
      // no proven-complete, non-empty candidate set (also covers a NaN band): exact full scan
      S.sat[w][r] = (sg != 0u) || !finite_min || g1 == 0u;
      S.nc[w][r] = __popc(g1) + __popc(g2);
    }
    const unsigned below = (1u << c16) - 1u;
    const int pos = __popc(g1 & below) + __popc(g2 & below);
    if (c1) S.cand[w][r][pos] = i1[v];
    if (c2) S.cand[w][r][pos + 1] = i2[v];
  }
}

// Exact decision among a row's candidates (A layout: lane (q, c16) holds row c16's quarter q).
template <int KS, bool VEC, bool SP>
__device__ __forceinline__ void decide(const AssignParams& P, RowShared& S, int w, int c16, int q,
                                       const float (&xa)[KS], const float (&ra)[KS], float rr,
                                       int pi, int& best_j, float& best_v) {
  const int nc = S.nc[w][c16];
  float best = kInf;
  int bj = 0x7fffffff;
  for (int k = 0; k < nc; ++k) {
    const int j = S.cand[w][c16][k];
    float sq, pj;
    direct32<KS, VEC, SP>(P.C, P.d, j, q, xa, ra, sq, pj);
    const float val = (SP && rr > 0.f) ? sq + P.lam * (pj * pj) / rr : sq;
    S.cv[w][c16][k] = val;
    if (val < best || (val == best && j < bj)) { best = val; bj = j; }
  }
  const float lim = best + best * P.tie_rel;
  int ntie = 0;
  for (int k = 0; k < nc; ++k) ntie += S.cv[w][c16][k] <= lim;
  if (ntie >= 2) {
    double bd = __builtin_inf();
    int bdj = 0x7fffffff;
    for (int k = 0; k < nc; ++k) {
      if (S.cv[w][c16][k] <= lim) {
        const int j = S.cand[w][c16][k];
        argmin_d(bd, bdj, direct64<KS, VEC, SP>(P.C, P.d, j, pi, q, xa, P.lam), j);
      }
    }
    best = (float)bd;
    bj = bdj;
    if (q == 0) atomicAdd(&P.counters[CNT_FP64], 1u);
  }
  best_j = bj;
  best_v = best;
}

template <int DP, int BN, bool SPILL, bool VEC>
__global__ __launch_bounds__(256) void assign_f32_kernel(AssignParams P) {
  constexpr int KS = DP / 4, LDW = DP + 4;
  __shared__ __attribute__((aligned(16))) float s_c[2 * BN * LDW];
  __shared__ float s_cn[2 * BN];
  __shared__ RowShared S;

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, q = lane >> 4, c16 = lane & 15;
  const int64_t n = live_rows(P.n, P.live_n);
  if ((int64_t)blockIdx.x * 64 >= n) return;   // whole block past the live rows
  const int64_t row = (int64_t)blockIdx.x * 64 + w * 16 + c16;  // A-layout row of this lane
  const bool ok = row < n;
  const float cmax = sqrtf(__uint_as_float(P.counters[CNT_CMAX2]));

  float xa[KS], ra[KS];
  load_quarter<KS, VEC>(P.X, row, P.d, q, ok, xa);
  bool fin = true;
  float n0 = 0.f, n1 = 0.f, n2 = 0.f, n3 = 0.f;
#pragma unroll
  for (int s = 0; s < KS; s += 4) {
    fin = fin && all_finite4(v4f{xa[s], xa[s + 1], xa[s + 2], xa[s + 3]});
    n0 = fmaf(xa[s], xa[s], n0); n1 = fmaf(xa[s + 1], xa[s + 1], n1);
    n2 = fmaf(xa[s + 2], xa[s + 2], n2); n3 = fmaf(xa[s + 3], xa[s + 3], n3);
    ra[s] = ra[s + 1] = ra[s + 2] = ra[s + 3] = 0.f;
  }
  if (!fin) atomicOr(&P.counters[CNT_NONFINITE], 1u);
  const float xnorm = sqrtf(sum_quad_f((n0 + n1) + (n2 + n3)));
  const float scale2 = (xnorm + cmax) * (xnorm + cmax);
  if (q == 0) S.band[w][c16] = P.band_p * scale2;
  __syncthreads();

  // ---------------- primary pass ----------------
  float b1[4], b2[4], b3[4], lp[4], av[4];
  int i1[4], i2[4], pr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    b1[v] = b2[v] = b3[v] = kInf; i1[v] = i2[v] = 0x7fffffff;
    lp[v] = av[v] = 0.f; pr[v] = -1;
  }
  sweep<DP, BN, VEC, false>(P, s_c, s_cn, tid, xa, ra, lp, av, pr, b1, i1, b2, i2, b3);
  publish_candidates(S, w, lane, b1, i1, b2, i2, b3);
  __syncthreads();

  int pi = -1;
  float pdist = 0.f;
  bool psat = S.sat[w][c16] != 0;
  if (!psat) decide<KS, VEC, false>(P, S, w, c16, q, xa, ra, 0.f, 0, pi, pdist);
  if (pi < 0 || pi >= P.K) psat = true;
  if (ok && q == 0) {
    if (psat) {
      const unsigned slot = atomicAdd(&P.counters[CNT_FULLSCAN], 1u);
      P.full_rows[slot] = (int32_t)row;
    } else {
      P.primary[row] = pi;
      if (P.pdist) P.pdist[row] = pdist;
    }
  }
  if constexpr (!SPILL) return;

  // ---------------- residual ----------------
  if (psat) pi = -1;
  float rr = 0.f, a = 0.f;
  if (pi >= 0) {
    float cp[KS];
    load_quarter<KS, VEC>(P.C, pi, P.d, q, true, cp);
    float r0 = 0.f, r1 = 0.f, r2 = 0.f, r3 = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      ra[s] = xa[s] - cp[s]; ra[s + 1] = xa[s + 1] - cp[s + 1];
      ra[s + 2] = xa[s + 2] - cp[s + 2]; ra[s + 3] = xa[s + 3] - cp[s + 3];
      r0 = fmaf(ra[s], ra[s], r0); r1 = fmaf(ra[s + 1], ra[s + 1], r1);
      r2 = fmaf(ra[s + 2], ra[s + 2], r2); r3 = fmaf(ra[s + 3], ra[s + 3], r3);
      a0 = fmaf(ra[s], xa[s], a0); a1 = fmaf(ra[s + 1], xa[s + 1], a1);
      a2 = fmaf(ra[s + 2], xa[s + 2], a2); a3 = fmaf(ra[s + 3], xa[s + 3], a3);
    }
    rr = sum_quad_f((r0 + r1) + (r2 + r3));
    a = sum_quad_f((a0 + a1) + (a2 + a3));
  }
  if (q == 0) {
    S.pi[w][c16] = pi;
    S.lp[w][c16] = rr > 0.f ? P.lam / rr : 0.f;
    S.av[w][c16] = a;
    S.band[w][c16] = P.band_s * scale2;
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * q + v;
    lp[v] = S.lp[w][r]; av[v] = S.av[w][r]; pr[v] = S.pi[w][r];
    b1[v] = b2[v] = b3[v] = kInf; i1[v] = i2[v] = 0x7fffffff;
  }

  // ---------------- spill pass ----------------
  sweep<DP, BN, VEC, true>(P, s_c, s_cn, tid, xa, ra, lp, av, pr, b1, i1, b2, i2, b3);
  publish_candidates(S, w, lane, b1, i1, b2, i2, b3);
  __syncthreads();
  if (pi < 0) return;  // full-scan rows are finished by the full-scan kernel
  bool ssat = S.sat[w][c16] != 0;
  int sj = -1;
  float sl = 0.f;
  if (!ssat) decide<KS, VEC, true>(P, S, w, c16, q, xa, ra, rr, pi, sj, sl);
  if (sj < 0 || sj >= P.K) ssat = true;
  if (ok && q == 0) {
    if (ssat) {
      const unsigned slot = atomicAdd(&P.counters[CNT_FULLSCAN], 1u);
      P.full_rows[slot] = (int32_t)row;
    } else {
      P.spill[row] = sj;
      if (P.sloss) P.sloss[row] = sl;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Exact full scan over all K for the rows listed by the assignment kernel (one workgroup a row).
// Each wave takes one centroid at a time with its lanes across the dimensions (coalesced loads),
// and a 64-lane tree gives the sum (at most 4 sequential terms per lane for d <= 256).
// ------------------------------------------------------------------------------------------------
constexpr int FS_THREADS = 256;
constexpr int FS_WAVES = FS_THREADS / 64;

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// FP32 value of centroid j for this row: ||x - c||^2, or the SOAR loss given r and ||r||^2.
template <bool SP>
__device__ __forceinline__ float fs_value32(const float* __restrict__ c, const float* sx,
                                            const float* sr, float rr, float lam, int d, int lane) {
  float sq = 0.f, pj = 0.f;
  for (int k = lane; k < d; k += 64) {
    const float e = sx[k] - c[k];
    sq = fmaf(e, e, sq);
    if (SP) pj = fmaf(sr[k], e, pj);
  }
  sq = wave_sum_f(sq);
  if (!SP) return sq;
  pj = wave_sum_f(pj);
  return rr > 0.f ? sq + lam * (pj * pj) / rr : sq;
}

// FP64 value with the residual formed exactly from C[pi] (near-tie decisions).
template <bool SP>
__device__ __forceinline__ double fs_value64(const float* __restrict__ c, const float* sx,
                                             const float* scp, float lam, int d, int lane) {
  double sq = 0.0, pj = 0.0, rr = 0.0;
  for (int k = lane; k < d; k += 64) {
    const double e = (double)sx[k] - (double)c[k];
    sq = fma(e, e, sq);
    if (SP) {
      const double rk = (double)sx[k] - (double)scp[k];
      pj = fma(rk, e, pj);
      rr = fma(rk, rk, rr);
    }
  }
  sq = wave_sum_d(sq);
  if (!SP) return sq;
  pj = wave_sum_d(pj);
  rr = wave_sum_d(rr);
  return rr > 0.0 ? sq + (double)lam * (pj * pj) / rr : sq;
}

template <typename T>
__device__ __forceinline__ void wg_argmin(T& v, int& j, T* sv, int* sj) {
  const int tid = threadIdx.x, w = tid >> 6;
  if ((tid & 63) == 0) { sv[w] = v; sj[w] = j; }
  __syncthreads();
  if (tid == 0) {
    for (int i = 1; i < FS_WAVES; ++i)
      if (sv[i] < sv[0] || (sv[i] == sv[0] && sj[i] < sj[0])) { sv[0] = sv[i]; sj[0] = sj[i]; }
  }
  __syncthreads();
  v = sv[0];
  j = sj[0];
  __syncthreads();
}

// Exact arg-min over all columns j != skip; FP32 direct values, then FP64 among near-ties.
template <bool SP>
__device__ void fs_argmin(const AssignParams& P, const float* sx, const float* sr, float rr,
                          const float* scp, int skip, int& out_j, float& out_v) {
  __shared__ float rv[FS_WAVES];
  __shared__ int rj[FS_WAVES];
  __shared__ double rd[FS_WAVES];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, K = P.K, d = P.d;
  float bv = kInf;
  int bj = 0x7fffffff;
  for (int j = w; j < K; j += FS_WAVES) {
    if (j == skip) continue;
    const float v = fs_value32<SP>(P.C + (int64_t)j * d, sx, sr, rr, P.lam, d, lane);
    if (v < bv) { bv = v; bj = j; }
  }
  wg_argmin<float>(bv, bj, rv, rj);
  if (!(bv < kInf)) { out_j = -1; out_v = kInf; return; }
  const float lim = bv + bv * P.tie_rel;
  double dv = __builtin_inf();
  int dj = 0x7fffffff;
  for (int j = w; j < K; j += FS_WAVES) {
    if (j == skip) continue;
    const float* c = P.C + (int64_t)j * d;
    const float v = fs_value32<SP>(c, sx, sr, rr, P.lam, d, lane);
    if (v <= lim) argmin_d(dv, dj, fs_value64<SP>(c, sx, scp, P.lam, d, lane), j);
  }
  wg_argmin<double>(dv, dj, rd, rj);
  out_j = dj;
  out_v = (float)dv;
}

template <bool SPILL>
__global__ __launch_bounds__(FS_THREADS) void full_scan_kernel(AssignParams P) {
  extern __shared__ float fs_smem[];
  float* sx = fs_smem;
  float* sr = fs_smem + P.d;
  float* scp = fs_smem + 2 * P.d;
  __shared__ float s_rr;
  const unsigned count = P.counters[CNT_FULLSCAN];
  const int d = P.d, tid = threadIdx.x, lane = tid & 63;
  for (unsigned e = blockIdx.x; e < count; e += gridDim.x) {
    const int64_t row = P.full_rows[e];
    for (int k = tid; k < d; k += FS_THREADS) sx[k] = P.X[row * d + k];
    __syncthreads();
    int pi;
    float pd;
    fs_argmin<false>(P, sx, sr, 0.f, scp, -1, pi, pd);
    if (pi >= P.K) pi = -1;
    if (tid == 0) {
      P.primary[row] = pi;
      if (P.pdist) P.pdist[row] = pd;
      atomicAdd(&P.counters[CNT_FP64], 1u);
    }
    if (SPILL) {
      if (pi >= 0)
        for (int k = tid; k < d; k += FS_THREADS) {
          const float c = P.C[(int64_t)pi * d + k];
          scp[k] = c;
          sr[k] = sx[k] - c;
        }
      __syncthreads();
      if (tid < 64) {
        float a = 0.f;
        for (int k = lane; k < d; k += 64) a = fmaf(sr[k], sr[k], a);
        a = wave_sum_f(a);
        if (tid == 0) s_rr = a;
      }
      __syncthreads();
      int sj = -1;
      float sl = kInf;
      if (pi >= 0) {
        fs_argmin<true>(P, sx, sr, s_rr, scp, pi, sj, sl);
        if (sj >= P.K) sj = -1;
      }
      if (tid == 0) {
        P.spill[row] = sj;
        if (P.sloss) P.sloss[row] = sl;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------------
// Codebook preparation: ||c_j||^2, max ||c||^2 and the finiteness flag; counter reset.
// ------------------------------------------------------------------------------------------------
__global__ void reset_counters_kernel(unsigned* counters, int words) {
  if ((int)threadIdx.x < words) counters[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void prep_codebook_kernel(const float* __restrict__ C, int K,
                                                            int d, float* __restrict__ cnorm,
                                                            unsigned* counters) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0.f;
  bool fin = true;
  if (j < K) {
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    const float* c = C + (int64_t)j * d;
    int k = 0;
    for (; k + 4 <= d; k += 4) {
      const float v0 = c[k], v1 = c[k + 1], v2 = c[k + 2], v3 = c[k + 3];
      fin = fin && all_finite4(v4f{v0, v1, v2, v3});
      a0 = fmaf(v0, v0, a0); a1 = fmaf(v1, v1, a1); a2 = fmaf(v2, v2, a2); a3 = fmaf(v3, v3, a3);
    }
    for (; k < d; ++k) { fin = fin && __builtin_isfinite(c[k]); a0 = fmaf(c[k], c[k], a0); }
    s = (a0 + a1) + (a2 + a3);
    cnorm[j] = s;
  }
  if (!__builtin_isfinite(s)) { fin = false; s = 0.f; }
  unsigned m = __float_as_uint(s);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off));
  const uint64_t bad = __ballot(!fin);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&counters[CNT_CMAX2], m);
    if (bad) atomicOr(&counters[CNT_NONFINITE], 1u);
  }
}

// ------------------------------------------------------------------------------------------------
// Host-side launchers
// ------------------------------------------------------------------------------------------------
template <int DP, int BN>
static hipError_t launch_dp(const AssignParams& P, bool spill, bool vec, hipStream_t st) {
  const dim3 grid((unsigned)((P.n + 63) / 64)), block(256);
  if (spill) {
    if (vec) hipLaunchKernelGGL((assign_f32_kernel<DP, BN, true, true>), grid, block, 0, st, P);
    else hipLaunchKernelGGL((assign_f32_kernel<DP, BN, true, false>), grid, block, 0, st, P);
  } else {
    if (vec) hipLaunchKernelGGL((assign_f32_kernel<DP, BN, false, true>), grid, block, 0, st, P);
    else hipLaunchKernelGGL((assign_f32_kernel<DP, BN, false, false>), grid, block, 0, st, P);
  }
  return hipGetLastError();
}

int fp32_padded_dim(int d) {
  static const int dps[] = {16, 32, 48, 64, 96, 128, 192, 256};
  for (int dp : dps)
    if (d <= dp) return dp;
  return -1;
}

hipError_t launch_prep_codebook(const float* C, int K, int d, float* cnorm, unsigned* counters,
                                hipStream_t st) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, counters, (int)CNT_WORDS);
  hipLaunchKernelGGL(prep_codebook_kernel, dim3((K + 255) / 256), dim3(256), 0, st, C, K, d,
                     cnorm, counters);
  return hipGetLastError();
}

hipError_t launch_reset_step_counters(unsigned* counters, hipStream_t st) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, counters,
                     (int)CNT_STEP_WORDS);
  return hipGetLastError();
}

hipError_t launch_assign_fp32(const AssignParams& P, bool spill, bool vec, hipStream_t st,
                              hipEvent_t ev_begin, hipEvent_t ev_end) {
  hipError_t e;
  if (ev_begin) (void)hipEventRecord(ev_begin, st);
  switch (fp32_padded_dim(P.d)) {
    case 16: e = launch_dp<16, 64>(P, spill, vec, st); break;
    case 32: e = launch_dp<32, 64>(P, spill, vec, st); break;
    case 48: e = launch_dp<48, 64>(P, spill, vec, st); break;
    case 64: e = launch_dp<64, 64>(P, spill, vec, st); break;
    case 96: e = launch_dp<96, 64>(P, spill, vec, st); break;
    case 128: e = launch_dp<128, 64>(P, spill, vec, st); break;
    case 192: e = launch_dp<192, 32>(P, spill, vec, st); break;
    case 256: e = launch_dp<256, 32>(P, spill, vec, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (ev_end) (void)hipEventRecord(ev_end, st);
  const size_t smem = (size_t)3 * P.d * sizeof(float);
  if (spill)
    hipLaunchKernelGGL(full_scan_kernel<true>, dim3(1024), dim3(FS_THREADS), smem, st, P);
  else
    hipLaunchKernelGGL(full_scan_kernel<false>, dim3(1024), dim3(FS_THREADS), smem, st, P);
  return hipGetLastError();
}

}  // namespace soar
