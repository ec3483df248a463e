// FP32 SOAR assignment on gfx950: primary (Section 2.2) and spill (Section 3.4, Eq. 2 via
// Theorem 3.1) for a block of rows in one kernel.
//
// Layout of the work.  A workgroup of 4 waves owns 64 consecutive rows (16 per wave).  Each wave
// keeps its 16 rows of X -- and, for the spill, of R = X - C[pi] -- in VGPRs in the A-operand
// layout of v_mfma_f32_16x16x4_f32, and the workgroup streams the codebook through a two-stage
// LDS ring filled by direct global->LDS copies of packed tile records (no register staging).
// The contraction dimension is permuted so that lane group q = lane/16 holds the contiguous
// quarter [q*DP/4, (q+1)*DP/4) of every row: at MFMA step s lane (q, i) supplies X[i][q*DP/4 + s]
// and C[j][q*DP/4 + s], so both operands load as float4.  Rows longer than 256 are cut into
// chunks of DP = 128: the ring then carries one (tile, chunk) record per step, the accumulators
// run across the chunks of a tile, and each wave reloads its rows' chunk from L2 one step ahead.
//
// Exactness.  The tile epilogue ranks centroids by the expanded value (constants of the row
// dropped)
//     primary: ||c||^2 - 2<x,c>
//     spill:   ||c||^2 - 2<x,c> + lambda/||r||^2 * (<r,c> - <r,x>)^2,  masked at j = pi
// With delta_j = A_row (||x|| + ||c_j||)^2 a proven bound on the rounding error of centroid j's
// expanded value v_j (A_row from d, lambda and, in the Gram form, ||x|| + ||c_pi|| and ||r||),
// lo_j = v_j - delta_j and hi_j = v_j + delta_j bracket the exact value, so the exact arg-min has
// lo_j <= U for any upper end U = hi_k.  Every lane keeps, per row, the two smallest lo with their
// indices and the third smallest lo over the columns it sees; U is the smallest hi among the
// lanes' best entries.  The candidates are the tracked entries with lo <= U, and they are
// complete unless some lane's third smallest lo is also <= U, in which case the row is handed to
// the exact full scan.  (lo and U are kept shifted by the row constant A_row ||x||^2.)  Candidates are re-scored
// by direct differences in FP32 (16 partial sums per row), and candidates within the near-tie
// gap of the best are re-decided in FP64.  Ties go to the lowest index.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace soar {

// Packed codebook record of tile t (centroids [t*BN, t*BN + BN)) and chunk ch (dimensions
// [ch*DP, ch*DP + DP)), records ordered by (t, ch):
//   [BN rows of DP floats, row stride LDW = DP + 4 (the pad keeps the B-operand reads of the 16
//    lanes of a group on distinct banks); zeros past d and past K]
//   [BN floats ||c_j||^2, +inf past K]
//   [BN floats ||c_j||, 0 past K]
//   [BN floats ||c_j||^2 - A_p ||c_j||^2, +inf past K] (A_p: the primary pass's error
//    coefficient, so the primary's lower ends need one fma per column term)
// Each record is copied with NI whole wave-group copies (4 waves x 64 lanes x 16 bytes).
template <int DP, int BN>
struct F32Rec {
  static constexpr int LDW = DP + 4;
  static constexpr int CN_OFF = BN * LDW * 4;
  static constexpr int SN_OFF = CN_OFF + BN * 4;
  static constexpr int CA_OFF = SN_OFF + BN * 4;
  static constexpr int BYTES = CA_OFF + BN * 4;
  static constexpr int NI = (BYTES + 4095) / 4096;
  static constexpr int STAGE = NI * 4096;
};

template <int DP, int BN>
__device__ __forceinline__ const float* rec_row(const char* recs, int nch, int j, int ch) {
  using R = F32Rec<DP, BN>;
  return reinterpret_cast<const float*>(recs + ((int64_t)(j / BN) * nch + ch) * R::BYTES) +
         (j % BN) * R::LDW;
}

// KS consecutive values of row `row` of a row-major [* x d] matrix from column k0 (zeros past d
// and for rows that do not exist).
template <int KS, bool VEC>
__device__ __forceinline__ void load_seg(const float* __restrict__ base, int64_t row, int d,
                                         int k0, bool ok, float (&v)[KS]) {
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

// KS consecutive values of a record row (16-byte aligned, zero padded).
template <int KS>
__device__ __forceinline__ void load_rec(const float* p, float (&v)[KS]) {
#pragma unroll
  for (int s = 0; s < KS; s += 4) {
    const v4f t = *reinterpret_cast<const v4f*>(p + s);
    v[s] = t.x; v[s + 1] = t.y; v[s + 2] = t.z; v[s + 3] = t.w;
  }
}

// Direct ||x - c_j||^2 (and <r, x - c_j>) over this lane's share of the dimensions, 4 partial
// sums per lane; with CH the rows' chunks are read again from X and the record of C[pi].
template <int DP, int BN, bool CH, bool VEC, bool SP>
__device__ __forceinline__ void direct32(const AssignParams& P, int nch, int64_t row, bool ok,
                                         int pi, int j, int q, const float (&xa)[DP / 4],
                                         const float (&ra)[DP / 4], float& sq, float& pj) {
  constexpr int KS = DP / 4;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
  for (int ch = 0; ch < (CH ? nch : 1); ++ch) {
    float c[KS], xs[KS], rs[KS];
    load_rec<KS>(rec_row<DP, BN>(P.Crec, nch, j, ch) + q * KS, c);
    if constexpr (CH) {
      load_seg<KS, VEC>(P.X, row, P.d, ch * DP + q * KS, ok, xs);
      if constexpr (SP) {
        load_rec<KS>(rec_row<DP, BN>(P.Crec, nch, pi, ch) + q * KS, rs);
#pragma unroll
        for (int s = 0; s < KS; ++s) rs[s] = xs[s] - rs[s];
      }
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s) { xs[s] = xa[s]; rs[s] = ra[s]; }
    }
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      const float e0 = xs[s] - c[s], e1 = xs[s + 1] - c[s + 1];
      const float e2 = xs[s + 2] - c[s + 2], e3 = xs[s + 3] - c[s + 3];
      s0 = fmaf(e0, e0, s0); s1 = fmaf(e1, e1, s1); s2 = fmaf(e2, e2, s2); s3 = fmaf(e3, e3, s3);
      if constexpr (SP) {
        p0 = fmaf(rs[s], e0, p0); p1 = fmaf(rs[s + 1], e1, p1);
        p2 = fmaf(rs[s + 2], e2, p2); p3 = fmaf(rs[s + 3], e3, p3);
      }
    }
  }
  sq = sum_quad_f((s0 + s1) + (s2 + s3));
  pj = SP ? sum_quad_f((p0 + p1) + (p2 + p3)) : 0.f;
}

// The same in FP64 with the residual formed exactly from C[pi] (near-tie decisions only).  The
// rows are taken 8 values at a time (a rolled loop), which keeps this rare path's registers low.
template <int DP, int BN, bool CH, bool VEC, bool SP>
__device__ __forceinline__ double direct64(const AssignParams& P, int nch, int64_t row, bool ok,
                                           int pi, int j, int q, const float (&xa)[DP / 4]) {
  constexpr int KS = DP / 4;
  constexpr int G = KS % 8 == 0 ? 8 : 4;         // values per step (KS is a multiple of 4)
  double sq0 = 0.0, sq1 = 0.0, pj0 = 0.0, pj1 = 0.0, rr0 = 0.0, rr1 = 0.0;
  for (int ch = 0; ch < (CH ? nch : 1); ++ch) {
    const float* cj = rec_row<DP, BN>(P.Crec, nch, j, ch) + q * KS;
    // (pi indexes the whole codebook; under codebook splits P.Crec holds the split's tiles only)
    const float* cpi = rec_row<DP, BN>(P.Crec_all ? P.Crec_all : P.Crec, nch, pi, ch) + q * KS;
    float xs[CH ? KS : 1];
    if constexpr (CH) load_seg<KS, VEC>(P.X, row, P.d, ch * DP + q * KS, ok, xs);
#pragma unroll 1
    for (int s0 = 0; s0 < KS; s0 += G) {
      float c[G], cp[G], xg[G];
      load_rec<G>(cj + s0, c);
      if constexpr (SP) load_rec<G>(cpi + s0, cp);
#pragma unroll
      for (int s = 0; s < G; ++s) {
        // (a rolled loop cannot index the register arrays: select the values explicitly)
        float xv = 0.f;
#pragma unroll
        for (int k = 0; k < KS; k += G) xv = (k == s0) ? (CH ? xs[k + s] : xa[k + s]) : xv;
        xg[s] = xv;
      }
#pragma unroll
      for (int s = 0; s < G; s += 2) {
        const double e0 = (double)xg[s] - (double)c[s], e1 = (double)xg[s + 1] - (double)c[s + 1];
        sq0 = fma(e0, e0, sq0); sq1 = fma(e1, e1, sq1);
        if constexpr (SP) {
          const double r0 = (double)xg[s] - (double)cp[s];
          const double r1 = (double)xg[s + 1] - (double)cp[s + 1];
          pj0 = fma(r0, e0, pj0); pj1 = fma(r1, e1, pj1);
          rr0 = fma(r0, r0, rr0); rr1 = fma(r1, r1, rr1);
        }
      }
    }
  }
  const double sq = sum_quad_d(sq0 + sq1);
  if constexpr (!SP) return sq;
  const double pj = sum_quad_d(pj0 + pj1);
  const double rr = sum_quad_d(rr0 + rr1);
  return rr > 0.0 ? sq + (double)P.lam * (pj * pj) / rr : sq;
}

// One sweep over all K centroids for the wave's 16 rows.  Output-layout lane (q, c16) sees rows
// 4q+v (v = 0..3) at column c16 of every 16-column block.  A-layout lane (q, c16) holds row
// `row` (primary pia).  Ends with a workgroup barrier: the ring is free afterwards.
// GR (spill only): <r, c_j> comes from <x, c_j> - G[pi][j], one MFMA stream instead of two; the
// G values of tile t+1 are loaded during tile t.
template <int DP, int BN, bool CH, bool VEC, bool SP, bool GR = false, bool GP = false>
__device__ __forceinline__ void sweep(const AssignParams& P, char* ring, int nch, int tid,
                                      int64_t row, bool ok, int pia, float (&xa)[DP / 4],
                                      float (&ra)[DP / 4], const float (&lp)[4],
                                      const float (&av)[4], const int (&pr)[4],
                                      const float (&xv)[4], const float (&Av)[4], float (&b1)[4],
                                      int (&i1)[4], float (&b2)[4], int (&i2)[4],
                                      float (&b3)[4]) {
  using R = F32Rec<DP, BN>;
  constexpr int KS = DP / 4, LDW = R::LDW, NB = BN / 16;
  static_assert(!GR || (SP && !CH), "Gram form: spill sweep of resident rows only");
  static_assert(!GP || (SP && !GR), "grouped form: spill sweep only");
  const int lane = tid & 63, w = tid >> 6, q = lane >> 4, c16 = lane & 15;
  const int ntiles = (P.K + BN - 1) / BN;
  const int nsteps = ntiles * (CH ? nch : 1);
  const char* recs = P.Crec;
  // lower ends, shifted by A_row ||x||^2:
  //   lo' = v - A_row (||c||^2 + 2 ||x|| ||c||)    (primary: (||c||^2 - A ||c||^2) from the record)
  //   (the spill forms ||c||^2 as ||c|| ||c||: ||c|| is 0 past K, where ||c||^2 is +inf)
  float kx[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) kx[v] = SP ? 2.f * xv[v] : -2.f * Av[v] * xv[v];
  // grouped form: every row of the stripe has the primary pia, so only the tile holding it needs
  // the mask
  const int pia_tile = GP ? __builtin_amdgcn_readfirstlane(pia) / BN : -1;
  // Gram rows of the lane's output rows (row 0 stands in for rows without a primary)
  const float* grow[4];
  float gcur[GR ? NB : 1][4], gnxt[GR ? NB : 1][4];
  if constexpr (GR) {
#pragma unroll
    for (int v = 0; v < 4; ++v) grow[v] = P.G + (int64_t)(pr[v] >= 0 ? pr[v] : 0) * P.K;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = b * 16 + c16;
#pragma unroll
      for (int v = 0; v < 4; ++v) gcur[b][v] = j < P.K ? grow[v][j] : 0.f;
    }
  }
  // chunked rows: chunk 0 now, chunk u+1 during step u.  In the grouped form stripe row 15 is
  // the centroid c_pia, read from its record.
  float xn[CH ? KS : 1], cn[CH && SP && !GP ? KS : 1];
  auto load_x = [&](int ch, float(&v)[KS]) __attribute__((always_inline)) {
    if (GP && c16 == 15) load_rec<KS>(rec_row<DP, BN>(recs, nch, pia, ch) + q * KS, v);
    else load_seg<KS, VEC>(P.X, row, P.d, ch * DP + q * KS, ok, v);
  };
  if constexpr (CH) {
    load_x(0, xa);
    if constexpr (SP && !GP) {
      if (pia >= 0) {
        load_rec<KS>(rec_row<DP, BN>(recs, nch, pia, 0) + q * KS, cn);
#pragma unroll
        for (int s = 0; s < KS; ++s) ra[s] = xa[s] - cn[s];
      }
    }
  }
  issue_record<R::BYTES, R::STAGE, R::NI, 2>(recs, ring, 0, w, lane);
  v4f accS[NB], accT[NB];
  for (int u = 0; u < nsteps; ++u) {
    const int ch = CH ? u % nch : 0, t = CH ? u / nch : u;
    // record u has landed for this wave, then for every wave; every wave is also done reading
    // the stage refilled next (the one step u - 1 used)
    wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if constexpr (CH) {
      if (u + 1 < nsteps) {
        const int cnx = (u + 1) % nch;
        load_x(cnx, xn);
        if constexpr (SP && !GP) {
          if (pia >= 0) load_rec<KS>(rec_row<DP, BN>(recs, nch, pia, cnx) + q * KS, cn);
        }
      }
    }
    if (u + 1 < nsteps) issue_record<R::BYTES, R::STAGE, R::NI, 2>(recs, ring, u + 1, w, lane);
    if constexpr (GR) {
      if (u + 1 < nsteps) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int j = (t + 1) * BN + b * 16 + c16;
#pragma unroll
          for (int v = 0; v < 4; ++v) gnxt[b][v] = j < P.K ? grow[v][j] : 0.f;
        }
      }
    }
    const float* sb = reinterpret_cast<const float*>(ring + (u & 1) * R::STAGE);
    if (ch == 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        accS[b] = v4f{0.f, 0.f, 0.f, 0.f};
        accT[b] = v4f{0.f, 0.f, 0.f, 0.f};
      }
    }
    // B operands one step ahead: the reads of step s + 4 are in flight during the MFMAs of step s
    v4f bv[2][NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
      bv[0][b] = *reinterpret_cast<const v4f*>(sb + (b * 16 + c16) * LDW + q * KS);
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      const int cur = (s / 4) & 1;
      if (s + 4 < KS) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
          bv[cur ^ 1][b] =
              *reinterpret_cast<const v4f*>(sb + (b * 16 + c16) * LDW + q * KS + s + 4);
      }
      __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of this step's MFMAs
      // consecutive MFMAs write different accumulators so none waits on the one before
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          accS[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[s + e], bv[cur][b][e], accS[b], 0, 0,
                                                         0);
          if constexpr (SP && !GR && !GP)
            accT[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[s + e], bv[cur][b][e], accT[b], 0,
                                                           0, 0);
        }
      }
    }
    if (!CH || ch == nch - 1) {
      const float* scn = reinterpret_cast<const float*>(ring + (u & 1) * R::STAGE + R::CN_OFF);
      const float* ssn = reinterpret_cast<const float*>(ring + (u & 1) * R::STAGE + R::SN_OFF);
      const float* sca = reinterpret_cast<const float*>(ring + (u & 1) * R::STAGE + R::CA_OFF);
      auto epilogue = [&](auto with_mask) __attribute__((always_inline)) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int j = t * BN + b * 16 + c16;
          const float cnv = SP ? scn[b * 16 + c16] : sca[b * 16 + c16];
          const float snv = ssn[b * 16 + c16];
          // grouped form: row 15 of the stripe is the centroid c_p (lane group 3, register 3)
          const float spv = GP ? __shfl(accS[b][3], 48 + c16) : 0.f;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float val;
            if constexpr (SP) {
              // <r, c_j> - <r, x>: directly, as (<x, c_j> - G[pi][j]) - <r, x>, or with
              // <c_pi, c_j> from the stripe's centroid row
              const float e = GP ? (accS[b][v] - spv) - av[v]
                                 : (GR ? (accS[b][v] - gcur[b][v]) - av[v] : accT[b][v] - av[v]);
              const float wv = fmaf(-2.f, accS[b][v], cnv);
              val = fmaf(lp[v] * e, e, wv);
              if (decltype(with_mask)::value && j == pr[v]) val = kInf;
            } else {
              val = fmaf(-2.f, accS[b][v], cnv);   // here cnv = ||c||^2 - A ||c||^2
            }
            // the lower end (shifted), then (b1, i1) <= (b2, i2) <= b3 over the columns seen
            // (selects, not branches: the conditions differ from lane to lane).  With
            // b1 <= b2 <= b3, the new b3 is min(b3, max(b2, lo)) = med3(b2, lo, b3) and the
            // new b2 is med3(b1, lo, b2).  A NaN lo (med3 then takes the min of the other two,
            // as fminf/fmaxf would) pulls b3 down to b2, so the row reads as unscreened.
            const float lo = SP ? fmaf(-(Av[v] * (snv + kx[v])), snv, val) : fmaf(kx[v], snv, val);
            const bool lt1 = lo < b1[v], lt2 = lo < b2[v];
            b3[v] = __builtin_amdgcn_fmed3f(b2[v], lo, b3[v]);
            const int t2 = __builtin_unpredictable(lt2) ? j : i2[v];
            i2[v] = __builtin_unpredictable(lt1) ? i1[v] : t2;
            b2[v] = __builtin_amdgcn_fmed3f(b1[v], lo, b2[v]);
            i1[v] = __builtin_unpredictable(lt1) ? j : i1[v];
            b1[v] = fminf(b1[v], lo);
          }
        }
      };
      if (!GP || t == pia_tile) epilogue(std::true_type{});
      else epilogue(std::false_type{});
    }
    if constexpr (GR) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) gcur[b][v] = gnxt[b][v];
    }
    if constexpr (CH) {
      if (u + 1 < nsteps) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          xa[s] = xn[s];
          if constexpr (SP && !GP) ra[s] = pia >= 0 ? xn[s] - cn[s] : 0.f;
        }
      }
    }
  }
  __syncthreads();
}

struct RowShared {
  float xn[4][16];     // per wave, per row: ||x||
  float A[4][16];      // error coefficient of the current pass: delta_j = A (||x|| + ||c_j||)^2
  float lp[4][16];     // lambda / ||r||^2 (0 when r = 0)
  float av[4][16];     // <r, x>
  int pi[4][16];       // primary (-1: the row went to the full scan)
  int nc[4][16];       // number of candidates
  int sat[4][16];      // candidate set not proven complete
  int valid[4][16];    // grouped form: the stripe row is a data row
};
// Candidate lists; they live in the codebook ring, which is idle between the sweeps.
struct CandShared {
  int cand[4][16][32];
  float cv[4][16][32];
};

// Reduce the lane-level state to per-row candidate lists in LDS (output layout -> LDS).
__device__ __forceinline__ void publish_candidates(const AssignParams& P, RowShared& S,
                                                   CandShared& CS, int w, int lane,
                                                   const float (&xv)[4], const float (&Av)[4],
                                                   const float (&b1)[4], const int (&i1)[4],
                                                   const float (&b2)[4], const int (&i2)[4],
                                                   const float (&b3)[4]) {
  const int q = lane >> 4, c16 = lane & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * q + v;
    // an upper end of the exact minimum: the upper end hi' = lo' + 2 A_row (||x|| + ||c||)^2 of
    // the lane's best entry, least over the row's lanes; no centroid with a larger lower end can
    // be the arg-min
    float thr = kInf;
    if (b1[v] < kInf && i1[v] >= 0 && i1[v] < P.K) {
      const float tt = xv[v] + sqrtf(P.cnorm[i1[v]]);
      thr = fmaf(2.f * Av[v] * tt, tt, b1[v]);
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) thr = fminf(thr, __shfl_xor(thr, off));
    const bool finite_min = thr < kInf;
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
    if (c1) CS.cand[w][r][pos] = i1[v];
    if (c2) CS.cand[w][r][pos + 1] = i2[v];
  }
}

// Exact decision among a row's candidates (A layout: lane (q, c16) holds row c16's quarter q).
template <int DP, int BN, bool CH, bool VEC, bool SP>
__device__ __forceinline__ void decide(const AssignParams& P, RowShared& S, CandShared& CS, int nch,
                                       int w, int c16, int q, int64_t row, bool ok,
                                       const float (&xa)[DP / 4], const float (&ra)[DP / 4],
                                       float rr, int pi, int& best_j, float& best_v) {
  const int nc = S.nc[w][c16];
  float best = kInf;
  int bj = 0x7fffffff;
  for (int k = 0; k < nc; ++k) {
    const int j = CS.cand[w][c16][k];
    float sq, pj;
    direct32<DP, BN, CH, VEC, SP>(P, nch, row, ok, pi, j, q, xa, ra, sq, pj);
    const float val = (SP && rr > 0.f) ? sq + P.lam * (pj * pj) / rr : sq;
    CS.cv[w][c16][k] = val;
    if (val < best || (val == best && j < bj)) { best = val; bj = j; }
  }
  const float lim = best + best * P.tie_rel;
  int ntie = 0;
  for (int k = 0; k < nc; ++k) ntie += CS.cv[w][c16][k] <= lim;
  if (ntie >= 2) {
    double bd = __builtin_inf();
    int bdj = 0x7fffffff;
    for (int k = 0; k < nc; ++k) {
      if (CS.cv[w][c16][k] <= lim) {
        const int j = CS.cand[w][c16][k];
        argmin_d(bd, bdj, direct64<DP, BN, CH, VEC, SP>(P, nch, row, ok, pi, j, q, xa), j);
      }
    }
    best = (float)bd;
    bj = bdj;
    if (q == 0) atomicAdd(&P.counters[CNT_FP64], 1u);
  }
  best_j = bj;
  best_v = best;
}

// Two waves per SIMD (at most 256 registers, two workgroups' rings per CU) for rows that stay
// resident up to 128 dimensions; the wider shapes run one.
template <int DP, bool CH>
constexpr int f32_waves() { return (!CH && DP <= 128) ? 2 : 1; }
// The primary-only pass and the grouped spill pass hold no residual rows during the sweep: they
// run three waves per SIMD where three workgroups' rings fit in the 160 KB of LDS.
template <int DP, int BN, bool CH, bool SPILL>
constexpr int f32_kernel_waves() {
  return (!SPILL && !CH && DP <= 128 &&
          2 * F32Rec<DP, BN>::STAGE + (int)sizeof(RowShared) <= 53 * 1024)
             ? 3
             : f32_waves<DP, CH>();
}

// SPLIT (codebook splits, serving steps): gridDim.y splits share the tiles; split s sweeps its own
// tile range with the parameters offset to it (columns split-relative) and writes its exact
// arg-min and value to split_idx / split_val, its unproven rows to its own full-scan list.  The
// primary pass (SPLIT, !SPILL) runs first and split_merge_kernel joins the splits; the spill pass
// (SPLIT, SPILL) then takes the joined primary from P.primary instead of computing it.
template <int DP, int BN, bool CH, bool SPILL, bool VEC, bool GR, bool SPLIT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    f32_kernel_waves<DP, BN, CH, SPILL>(),
    f32_kernel_waves<DP, BN, CH, SPILL>() > 2 ? f32_kernel_waves<DP, BN, CH, SPILL>() : 2)))
void assign_f32_kernel(AssignParams P0) {
  using R = F32Rec<DP, BN>;
  constexpr int KS = DP / 4;
  static_assert(2 * R::STAGE >= (int)sizeof(CandShared), "candidate lists must fit in the ring");
  static_assert(!SPLIT || (!CH && !GR), "codebook splits: resident rows, direct form");
  AssignParams P = P0;
  int kbase = 0;                         // first column of the split
  size_t so = 0;                         // offset of the split's outputs
  if constexpr (SPLIT) {
    const int nt = (P0.K + BN - 1) / BN;
    const int t0 = (int)((int64_t)nt * blockIdx.y / gridDim.y);
    const int t1 = (int)((int64_t)nt * (blockIdx.y + 1) / gridDim.y);
    kbase = t0 * BN;
    P.Crec = P0.Crec + (size_t)t0 * R::BYTES;
    P.Crec_all = P0.Crec;
    P.cnorm = P0.cnorm + kbase;
    P.C = P0.C + (size_t)kbase * P0.d;
    P.K = min(P0.K, t1 * BN) - kbase;
    so = (size_t)blockIdx.y * (size_t)P0.n;
  }
  // one LDS object: [ring of two record stages | per-row state]
  __shared__ __attribute__((aligned(16))) char lds[2 * R::STAGE + sizeof(RowShared)];
  char* ring = lds;
  RowShared& S = *reinterpret_cast<RowShared*>(lds + 2 * R::STAGE);
  CandShared& CS = *reinterpret_cast<CandShared*>(ring);

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, q = lane >> 4, c16 = lane & 15;
  const int64_t n = live_rows(P.n, P.live_n);
  if ((int64_t)blockIdx.x * 64 >= n) return;   // whole block past the live rows
  const int64_t row = (int64_t)blockIdx.x * 64 + w * 16 + c16;  // A-layout row of this lane
  const bool ok = row < n;
  const int nch = CH ? (P.d + DP - 1) / DP : 1;

  float xa[KS], ra[KS];
  bool fin = true;
  float n0 = 0.f, n1 = 0.f, n2 = 0.f, n3 = 0.f;
  for (int ch = 0; ch < nch; ++ch) {
    load_seg<KS, VEC>(P.X, row, P.d, ch * DP + q * KS, ok, xa);
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      fin = fin && all_finite4(v4f{xa[s], xa[s + 1], xa[s + 2], xa[s + 3]});
      n0 = fmaf(xa[s], xa[s], n0); n1 = fmaf(xa[s + 1], xa[s + 1], n1);
      n2 = fmaf(xa[s + 2], xa[s + 2], n2); n3 = fmaf(xa[s + 3], xa[s + 3], n3);
      ra[s] = ra[s + 1] = ra[s + 2] = ra[s + 3] = 0.f;
    }
  }
  if (!fin) atomicOr(&P.counters[CNT_NONFINITE], 1u);
  const float xnorm = sqrtf(sum_quad_f((n0 + n1) + (n2 + n3)));
  if (q == 0) {
    S.xn[w][c16] = xnorm;
    S.A[w][c16] = 0.5f * P.band_p;
  }
  __syncthreads();

  // ---------------- primary pass ----------------
  float b1[4], b2[4], b3[4], lp[4], av[4], xv[4], Av[4];
  int i1[4], i2[4], pr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    b1[v] = b2[v] = b3[v] = kInf; i1[v] = i2[v] = 0x7fffffff;
    lp[v] = av[v] = 0.f; pr[v] = -1;
    xv[v] = S.xn[w][4 * q + v];
    Av[v] = S.A[w][4 * q + v];
  }
  int pi = -1;
  float pdist = 0.f;
  bool psat = false;
  if constexpr (!(SPLIT && SPILL)) {
    sweep<DP, BN, CH, VEC, false>(P, ring, nch, tid, row, ok, -1, xa, ra, lp, av, pr, xv, Av, b1,
                                  i1, b2, i2, b3);
    publish_candidates(P, S, CS, w, lane, xv, Av, b1, i1, b2, i2, b3);
    __syncthreads();

    psat = S.sat[w][c16] != 0;
    if (!psat) decide<DP, BN, CH, VEC, false>(P, S, CS, nch, w, c16, q, row, ok, xa, ra, 0.f, 0, pi, pdist);
    if (pi < 0 || pi >= P.K) psat = true;
    if (ok && q == 0) {
      if constexpr (SPLIT) {
        if (psat) {
          const unsigned slot = atomicAdd(&P0.split_cnt[blockIdx.y], 1u);
          P0.split_rows[so + slot] = (int32_t)row;
        }
        P0.split_idx[so + row] = psat ? -1 : pi;
        P0.split_val[so + row] = psat ? kInf : pdist;
      } else if (psat) {
        const unsigned slot = atomicAdd(&P.counters[CNT_FULLSCAN], 1u);
        P.full_rows[slot] = (int32_t)row;
        P.primary[row] = -1;   // finished by the full scan; left out of a grouped spill
      } else {
        P.primary[row] = pi;
        if (P.pdist) P.pdist[row] = pdist;
      }
    }
    if constexpr (!SPILL) return;
  } else {
    // the joined primary of the splits (global index)
    pi = ok ? P0.primary[row] : -1;
    if (pi < 0 || pi >= P0.K) { pi = -1; psat = true; }
  }

  // ---------------- residual ----------------
  if (psat) pi = -1;
  float rr = 0.f, a = 0.f;
  if (pi >= 0) {
    float r0 = 0.f, r1 = 0.f, r2 = 0.f, r3 = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int ch = 0; ch < nch; ++ch) {
      float cp[KS];
      load_rec<KS>(rec_row<DP, BN>(P0.Crec, nch, pi, ch) + q * KS, cp);   // (all of C)
      if constexpr (CH) load_seg<KS, VEC>(P.X, row, P.d, ch * DP + q * KS, ok, xa);
#pragma unroll
      for (int s = 0; s < KS; s += 4) {
        ra[s] = xa[s] - cp[s]; ra[s + 1] = xa[s + 1] - cp[s + 1];
        ra[s + 2] = xa[s + 2] - cp[s + 2]; ra[s + 3] = xa[s + 3] - cp[s + 3];
        r0 = fmaf(ra[s], ra[s], r0); r1 = fmaf(ra[s + 1], ra[s + 1], r1);
        r2 = fmaf(ra[s + 2], ra[s + 2], r2); r3 = fmaf(ra[s + 3], ra[s + 3], r3);
        a0 = fmaf(ra[s], xa[s], a0); a1 = fmaf(ra[s + 1], xa[s + 1], a1);
        a2 = fmaf(ra[s + 2], xa[s + 2], a2); a3 = fmaf(ra[s + 3], xa[s + 3], a3);
      }
    }
    rr = sum_quad_f((r0 + r1) + (r2 + r3));
    a = sum_quad_f((a0 + a1) + (a2 + a3));
  }
  if (q == 0) {
    S.pi[w][c16] = pi;
    S.lp[w][c16] = rr > 0.f ? P.lam / rr : 0.f;
    S.av[w][c16] = a;
    float A = 0.5f * P.band_s;
    if (GR && rr > 0.f) {
      // Gram form: <r, c_j> carries an error of gamma (||x|| + ||c_pi||) (||x|| + ||c_j||)
      const float Pn = xnorm + sqrtf(P.cnorm[pi]);
      const float inv = 1.f / sqrtf(rr);
      A += 0.5f * (P.band_g1 * Pn * inv + P.band_g2 * Pn * Pn * inv * inv);
    }
    S.A[w][c16] = A;
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * q + v;
    // (split-relative under SPLIT: the mask compares split columns)
    lp[v] = S.lp[w][r]; av[v] = S.av[w][r]; pr[v] = S.pi[w][r] - kbase; Av[v] = S.A[w][r];
    b1[v] = b2[v] = b3[v] = kInf; i1[v] = i2[v] = 0x7fffffff;
  }

  // ---------------- spill pass ----------------
  sweep<DP, BN, CH, VEC, true, GR>(P, ring, nch, tid, row, ok, pi, xa, ra, lp, av, pr, xv, Av,
                                   b1, i1, b2, i2, b3);
  publish_candidates(P, S, CS, w, lane, xv, Av, b1, i1, b2, i2, b3);
  __syncthreads();
  if (pi < 0) {
    // full-scan rows are finished by the full-scan kernel; under SPLIT a row without a primary
    // has no spill
    if constexpr (SPLIT) {
      if (ok && q == 0) P0.split_idx[so + row] = -1;
    }
    return;
  }
  if constexpr (GR) {
    // the Gram sweep does not read R: form it again here rather than hold it across the sweep
    float cp[KS];
    load_rec<KS>(rec_row<DP, BN>(P.Crec, nch, pi, 0) + q * KS, cp);
#pragma unroll
    for (int s = 0; s < KS; ++s) ra[s] = xa[s] - cp[s];
  }
  bool ssat = S.sat[w][c16] != 0;
  int sj = -1;
  float sl = 0.f;
  if (!ssat) decide<DP, BN, CH, VEC, true>(P, S, CS, nch, w, c16, q, row, ok, xa, ra, rr, pi, sj, sl);
  if (sj < 0 || sj >= P.K) ssat = true;
  if (ok && q == 0) {
    if constexpr (SPLIT) {
      if (ssat) {
        const unsigned slot = atomicAdd(&P0.split_cnt[blockIdx.y], 1u);
        P0.split_rows[so + slot] = (int32_t)row;
      }
      P0.split_idx[so + row] = ssat ? -1 : sj;
      P0.split_val[so + row] = ssat ? kInf : sl;
    } else if (ssat) {
      const unsigned slot = atomicAdd(&P.counters[CNT_FULLSCAN], 1u);
      P.full_rows[slot] = (int32_t)row;
    } else {
      P.spill[row] = sj;
      if (P.sloss) P.sloss[row] = sl;
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Grouped form of the spill pass.  A wave takes one stripe: up to 15 rows sharing the primary p
// (A-layout rows 0..14) and c_p itself as row 15, so the single MFMA stream X C^T also yields
// <c_p, c_j> and <r_i, c_j> = <x_i, c_j> - <c_p, c_j> needs no second stream and no Gram table.
// The error bound is the Gram form's.  Stripe rows past the stripe's size are zero and, like
// row 15, produce no output.
// ------------------------------------------------------------------------------------------------
// Chunked rows (d > 256) run two waves per SIMD: two workgroups' rings fill the LDS.
template <int DP, int BN, bool CH>
constexpr int f32_grouped_waves() { return CH ? 2 : f32_kernel_waves<DP, BN, false, false>(); }

template <int DP, int BN, bool CH, bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    f32_grouped_waves<DP, BN, CH>(),
    f32_grouped_waves<DP, BN, CH>() > 2 ? f32_grouped_waves<DP, BN, CH>() : 2)))
void assign_f32_spill_grouped(AssignParams P) {
  using R = F32Rec<DP, BN>;
  constexpr int KS = DP / 4;
  static_assert(2 * R::STAGE >= (int)sizeof(CandShared), "candidate lists must fit in the ring");
  __shared__ __attribute__((aligned(16))) char lds[2 * R::STAGE + sizeof(RowShared)];
  char* ring = lds;
  RowShared& S = *reinterpret_cast<RowShared*>(lds + 2 * R::STAGE);
  CandShared& CS = *reinterpret_cast<CandShared*>(ring);

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, q = lane >> 4, c16 = lane & 15;
  const int ns = *P.nstripes;
  if (blockIdx.x * 4 >= ns) return;             // whole block past the stripes
  const int sidx = blockIdx.x * 4 + w;
  const int4 sd = sidx < ns ? P.stripes[sidx] : int4{0, 0, 0, 0};   // {p, first, rows, -}
  const int p = sd.x, nrows = sd.z;
  const bool data = c16 < nrows;
  const int64_t row = data ? (int64_t)P.perm[sd.y + c16] : 0;
  const int nch = CH ? (P.d + DP - 1) / DP : 1;

  // Row constants over all chunks; stripe row 15 is the centroid c_p.  c_p and R are not kept
  // through the sweep (registers for a third wave per SIMD): the constants take r = x - c_p as
  // they go, and R is formed again afterwards where the rows stay resident.
  float xa[KS], ra[KS];
  float n0 = 0.f, n1 = 0.f, r0 = 0.f, r1 = 0.f, a0 = 0.f, a1 = 0.f;
  for (int ch = 0; ch < nch; ++ch) {
    float cp[KS];
    load_rec<KS>(rec_row<DP, BN>(P.Crec, nch, p, ch) + q * KS, cp);
    if (c16 == 15) {
#pragma unroll
      for (int s = 0; s < KS; ++s) xa[s] = cp[s];
    } else {
      load_seg<KS, VEC>(P.X, row, P.d, ch * DP + q * KS, data, xa);
    }
#pragma unroll
    for (int s = 0; s < KS; s += 2) {
      const float e0 = xa[s] - cp[s], e1 = xa[s + 1] - cp[s + 1];
      n0 = fmaf(xa[s], xa[s], n0); n1 = fmaf(xa[s + 1], xa[s + 1], n1);
      r0 = fmaf(e0, e0, r0); r1 = fmaf(e1, e1, r1);
      a0 = fmaf(e0, xa[s], a0); a1 = fmaf(e1, xa[s + 1], a1);
    }
  }
  const float xnorm = sqrtf(sum_quad_f(n0 + n1));
  const float rr = sum_quad_f(r0 + r1);
  const float a = sum_quad_f(a0 + a1);
  if (q == 0) {
    float A = 0.5f * P.band_s;
    if (rr > 0.f) {
      const float Pn = xnorm + sqrtf(P.cnorm[p]);
      const float inv = 1.f / sqrtf(rr);
      A += 0.5f * (P.band_g1 * Pn * inv + P.band_g2 * Pn * Pn * inv * inv);
    }
    S.xn[w][c16] = xnorm;
    S.A[w][c16] = A;
    S.lp[w][c16] = (data && rr > 0.f) ? P.lam / rr : 0.f;
    S.av[w][c16] = a;
    S.pi[w][c16] = p;
    S.valid[w][c16] = data;
  }
  __syncthreads();
  float b1[4], b2[4], b3[4], lp[4], av[4], xv[4], Av[4];
  int i1[4], i2[4], pr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * q + v;
    b1[v] = b2[v] = b3[v] = kInf; i1[v] = i2[v] = 0x7fffffff;
    lp[v] = S.lp[w][r]; av[v] = S.av[w][r]; pr[v] = p; xv[v] = S.xn[w][r]; Av[v] = S.A[w][r];
  }
  sweep<DP, BN, CH, VEC, true, false, true>(P, ring, nch, tid, row, data, p, xa, ra, lp, av, pr,
                                            xv, Av, b1, i1, b2, i2, b3);
  publish_candidates(P, S, CS, w, lane, xv, Av, b1, i1, b2, i2, b3);
  __syncthreads();
  if (!data) return;
  if constexpr (!CH) {
    // R again: c_p from its record (chunked rows are read again chunk by chunk instead)
    load_rec<KS>(rec_row<DP, BN>(P.Crec, 1, p, 0) + q * KS, ra);
#pragma unroll
    for (int s = 0; s < KS; ++s) ra[s] = xa[s] - ra[s];
  }
  bool ssat = S.sat[w][c16] != 0;
  int sj = -1;
  float sl = 0.f;
  if (!ssat) decide<DP, BN, CH, VEC, true>(P, S, CS, nch, w, c16, q, row, true, xa, ra, rr, p, sj, sl);
  if (sj < 0 || sj >= P.K) ssat = true;
  if (q == 0) {
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
// The 1024 threads form 64 groups of 16 lanes; a group takes one centroid at a time with its lanes
// across the dimensions, and a 16-lane tree gives the sum.  The row (and its residual) sit in LDS.
// The scan is latency-bound (few rows, each a chain of dependent loads), so the workgroup is as
// wide as possible: 256 centroid loads in flight per pass.
// ------------------------------------------------------------------------------------------------
constexpr int FS_THREADS = 1024;
constexpr int FS_WAVES = FS_THREADS / 64;
constexpr int FS_GROUPS = FS_THREADS / 16;

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ float sum16_f(float v) {
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ double sum16_d(double v) {
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// FP32 value of centroid j for this row: ||x - c||^2, or the SOAR loss given r and ||r||^2.
template <bool SP>
__device__ __forceinline__ float fs_value32(const float* __restrict__ c, const float* sx,
                                            const float* sr, float rr, float lam, int d, int l) {
  float sq0 = 0.f, sq1 = 0.f, pj0 = 0.f, pj1 = 0.f;
  int k = l;
  for (; k + 16 < d; k += 32) {
    const float e0 = sx[k] - c[k], e1 = sx[k + 16] - c[k + 16];
    sq0 = fmaf(e0, e0, sq0); sq1 = fmaf(e1, e1, sq1);
    if (SP) { pj0 = fmaf(sr[k], e0, pj0); pj1 = fmaf(sr[k + 16], e1, pj1); }
  }
  if (k < d) {
    const float e0 = sx[k] - c[k];
    sq0 = fmaf(e0, e0, sq0);
    if (SP) pj0 = fmaf(sr[k], e0, pj0);
  }
  const float sq = sum16_f(sq0 + sq1);
  if (!SP) return sq;
  const float pj = sum16_f(pj0 + pj1);
  return rr > 0.f ? sq + lam * (pj * pj) / rr : sq;
}

// FP64 value with the residual formed exactly from C[pi] (near-tie decisions).
template <bool SP>
__device__ __forceinline__ double fs_value64(const float* __restrict__ c, const float* sx,
                                             const float* scp, float lam, int d, int l) {
  double sq = 0.0, pj = 0.0, rr = 0.0;
  for (int k = l; k < d; k += 16) {
    const double e = (double)sx[k] - (double)c[k];
    sq = fma(e, e, sq);
    if (SP) {
      const double rk = (double)sx[k] - (double)scp[k];
      pj = fma(rk, e, pj);
      rr = fma(rk, rk, rr);
    }
  }
  sq = sum16_d(sq);
  if (!SP) return sq;
  pj = sum16_d(pj);
  rr = sum16_d(rr);
  return rr > 0.0 ? sq + (double)lam * (pj * pj) / rr : sq;
}

// Workgroup (value, index) minimum; every 16-lane group enters with its own candidate.
template <typename T>
__device__ __forceinline__ void wg_argmin(T& v, int& j, T* sv, int* sj) {
  const int tid = threadIdx.x, w = tid >> 6;
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
    const T ov = __shfl_xor(v, off);
    const int oj = __shfl_xor(j, off);
    if (ov < v || (ov == v && oj < j)) { v = ov; j = oj; }
  }
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

// Exact arg-min over all columns j != skip; FP32 direct values, then FP64 among near-ties.  A
// group evaluates 4 centroids per iteration (their loads in flight together); with sv non-null
// (K <= FS_LDS_K) the FP32 values are kept in LDS for the near-tie pass.
constexpr int FS_UNROLL = 4;
constexpr int FS_LDS_K = 8192;

template <bool SP>
__device__ void fs_argmin(const AssignParams& P, const float* sx, const float* sr, float rr,
                          const float* scp, int skip, float* sv, int& out_j, float& out_v) {
  __shared__ float rv[FS_WAVES];
  __shared__ int rj[FS_WAVES];
  __shared__ double rd[FS_WAVES];
  const int l = threadIdx.x & 15, g = threadIdx.x >> 4, K = P.K, d = P.d;
  float bv = kInf;
  int bj = 0x7fffffff;
  for (int j0 = g; j0 < K; j0 += FS_UNROLL * FS_GROUPS) {
    float v[FS_UNROLL];
#pragma unroll
    for (int u = 0; u < FS_UNROLL; ++u) {
      const int j = j0 + u * FS_GROUPS;
      const int jj = j < K ? j : K - 1;     // in-bounds address; the value is masked below
      v[u] = fs_value32<SP>(P.C + (int64_t)jj * d, sx, sr, rr, P.lam, d, l);
      if (j >= K || j == skip) v[u] = kInf;
    }
#pragma unroll
    for (int u = 0; u < FS_UNROLL; ++u) {
      const int j = j0 + u * FS_GROUPS;
      if (sv && j < K && l == 0) sv[j] = v[u];
      if (v[u] < bv) { bv = v[u]; bj = j; }
    }
  }
  wg_argmin<float>(bv, bj, rv, rj);   // (its barriers also publish sv)
  if (!(bv < kInf)) { out_j = -1; out_v = kInf; return; }
  const float lim = bv + bv * P.tie_rel;
  double dv = __builtin_inf();
  int dj = 0x7fffffff;
  for (int j = g; j < K; j += FS_GROUPS) {
    if (j == skip) continue;
    const float* c = P.C + (int64_t)j * d;
    const float v = sv ? sv[j] : fs_value32<SP>(c, sx, sr, rr, P.lam, d, l);
    if (v <= lim) argmin_d(dv, dj, fs_value64<SP>(c, sx, scp, P.lam, d, l), j);
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
  float* sv = P.K <= FS_LDS_K ? fs_smem + 3 * P.d : nullptr;
  __shared__ float s_rr;
  const unsigned count = P.counters[CNT_FULLSCAN];
  const int d = P.d, tid = threadIdx.x, lane = tid & 63;
  for (unsigned e = blockIdx.x; e < count; e += gridDim.x) {
    const int64_t row = P.full_rows[e];
    for (int k = tid; k < d; k += FS_THREADS) sx[k] = P.X[row * d + k];
    __syncthreads();
    int pi;
    float pd;
    fs_argmin<false>(P, sx, sr, 0.f, scp, -1, sv, pi, pd);
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
        fs_argmin<true>(P, sx, sr, s_rr, scp, pi, sv, sj, sl);
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
// Codebook splits (serving steps): the exact full scan of a split's unproven rows over the split's
// columns, and the join of the splits' answers.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ void split_range(int K, int BN, int s, int S, int& kb, int& ks) {
  const int nt = (K + BN - 1) / BN;
  const int t0 = (int)((int64_t)nt * s / S), t1 = (int)((int64_t)nt * (s + 1) / S);
  kb = t0 * BN;
  ks = min(K, t1 * BN) - kb;
}

template <bool SPILL>
__global__ __launch_bounds__(FS_THREADS) void full_scan_split_kernel(AssignParams P0, int BN) {
  extern __shared__ float fs_smem[];
  const int d = P0.d, tid = threadIdx.x, lane = tid & 63;
  const int s = blockIdx.y, S = gridDim.y;
  int kb, ks;
  split_range(P0.K, BN, s, S, kb, ks);
  AssignParams P = P0;
  P.C = P0.C + (size_t)kb * d;
  P.K = ks;
  // (the launch sizes the value cache for the largest split, ceil(tiles / S) tiles)
  const int kmax = ((P0.K + BN - 1) / BN + S - 1) / S * BN;
  float* sx = fs_smem;
  float* sr = fs_smem + d;
  float* scp = fs_smem + 2 * d;
  float* sv = kmax <= FS_LDS_K ? fs_smem + 3 * d : nullptr;
  __shared__ float s_rr;
  const size_t so = (size_t)s * (size_t)P0.n;
  const unsigned count = P0.split_cnt[s];
  for (unsigned e = blockIdx.x; e < count; e += gridDim.x) {
    const int64_t row = P0.split_rows[so + e];
    for (int k = tid; k < d; k += FS_THREADS) sx[k] = P0.X[row * d + k];
    __syncthreads();
    int j = -1;
    float v = kInf;
    if constexpr (!SPILL) {
      fs_argmin<false>(P, sx, sr, 0.f, scp, -1, sv, j, v);
    } else {
      const int pi = P0.primary[row];     // joined primary (whole codebook)
      const int pc = (pi >= 0 && pi < P0.K) ? pi : 0;   // (rows without one are not listed)
      for (int k = tid; k < d; k += FS_THREADS) {
        const float c = P0.C[(int64_t)pc * d + k];
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
      if (pi >= 0 && pi < P0.K) fs_argmin<true>(P, sx, sr, s_rr, scp, pi - kb, sv, j, v);
    }
    if (tid == 0) {
      P0.split_idx[so + row] = (j >= 0 && j < ks) ? j : -1;
      P0.split_val[so + row] = v;
      atomicAdd(&P0.counters[CNT_FP64], 1u);
    }
    __syncthreads();
  }
}

// Join of the S splits' answers for every row: the least value (then the lowest index); splits
// whose value lies within the near-tie gap of it are decided again in FP64 by direct differences
// (distance, or the SOAR loss with the residual formed exactly from the joined primary).
template <bool SPILL>
__global__ __launch_bounds__(256) void split_merge_kernel(AssignParams P0, int S, int BN) {
  const int64_t n = live_rows(P0.n, P0.live_n);
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  const int d = P0.d;
  const float* x = P0.X + row * d;
  int pi = -1;
  if constexpr (SPILL) {
    pi = P0.primary[row];
    if (pi < 0 || pi >= P0.K) {
      P0.spill[row] = -1;
      if (P0.sloss) P0.sloss[row] = kInf;
      return;
    }
  }
  float best = kInf;
  int bj = 0x7fffffff;
  for (int s = 0; s < S; ++s) {
    const int idx = P0.split_idx[(size_t)s * P0.n + row];
    if (idx < 0) continue;
    int kb, ks;
    split_range(P0.K, BN, s, S, kb, ks);
    const float v = P0.split_val[(size_t)s * P0.n + row];
    const int j = kb + idx;
    if (v < best || (v == best && j < bj)) { best = v; bj = j; }
  }
  if (bj != 0x7fffffff) {
    const float lim = best + best * P0.tie_rel;
    int near = 0;
    for (int s = 0; s < S; ++s)
      near += P0.split_idx[(size_t)s * P0.n + row] >= 0 &&
              P0.split_val[(size_t)s * P0.n + row] <= lim;
    if (near >= 2) {
      double bd = __builtin_inf();
      int bdj = 0x7fffffff;
      for (int s = 0; s < S; ++s) {
        const int idx = P0.split_idx[(size_t)s * P0.n + row];
        if (idx < 0 || !(P0.split_val[(size_t)s * P0.n + row] <= lim)) continue;
        int kb, ks;
        split_range(P0.K, BN, s, S, kb, ks);
        const int j = kb + idx;
        const float* c = P0.C + (int64_t)j * d;
        double sq = 0.0, pj = 0.0, rr = 0.0;
        for (int k = 0; k < d; ++k) {
          const double e = (double)x[k] - (double)c[k];
          sq = fma(e, e, sq);
          if constexpr (SPILL) {
            const double r = (double)x[k] - (double)P0.C[(int64_t)pi * d + k];
            pj = fma(r, e, pj);
            rr = fma(r, r, rr);
          }
        }
        const double val = (SPILL && rr > 0.0) ? sq + (double)P0.lam * (pj * pj) / rr : sq;
        argmin_d(bd, bdj, val, j);
      }
      best = (float)bd;
      bj = bdj;
      atomicAdd(&P0.counters[CNT_FP64], 1u);
    }
  }
  const int out = bj == 0x7fffffff ? -1 : bj;
  if constexpr (SPILL) {
    P0.spill[row] = out;
    if (P0.sloss) P0.sloss[row] = best;
  } else {
    P0.primary[row] = out;
    if (P0.pdist) P0.pdist[row] = best;
  }
}

// ------------------------------------------------------------------------------------------------
// Further spilled assignments (Section 3.5.1).  Given NP earlier assignments of a row, the next
// one minimises
//     ||x - c_j||^2 + lambda * sum_k <r_k, x - c_j>^2 / ||r_k||^2,   r_k = x - c_{prior_k},
// over the centroids not assigned yet (a term with r_k = 0 is dropped): one Theorem 3.1 penalty
// per earlier residual; with NP = 1 and the primary it is the SOAR spill.  The work is the direct
// spill form with NP residual streams: S = X C^T and T_k = R_k C^T on the matrix cores, the
// screen of the spill with lambda NP (each penalty term's rounding error is bounded like the
// spill's, so the bounds add up), the same candidate lists, FP32 re-scores by direct differences
// and FP64 near-tie decisions, and an exact full scan for rows whose candidate set is not proven
// complete.
// ------------------------------------------------------------------------------------------------
template <int NP>
struct FurtherShared {
  int pr[4][16][NP];    // earlier assignments of each row (-1: none)
  float lp[4][16][NP];  // lambda / ||r_k||^2 (0 when r_k = 0)
  float av[4][16][NP];  // <r_k, x>
};

template <int DP, int BN, bool CH, int NP>
__device__ __forceinline__ void sweep_further(const AssignParams& P, char* ring, int nch, int tid,
                                              int64_t row, bool ok, const int (&pk)[NP],
                                              float (&xa)[DP / 4], float (&ra)[NP][DP / 4],
                                              const float (&lp)[4][NP], const float (&av)[4][NP],
                                              const int (&pr)[4][NP], const float (&xv)[4],
                                              const float (&Av)[4], float (&b1)[4], int (&i1)[4],
                                              float (&b2)[4], int (&i2)[4], float (&b3)[4]) {
  using R = F32Rec<DP, BN>;
  constexpr int KS = DP / 4, LDW = R::LDW, NB = BN / 16;
  const int lane = tid & 63, w = tid >> 6, q = lane >> 4, c16 = lane & 15;
  const int ntiles = (P.K + BN - 1) / BN;
  const int nsteps = ntiles * (CH ? nch : 1);
  const char* recs = P.Crec;
  float kx[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) kx[v] = 2.f * xv[v];
  // chunked rows: chunk 0 now, chunk u+1 during step u
  float xn[CH ? KS : 1], cn[CH ? NP : 1][CH ? KS : 1];
  if constexpr (CH) {
    load_seg<KS, false>(P.X, row, P.d, q * KS, ok, xa);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      if (pk[k] >= 0) load_rec<KS>(rec_row<DP, BN>(recs, nch, pk[k], 0) + q * KS, cn[k]);
#pragma unroll
      for (int s = 0; s < KS; ++s) ra[k][s] = pk[k] >= 0 ? xa[s] - cn[k][s] : 0.f;
    }
  }
  issue_record<R::BYTES, R::STAGE, R::NI, 2>(recs, ring, 0, w, lane);
  v4f accS[NB], accT[NP][NB];
  for (int u = 0; u < nsteps; ++u) {
    const int ch = CH ? u % nch : 0, t = CH ? u / nch : u;
    wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if constexpr (CH) {
      if (u + 1 < nsteps) {
        const int cnx = (u + 1) % nch;
        load_seg<KS, false>(P.X, row, P.d, cnx * DP + q * KS, ok, xn);
#pragma unroll
        for (int k = 0; k < NP; ++k)
          if (pk[k] >= 0) load_rec<KS>(rec_row<DP, BN>(recs, nch, pk[k], cnx) + q * KS, cn[k]);
      }
    }
    if (u + 1 < nsteps) issue_record<R::BYTES, R::STAGE, R::NI, 2>(recs, ring, u + 1, w, lane);
    const float* sb = reinterpret_cast<const float*>(ring + (u & 1) * R::STAGE);
    if (ch == 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        accS[b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < NP; ++k) accT[k][b] = v4f{0.f, 0.f, 0.f, 0.f};
      }
    }
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      v4f bv[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b)
        bv[b] = *reinterpret_cast<const v4f*>(sb + (b * 16 + c16) * LDW + q * KS + s);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          accS[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[s + e], bv[b][e], accS[b], 0, 0, 0);
#pragma unroll
          for (int k = 0; k < NP; ++k)
            accT[k][b] =
                __builtin_amdgcn_mfma_f32_16x16x4f32(ra[k][s + e], bv[b][e], accT[k][b], 0, 0, 0);
        }
      }
    }
    if (!CH || ch == nch - 1) {
      const float* scn = reinterpret_cast<const float*>(ring + (u & 1) * R::STAGE + R::CN_OFF);
      const float* ssn = reinterpret_cast<const float*>(ring + (u & 1) * R::STAGE + R::SN_OFF);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = t * BN + b * 16 + c16;
        const float cnv = scn[b * 16 + c16];
        const float snv = ssn[b * 16 + c16];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float val = fmaf(-2.f, accS[b][v], cnv);
          bool masked = false;
#pragma unroll
          for (int k = 0; k < NP; ++k) {
            // <r_k, c_j> - <r_k, x>
            const float e = accT[k][b][v] - av[v][k];
            val = fmaf(lp[v][k] * e, e, val);
            masked = masked || j == pr[v][k];
          }
          if (masked) val = kInf;
          // the lower end (shifted) and the (b1, i1) <= (b2, i2) <= b3 update of the spill sweep
          const float lo = fmaf(-(Av[v] * (snv + kx[v])), snv, val);
          const bool lt1 = lo < b1[v], lt2 = lo < b2[v];
          b3[v] = __builtin_amdgcn_fmed3f(b2[v], lo, b3[v]);
          const int t2 = __builtin_unpredictable(lt2) ? j : i2[v];
          i2[v] = __builtin_unpredictable(lt1) ? i1[v] : t2;
          b2[v] = __builtin_amdgcn_fmed3f(b1[v], lo, b2[v]);
          i1[v] = __builtin_unpredictable(lt1) ? j : i1[v];
          b1[v] = fminf(b1[v], lo);
        }
      }
    }
    if constexpr (CH) {
      if (u + 1 < nsteps) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          xa[s] = xn[s];
#pragma unroll
          for (int k = 0; k < NP; ++k) ra[k][s] = pk[k] >= 0 ? xn[s] - cn[k][s] : 0.f;
        }
      }
    }
  }
  __syncthreads();
}

// FP32 ||x - c_j||^2 and <r_k, x - c_j> over this lane's quarter of the dimensions; with CH the
// rows' chunks are read again from X and the records of the earlier assignments.
template <int DP, int BN, bool CH, int NP>
__device__ __forceinline__ void direct32_further(const AssignParams& P, int nch, int64_t row,
                                                 const int (&pk)[NP], int j, int q,
                                                 const float (&xa)[DP / 4],
                                                 const float (&ra)[NP][DP / 4], float& sq,
                                                 float (&pj)[NP]) {
  constexpr int KS = DP / 4;
  float s0 = 0.f, s1 = 0.f, p0[NP], p1[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) p0[k] = p1[k] = 0.f;
  for (int ch = 0; ch < (CH ? nch : 1); ++ch) {
    float c[KS], xs[KS], e[KS];
    load_rec<KS>(rec_row<DP, BN>(P.Crec, nch, j, ch) + q * KS, c);
    if constexpr (CH) {
      load_seg<KS, false>(P.X, row, P.d, ch * DP + q * KS, true, xs);
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s) xs[s] = xa[s];
    }
#pragma unroll
    for (int s = 0; s < KS; s += 2) {
      e[s] = xs[s] - c[s];
      e[s + 1] = xs[s + 1] - c[s + 1];
      s0 = fmaf(e[s], e[s], s0);
      s1 = fmaf(e[s + 1], e[s + 1], s1);
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      float rs[KS];
      if constexpr (CH) {
        load_rec<KS>(rec_row<DP, BN>(P.Crec, nch, pk[k], ch) + q * KS, rs);
#pragma unroll
        for (int s = 0; s < KS; ++s) rs[s] = xs[s] - rs[s];
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) rs[s] = ra[k][s];
      }
#pragma unroll
      for (int s = 0; s < KS; s += 2) {
        p0[k] = fmaf(rs[s], e[s], p0[k]);
        p1[k] = fmaf(rs[s + 1], e[s + 1], p1[k]);
      }
    }
  }
  sq = sum_quad_f(s0 + s1);
#pragma unroll
  for (int k = 0; k < NP; ++k) pj[k] = sum_quad_f(p0[k] + p1[k]);
}

// The same in FP64 with every residual formed exactly from its centroid (near-tie decisions
// only); 4 values at a time in a rolled loop, which keeps this rare path's registers low.
template <int DP, int BN, bool CH, int NP>
__device__ __forceinline__ double direct64_further(const AssignParams& P, int nch, int64_t row,
                                                   const int (&pk)[NP], int j, int q,
                                                   const float (&xa)[DP / 4]) {
  constexpr int KS = DP / 4;
  double sq = 0.0, pj[NP], rr[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) pj[k] = rr[k] = 0.0;
  for (int ch = 0; ch < (CH ? nch : 1); ++ch) {
    const float* cj = rec_row<DP, BN>(P.Crec, nch, j, ch) + q * KS;
    float xs[CH ? KS : 1];
    if constexpr (CH) load_seg<KS, false>(P.X, row, P.d, ch * DP + q * KS, true, xs);
#pragma unroll 1
    for (int s0 = 0; s0 < KS; s0 += 4) {
      float c[4], xg[4];
      load_rec<4>(cj + s0, c);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        float xv = 0.f;
#pragma unroll
        for (int k = 0; k < KS; k += 4) xv = (k == s0) ? (CH ? xs[k + s] : xa[k + s]) : xv;
        xg[s] = xv;
      }
      double e[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        e[s] = (double)xg[s] - (double)c[s];
        sq = fma(e[s], e[s], sq);
      }
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        float cp[4];
        load_rec<4>(rec_row<DP, BN>(P.Crec, nch, pk[k], ch) + q * KS + s0, cp);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double r = (double)xg[s] - (double)cp[s];
          pj[k] = fma(r, e[s], pj[k]);
          rr[k] = fma(r, r, rr[k]);
        }
      }
    }
  }
  // the penalty terms are summed first, then added to the distance: integer inputs then give
  // the same FP64 value for every candidate whatever computes it, so exact ties break alike
  double pen = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double p = sum_quad_d(pj[k]), r = sum_quad_d(rr[k]);
    if (r > 0.0) pen += (double)P.lam * (p * p) / r;
  }
  return sum_quad_d(sq) + pen;
}

// Exact decision among a row's candidates (A layout), as for the spill.
template <int DP, int BN, bool CH, int NP>
__device__ __forceinline__ void decide_further(const AssignParams& P, RowShared& S, CandShared& CS,
                                               int nch, int w, int c16, int q, int64_t row,
                                               const int (&pk)[NP], const float (&xa)[DP / 4],
                                               const float (&ra)[NP][DP / 4],
                                               const float (&rr)[NP], int& best_j,
                                               float& best_v) {
  const int nc = S.nc[w][c16];
  float best = kInf;
  int bj = 0x7fffffff;
  for (int k = 0; k < nc; ++k) {
    const int j = CS.cand[w][c16][k];
    float sq, pj[NP];
    direct32_further<DP, BN, CH, NP>(P, nch, row, pk, j, q, xa, ra, sq, pj);
    float val = sq;
#pragma unroll
    for (int m = 0; m < NP; ++m)
      if (rr[m] > 0.f) val += P.lam * (pj[m] * pj[m]) / rr[m];
    CS.cv[w][c16][k] = val;
    if (val < best || (val == best && j < bj)) { best = val; bj = j; }
  }
  const float lim = best + best * P.tie_rel;
  int ntie = 0;
  for (int k = 0; k < nc; ++k) ntie += CS.cv[w][c16][k] <= lim;
  if (ntie >= 2) {
    double bd = __builtin_inf();
    int bdj = 0x7fffffff;
    for (int k = 0; k < nc; ++k) {
      if (CS.cv[w][c16][k] <= lim) {
        const int j = CS.cand[w][c16][k];
        argmin_d(bd, bdj, direct64_further<DP, BN, CH, NP>(P, nch, row, pk, j, q, xa), j);
      }
    }
    best = (float)bd;
    bj = bdj;
    if (q == 0) atomicAdd(&P.counters[CNT_FP64], 1u);
  }
  best_j = bj;
  best_v = best;
}

// One pass over all K for 64 rows (one workgroup), as the FP32 spill pass.  Prior indices
// outside [0, K) are not followed (the call has checked them and fails before any result is
// used); such a row's result is left unspecified.
template <int DP, int BN, bool CH, int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
void assign_f32_further(AssignParams P) {
  using R = F32Rec<DP, BN>;
  constexpr int KS = DP / 4;
  static_assert(2 * R::STAGE >= (int)sizeof(CandShared), "candidate lists must fit in the ring");
  __shared__ __attribute__((aligned(16)))
  char lds[2 * R::STAGE + sizeof(RowShared) + sizeof(FurtherShared<NP>)];
  char* ring = lds;
  RowShared& S = *reinterpret_cast<RowShared*>(lds + 2 * R::STAGE);
  FurtherShared<NP>& F =
      *reinterpret_cast<FurtherShared<NP>*>(lds + 2 * R::STAGE + sizeof(RowShared));
  CandShared& CS = *reinterpret_cast<CandShared*>(ring);

  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, q = lane >> 4, c16 = lane & 15;
  const int64_t n = P.n;
  if ((int64_t)blockIdx.x * 64 >= n) return;   // whole block past the rows
  const int64_t row = (int64_t)blockIdx.x * 64 + w * 16 + c16;  // A-layout row of this lane
  const bool ok = row < n;
  const int nch = CH ? (P.d + DP - 1) / DP : 1;
  int pk[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int v = ok ? P.prior[row * NP + k] : -1;
    pk[k] = (v >= 0 && v < P.K) ? v : -1;
  }
  // row constants over all chunks: ||x||, and per earlier assignment ||r_k||^2 and <r_k, x>
  float xa[KS], ra[NP][KS];
  float n0 = 0.f, n1 = 0.f, rq[NP], aq[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) rq[k] = aq[k] = 0.f;
  bool fin = true;
  for (int ch = 0; ch < nch; ++ch) {
    load_seg<KS, false>(P.X, row, P.d, ch * DP + q * KS, ok, xa);
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      fin = fin && all_finite4(v4f{xa[s], xa[s + 1], xa[s + 2], xa[s + 3]});
      n0 = fmaf(xa[s], xa[s], n0); n1 = fmaf(xa[s + 1], xa[s + 1], n1);
      n0 = fmaf(xa[s + 2], xa[s + 2], n0); n1 = fmaf(xa[s + 3], xa[s + 3], n1);
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      float cp[KS];
      if (pk[k] >= 0) {
        load_rec<KS>(rec_row<DP, BN>(P.Crec, nch, pk[k], ch) + q * KS, cp);
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) cp[s] = xa[s];
      }
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        ra[k][s] = xa[s] - cp[s];
        rq[k] = fmaf(ra[k][s], ra[k][s], rq[k]);
        aq[k] = fmaf(ra[k][s], xa[s], aq[k]);
      }
    }
  }
  if (!fin) atomicOr(&P.counters[CNT_NONFINITE], 1u);
  const float xnorm = sqrtf(sum_quad_f(n0 + n1));
  float rr[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    rr[k] = sum_quad_f(rq[k]);
    aq[k] = sum_quad_f(aq[k]);
  }
  if (q == 0) {
    S.xn[w][c16] = xnorm;
    S.A[w][c16] = 0.5f * P.band_s;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      F.pr[w][c16][k] = pk[k];
      F.lp[w][c16][k] = rr[k] > 0.f ? P.lam / rr[k] : 0.f;
      F.av[w][c16][k] = aq[k];
    }
  }
  __syncthreads();
  float b1[4], b2[4], b3[4], xv[4], Av[4], lp[4][NP], av[4][NP];
  int i1[4], i2[4], pr[4][NP];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * q + v;
    b1[v] = b2[v] = b3[v] = kInf; i1[v] = i2[v] = 0x7fffffff;
    xv[v] = S.xn[w][r];
    Av[v] = S.A[w][r];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      lp[v][k] = F.lp[w][r][k];
      av[v][k] = F.av[w][r][k];
      pr[v][k] = F.pr[w][r][k];
    }
  }
  sweep_further<DP, BN, CH, NP>(P, ring, nch, tid, row, ok, pk, xa, ra, lp, av, pr, xv, Av, b1, i1,
                                b2, i2, b3);
  publish_candidates(P, S, CS, w, lane, xv, Av, b1, i1, b2, i2, b3);
  __syncthreads();
  if (!ok) return;
  bool followed = true;                  // every earlier assignment in range
#pragma unroll
  for (int k = 0; k < NP; ++k) followed = followed && pk[k] >= 0;
  bool sat = S.sat[w][c16] != 0;
  int sj = -1;
  float sl = 0.f;
  if (!sat && followed)
    decide_further<DP, BN, CH, NP>(P, S, CS, nch, w, c16, q, row, pk, xa, ra, rr, sj, sl);
  if (sj < 0 || sj >= P.K) sat = true;
  if (q == 0) {
    if (sat) {
      const unsigned slot = atomicAdd(&P.counters[CNT_FULLSCAN], 1u);
      P.full_rows[slot] = (int32_t)row;
    } else {
      P.spill[row] = sj;
      if (P.sloss) P.sloss[row] = sl;
    }
  }
}

// Exact full scan of the listed rows for the further assignment (one workgroup a row): x, the
// residuals and the earlier centroids sit in LDS.
template <int NP>
__device__ __forceinline__ float fs_value32_further(const float* __restrict__ c, const float* sx,
                                                    const float* sr, const float* rr, float lam,
                                                    int d, int l) {
  float sq0 = 0.f, sq1 = 0.f, p0[NP], p1[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) p0[m] = p1[m] = 0.f;
  int k = l;
  for (; k + 16 < d; k += 32) {
    const float e0 = sx[k] - c[k], e1 = sx[k + 16] - c[k + 16];
    sq0 = fmaf(e0, e0, sq0); sq1 = fmaf(e1, e1, sq1);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      p0[m] = fmaf(sr[m * d + k], e0, p0[m]);
      p1[m] = fmaf(sr[m * d + k + 16], e1, p1[m]);
    }
  }
  if (k < d) {
    const float e0 = sx[k] - c[k];
    sq0 = fmaf(e0, e0, sq0);
#pragma unroll
    for (int m = 0; m < NP; ++m) p0[m] = fmaf(sr[m * d + k], e0, p0[m]);
  }
  float val = sum16_f(sq0 + sq1);
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const float p = sum16_f(p0[m] + p1[m]);
    if (rr[m] > 0.f) val += lam * (p * p) / rr[m];
  }
  return val;
}

template <int NP>
__device__ __forceinline__ double fs_value64_further(const float* __restrict__ c, const float* sx,
                                                     const float* scp, float lam, int d, int l) {
  double sq = 0.0, pj[NP], rr[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) pj[m] = rr[m] = 0.0;
  for (int k = l; k < d; k += 16) {
    const double e = (double)sx[k] - (double)c[k];
    sq = fma(e, e, sq);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      const double r = (double)sx[k] - (double)scp[m * d + k];
      pj[m] = fma(r, e, pj[m]);
      rr[m] = fma(r, r, rr[m]);
    }
  }
  double pen = 0.0;                        // penalties first, as in direct64_further
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const double p = sum16_d(pj[m]), r = sum16_d(rr[m]);
    if (r > 0.0) pen += (double)lam * (p * p) / r;
  }
  return sum16_d(sq) + pen;
}

template <int NP>
__global__ __launch_bounds__(FS_THREADS) void full_scan_further_kernel(AssignParams P) {
  extern __shared__ float fs_smem[];
  const int d = P.d, K = P.K, tid = threadIdx.x, lane = tid & 63;
  float* sx = fs_smem;
  float* sr = fs_smem + d;               // [NP x d] residuals
  float* scp = fs_smem + (1 + NP) * d;   // [NP x d] earlier centroids
  float* sv = K <= FS_LDS_K ? fs_smem + (1 + 2 * NP) * d : nullptr;
  __shared__ float s_rr[NP];
  __shared__ int s_pk[NP];
  __shared__ float rv[FS_WAVES];
  __shared__ int rj[FS_WAVES];
  __shared__ double rd[FS_WAVES];
  const unsigned count = P.counters[CNT_FULLSCAN];
  const int l = tid & 15, g = tid >> 4;
  for (unsigned e = blockIdx.x; e < count; e += gridDim.x) {
    const int64_t row = P.full_rows[e];
    if (tid < NP) {
      const int v = P.prior[row * NP + tid];
      s_pk[tid] = (v >= 0 && v < K) ? v : -1;
    }
    for (int k = tid; k < d; k += FS_THREADS) sx[k] = P.X[row * d + k];
    __syncthreads();
    bool valid = true;
#pragma unroll
    for (int m = 0; m < NP; ++m) valid = valid && s_pk[m] >= 0;
    if (!valid) {                         // not followed (the call reports SOAR_E_INVAL)
      if (tid == 0) P.spill[row] = -1;
      __syncthreads();
      continue;
    }
#pragma unroll
    for (int m = 0; m < NP; ++m)
      for (int k = tid; k < d; k += FS_THREADS) {
        const float c = P.C[(int64_t)s_pk[m] * d + k];
        scp[m * d + k] = c;
        sr[m * d + k] = sx[k] - c;
      }
    __syncthreads();
    if (tid < 64) {
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        float a = 0.f;
        for (int k = lane; k < d; k += 64) a = fmaf(sr[m * d + k], sr[m * d + k], a);
        a = wave_sum_f(a);
        if (tid == 0) s_rr[m] = a;
      }
    }
    __syncthreads();
    float rr[NP];
    int pk[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) { rr[m] = s_rr[m]; pk[m] = s_pk[m]; }
    auto skip = [&](int j) {
      bool s = false;
#pragma unroll
      for (int m = 0; m < NP; ++m) s = s || j == pk[m];
      return s;
    };
    // FP32 direct values over all columns, then FP64 among the near-ties
    float bv = kInf;
    int bj = 0x7fffffff;
    for (int j0 = g; j0 < K; j0 += FS_UNROLL * FS_GROUPS) {
      float v[FS_UNROLL];
#pragma unroll
      for (int u = 0; u < FS_UNROLL; ++u) {
        const int j = j0 + u * FS_GROUPS;
        const int jj = j < K ? j : K - 1;
        v[u] = fs_value32_further<NP>(P.C + (int64_t)jj * d, sx, sr, rr, P.lam, d, l);
        if (j >= K || skip(j)) v[u] = kInf;
      }
#pragma unroll
      for (int u = 0; u < FS_UNROLL; ++u) {
        const int j = j0 + u * FS_GROUPS;
        if (sv && j < K && l == 0) sv[j] = v[u];
        if (v[u] < bv) { bv = v[u]; bj = j; }
      }
    }
    wg_argmin<float>(bv, bj, rv, rj);
    int out_j = -1;
    float out_v = kInf;
    if (bv < kInf) {
      const float lim = bv + bv * P.tie_rel;
      double dv = __builtin_inf();
      int dj = 0x7fffffff;
      for (int j = g; j < K; j += FS_GROUPS) {
        if (skip(j)) continue;
        const float* c = P.C + (int64_t)j * d;
        const float v = sv ? sv[j] : fs_value32_further<NP>(c, sx, sr, rr, P.lam, d, l);
        if (v <= lim) argmin_d(dv, dj, fs_value64_further<NP>(c, sx, scp, P.lam, d, l), j);
      }
      wg_argmin<double>(dv, dj, rd, rj);
      out_j = dj < K ? dj : -1;
      out_v = (float)dv;
    }
    if (tid == 0) {
      P.spill[row] = out_j;
      if (P.sloss) P.sloss[row] = out_v;
      atomicAdd(&P.counters[CNT_FP64], 1u);
    }
    __syncthreads();
  }
}

__global__ void check_priors_kernel(const int32_t* __restrict__ prior, int64_t n, int np, int K,
                                    unsigned* counters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool bad = false;
  for (int a = 0; a < np; ++a) {
    const int v = prior[i * np + a];
    bad = bad || v < 0 || v >= K;
    for (int b = 0; b < a; ++b) bad = bad || prior[i * np + b] == v;
  }
  if (bad) atomicOr(&counters[CNT_BADINPUT], 1u);
}

// ------------------------------------------------------------------------------------------------
// Codebook preparation: ||c_j||^2, max ||c||^2 and the finiteness flag; counter reset.
// ------------------------------------------------------------------------------------------------
__global__ void reset_counters_kernel(unsigned* counters, int words) {
  if ((int)threadIdx.x < words) counters[threadIdx.x] = 0u;
}

// Status record of an enqueue-only call: its non-finite flag is kept in words the per-call reset
// leaves alone, behind two magic words, so that garbage in a fresh workspace never reads as a
// status.  The next blocking call reads the record and clears it.
__global__ void async_note_kernel(unsigned* counters) {
  if (threadIdx.x != 0 || counters[CNT_NONFINITE] == 0u) return;
  if (counters[CNT_ASYNC_M0] != kAsyncMagic0 || counters[CNT_ASYNC_M1] != kAsyncMagic1)
    counters[CNT_ASYNC_FLAGS] = 0u;
  counters[CNT_ASYNC_M0] = kAsyncMagic0;
  counters[CNT_ASYNC_M1] = kAsyncMagic1;
  counters[CNT_ASYNC_FLAGS] |= 1u;
}
__global__ void async_clear_kernel(unsigned* counters) {
  if (threadIdx.x < 3) counters[CNT_ASYNC_M0 + threadIdx.x] = 0u;
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
__global__ __launch_bounds__(256) void pack_f32_kernel(const float* __restrict__ C, int K, int d,
                                                       int nch, const float* __restrict__ cnorm,
                                                       char* __restrict__ rec, int64_t total,
                                                       float A_p) {
  using R = F32Rec<DP, BN>;
  constexpr int F4 = R::LDW / 4;   // float4 per record row (the last one is the pad)
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= total) return;
  const int f = (int)(g % F4);
  const int64_t jc = g / F4;
  const int ch = (int)(jc % nch), j = (int)(jc / nch);
  char* base = rec + ((int64_t)(j / BN) * nch + ch) * R::BYTES;
  const int jl = j % BN, k = ch * DP + f * 4;
  v4f v = {0.f, 0.f, 0.f, 0.f};
  if (j < K && f * 4 < DP) {
    const float* c = C + (int64_t)j * d;
    if (k < d) v.x = c[k];
    if (k + 1 < d) v.y = c[k + 1];
    if (k + 2 < d) v.z = c[k + 2];
    if (k + 3 < d) v.w = c[k + 3];
  }
  *reinterpret_cast<v4f*>(base + (jl * R::LDW + f * 4) * 4) = v;
  if (f == 0) {
    *reinterpret_cast<float*>(base + R::CN_OFF + jl * 4) = j < K ? cnorm[j] : kInf;
    *reinterpret_cast<float*>(base + R::SN_OFF + jl * 4) = j < K ? sqrtf(cnorm[j]) : 0.f;
    *reinterpret_cast<float*>(base + R::CA_OFF + jl * 4) =
        j < K ? fmaf(-A_p, cnorm[j], cnorm[j]) : kInf;
  }
}

// G = C C^T: a 64 x 64 block of G per workgroup, 4 x 4 outputs per thread, the two 64-row
// slices of C staged through LDS 16 dimensions at a time.
__global__ __launch_bounds__(256) void gram_kernel(const float* __restrict__ C, int K, int d,
                                                   float* __restrict__ G) {
  __shared__ float sa[16][65], sb[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < d; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int r = e >> 4, k = e & 15;
      sa[k][r] = (i0 + r < K && k0 + k < d) ? C[(int64_t)(i0 + r) * d + k0 + k] : 0.f;
      sb[k][r] = (j0 + r < K && k0 + k < d) ? C[(int64_t)(j0 + r) * d + k0 + k] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(sa[k][ty + 16 * a], sb[k][tx + 16 * b], acc[a][b]);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + ty + 16 * a, j = j0 + tx + 16 * b;
      if (i < K && j < K) G[(int64_t)i * K + j] = acc[a][b];
    }
}

bool fp32_uses_gram(int d, int K) { return K <= kGramMaxK && d <= 256; }

hipError_t launch_gram(const float* C, int K, int d, float* G, hipStream_t st) {
  const unsigned nb = (unsigned)((K + 63) / 64);
  hipLaunchKernelGGL(gram_kernel, dim3(nb, nb), dim3(256), 0, st, C, K, d, G);
  return hipGetLastError();
}

// Padded widths: rows of up to 256 stay resident; longer rows go in chunks of 128.
constexpr int kF32ChunkDP = 128, kF32ChunkBN = 64, kF32MaxD = 1024;

int fp32_padded_dim(int d) {
  static const int dps[] = {16, 32, 48, 64, 96, 128, 192, 256};
  for (int dp : dps)
    if (d <= dp) return dp;
  if (d <= kF32MaxD) return (d + kF32ChunkDP - 1) / kF32ChunkDP * kF32ChunkDP;
  return -1;
}

template <int DP, int BN>
static size_t rec_bytes(int d, int K) {
  const int nch = (d + DP - 1) / DP;
  return (size_t)((K + BN - 1) / BN) * nch * F32Rec<DP, BN>::BYTES;
}

template <int DP, int BN>
static hipError_t pack_dp(const float* C, int K, int d, const float* cnorm, void* rec,
                          hipStream_t st) {
  const int nch = (d + DP - 1) / DP;
  const int64_t total = (int64_t)((K + BN - 1) / BN) * BN * nch * (F32Rec<DP, BN>::LDW / 4);
  hipLaunchKernelGGL((pack_f32_kernel<DP, BN>), dim3((unsigned)((total + 255) / 256)), dim3(256),
                     0, st, C, K, d, nch, cnorm, static_cast<char*>(rec), total,
                     0.5f * band_coef_primary(d));
  return hipGetLastError();
}

template <int DP, int BN, bool CH>
static hipError_t launch_dp(const AssignParams& P, bool spill, bool vec, hipStream_t st) {
  const dim3 grid((unsigned)((P.n + 63) / 64)), block(256);
  if (spill && P.G) {
    if constexpr (!CH) {
      if (vec) hipLaunchKernelGGL((assign_f32_kernel<DP, BN, CH, true, true, true>), grid, block, 0, st, P);
      else hipLaunchKernelGGL((assign_f32_kernel<DP, BN, CH, true, false, true>), grid, block, 0, st, P);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (spill) {
    if (vec) hipLaunchKernelGGL((assign_f32_kernel<DP, BN, CH, true, true, false>), grid, block, 0, st, P);
    else hipLaunchKernelGGL((assign_f32_kernel<DP, BN, CH, true, false, false>), grid, block, 0, st, P);
  } else {
    if (vec) hipLaunchKernelGGL((assign_f32_kernel<DP, BN, CH, false, true, false>), grid, block, 0, st, P);
    else hipLaunchKernelGGL((assign_f32_kernel<DP, BN, CH, false, false, false>), grid, block, 0, st, P);
  }
  return hipGetLastError();
}

// Plain switches over the padded width (the shapes below and in the launcher must agree).
#define SOAR_F32_SHAPES(X)                \
  case 16: X(16, 64, false); break;       \
  case 32: X(32, 64, false); break;       \
  case 48: X(48, 64, false); break;       \
  case 64: X(64, 64, false); break;       \
  case 96: X(96, 32, false); break;       \
  case 128: X(128, 32, false); break;     \
  case 192: X(192, 32, false); break;     \
  case 256: X(256, 32, false); break;     \
  default: X(kF32ChunkDP, kF32ChunkBN, true); break;

size_t fp32_codebook_bytes(int d, int K) {
  const int dp = fp32_padded_dim(d);
  if (dp < 0) return 0;
#define SOAR_X(DP, BN, CH) return rec_bytes<DP, BN>(d, K)
  switch (dp) { SOAR_F32_SHAPES(SOAR_X) }
#undef SOAR_X
  return 0;
}

hipError_t launch_pack_fp32(const float* C, int K, int d, const float* cnorm, void* rec,
                            hipStream_t st) {
  const int dp = fp32_padded_dim(d);
  if (dp < 0) return hipErrorInvalidValue;
#define SOAR_X(DP, BN, CH) return pack_dp<DP, BN>(C, K, d, cnorm, rec, st)
  switch (dp) { SOAR_F32_SHAPES(SOAR_X) }
#undef SOAR_X
  return hipErrorInvalidValue;
}

hipError_t launch_prep_codebook(const float* C, int K, int d, float* cnorm, unsigned* counters,
                                hipStream_t st) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, counters, (int)CNT_WORDS);
  hipLaunchKernelGGL(prep_codebook_kernel, dim3((K + 255) / 256), dim3(256), 0, st, C, K, d,
                     cnorm, counters);
  return hipGetLastError();
}

hipError_t launch_async_note(unsigned* counters, hipStream_t st) {
  hipLaunchKernelGGL(async_note_kernel, dim3(1), dim3(64), 0, st, counters);
  return hipGetLastError();
}

hipError_t launch_async_clear(unsigned* counters, hipStream_t st) {
  hipLaunchKernelGGL(async_clear_kernel, dim3(1), dim3(64), 0, st, counters);
  return hipGetLastError();
}

hipError_t launch_reset_step_counters(unsigned* counters, hipStream_t st) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, counters,
                     (int)CNT_STEP_WORDS);
  return hipGetLastError();
}

template <int DP, int BN, bool CH>
static hipError_t launch_grouped_dp(const AssignParams& P, bool vec, hipStream_t st) {
  const int64_t ms = group_max_stripes(P.n, P.K);
  const dim3 grid((unsigned)((ms + 3) / 4)), block(256);
  if (vec) hipLaunchKernelGGL((assign_f32_spill_grouped<DP, BN, CH, true>), grid, block, 0, st, P);
  else hipLaunchKernelGGL((assign_f32_spill_grouped<DP, BN, CH, false>), grid, block, 0, st, P);
  return hipGetLastError();
}

hipError_t launch_assign_fp32(const AssignParams& P, bool spill, bool vec, hipStream_t st,
                              hipEvent_t* ev, const GroupLayout* grouped) {
  hipError_t e;
  const int dp = fp32_padded_dim(P.d);
  if (dp < 0 || !P.Crec) return hipErrorInvalidValue;
  auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], st); };
  if (spill && grouped) {
    // primary pass, rows grouped by primary, grouped spill pass
#define SOAR_X(DP, BN, CH) e = launch_dp<DP, BN, CH>(P, false, vec, st)
    switch (dp) { SOAR_F32_SHAPES(SOAR_X) }
#undef SOAR_X
    if (e != hipSuccess) return e;
    mark(0);
    mark(1);
    e = launch_group_by_primary(P.primary, P.n, P.live_n, P.K, *grouped, st);
    if (e != hipSuccess) return e;
    mark(2);
    AssignParams Q = P;
    Q.perm = grouped->perm;
    Q.stripes = grouped->stripes;
    Q.nstripes = grouped->meta;
    // the same shape table as the packing, so the kernel reads the records it was given
#define SOAR_X(DP, BN, CH) e = launch_grouped_dp<DP, BN, CH>(Q, vec, st)
    switch (dp) { SOAR_F32_SHAPES(SOAR_X) }
#undef SOAR_X
  } else {
#define SOAR_X(DP, BN, CH) e = launch_dp<DP, BN, CH>(P, spill, vec, st)
    switch (dp) { SOAR_F32_SHAPES(SOAR_X) }
#undef SOAR_X
    // one pass holds both sweeps: its time is the primary phase, the spill phases stay empty
    mark(0);
    mark(1);
    mark(2);
  }
  if (e != hipSuccess) return e;
  mark(3);
  const size_t smem = ((size_t)3 * P.d + (P.K <= FS_LDS_K ? (size_t)P.K : 0)) * sizeof(float);
  if (spill)
    hipLaunchKernelGGL(full_scan_kernel<true>, dim3(256), dim3(FS_THREADS), smem, st, P);
  else
    hipLaunchKernelGGL(full_scan_kernel<false>, dim3(256), dim3(FS_THREADS), smem, st, P);
  return hipGetLastError();
}

// ---- codebook splits (serving steps) ----
bool fp32_split_supported(int d) {
  const int dp = fp32_padded_dim(d);
  return dp > 0 && dp <= 256;
}

template <int DP, int BN>
static hipError_t launch_split_dp(const AssignParams& P, int S, bool vec, hipStream_t st) {
  const dim3 grid((unsigned)((P.n + 63) / 64), (unsigned)S), block(256);
  const dim3 mgrid((unsigned)((P.n + 255) / 256));
  const int nt = (P.K + BN - 1) / BN;
  const int kmax = (nt + S - 1) / S * BN;
  const size_t smem = ((size_t)3 * P.d + (kmax <= FS_LDS_K ? (size_t)kmax : 0)) * sizeof(float);
  // primary: the splits, their full scans, the join
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, P.split_cnt, S);
  if (vec) hipLaunchKernelGGL((assign_f32_kernel<DP, BN, false, false, true, false, true>), grid, block, 0, st, P);
  else hipLaunchKernelGGL((assign_f32_kernel<DP, BN, false, false, false, false, true>), grid, block, 0, st, P);
  hipLaunchKernelGGL(full_scan_split_kernel<false>, dim3(64, (unsigned)S), dim3(FS_THREADS), smem,
                     st, P, BN);
  hipLaunchKernelGGL(split_merge_kernel<false>, mgrid, dim3(256), 0, st, P, S, BN);
  // spill given the joined primary
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, P.split_cnt, S);
  if (vec) hipLaunchKernelGGL((assign_f32_kernel<DP, BN, false, true, true, false, true>), grid, block, 0, st, P);
  else hipLaunchKernelGGL((assign_f32_kernel<DP, BN, false, true, false, false, true>), grid, block, 0, st, P);
  hipLaunchKernelGGL(full_scan_split_kernel<true>, dim3(64, (unsigned)S), dim3(FS_THREADS), smem,
                     st, P, BN);
  hipLaunchKernelGGL(split_merge_kernel<true>, mgrid, dim3(256), 0, st, P, S, BN);
  return hipGetLastError();
}

hipError_t launch_assign_fp32_split(const AssignParams& P, int S, bool vec, hipStream_t st) {
  const int dp = fp32_padded_dim(P.d);
  if (dp < 0 || dp > 256 || S < 1 || S > 64 || !P.Crec || !P.split_idx || !P.split_val ||
      !P.split_rows || !P.split_cnt || !P.primary || !P.spill || P.K < S)
    return hipErrorInvalidValue;
  hipError_t e = hipErrorInvalidValue;
#define SOAR_X(DP, BN, CH)                                      \
  if constexpr (!CH) e = launch_split_dp<DP, BN>(P, S, vec, st); \
  else e = hipErrorInvalidValue
  switch (dp) { SOAR_F32_SHAPES(SOAR_X) }
#undef SOAR_X
  return e;
}

// ---- further spilled assignments ----
// Whole rows up to 128 dimensions; longer rows in chunks of 64, so that X and the NP residual
// rows (and their next chunks) stay in registers.
int fp32_further_padded_dim(int d) {
  static const int dps[] = {16, 32, 48, 64, 96, 128};
  for (int dp : dps)
    if (d <= dp) return dp;
  if (d <= kF32MaxD) return (d + 63) / 64 * 64;
  return -1;
}

#define SOAR_F32F_SHAPES(X)            \
  case 16: X(16, 64, false); break;   \
  case 32: X(32, 64, false); break;   \
  case 48: X(48, 64, false); break;   \
  case 64: X(64, 64, false); break;   \
  case 96: X(96, 32, false); break;   \
  case 128: X(128, 32, false); break; \
  default: X(64, 64, true); break;

size_t fp32_further_codebook_bytes(int d, int K) {
  const int dp = fp32_further_padded_dim(d);
  if (dp < 0) return 0;
#define SOAR_X(DP, BN, CH) return rec_bytes<DP, BN>(d, K)
  switch (dp) { SOAR_F32F_SHAPES(SOAR_X) }
#undef SOAR_X
  return 0;
}

hipError_t launch_pack_fp32_further(const float* C, int K, int d, const float* cnorm, void* rec,
                                    hipStream_t st) {
  const int dp = fp32_further_padded_dim(d);
  if (dp < 0) return hipErrorInvalidValue;
#define SOAR_X(DP, BN, CH) return pack_dp<DP, BN>(C, K, d, cnorm, rec, st)
  switch (dp) { SOAR_F32F_SHAPES(SOAR_X) }
#undef SOAR_X
  return hipErrorInvalidValue;
}

hipError_t launch_check_priors(const int32_t* prior, int64_t n, int np, int K, unsigned* counters,
                               hipStream_t st) {
  hipLaunchKernelGGL(check_priors_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     prior, n, np, K, counters);
  return hipGetLastError();
}

template <int DP, int BN, bool CH>
static hipError_t launch_further_dp(const AssignParams& P, int np, hipStream_t st) {
  const dim3 grid((unsigned)((P.n + 63) / 64)), block(256);
  switch (np) {
    case 1: hipLaunchKernelGGL((assign_f32_further<DP, BN, CH, 1>), grid, block, 0, st, P); break;
    case 2: hipLaunchKernelGGL((assign_f32_further<DP, BN, CH, 2>), grid, block, 0, st, P); break;
    case 3: hipLaunchKernelGGL((assign_f32_further<DP, BN, CH, 3>), grid, block, 0, st, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_further_fp32(const AssignParams& P, int np, hipStream_t st) {
  const int dp = fp32_further_padded_dim(P.d);
  if (dp < 0 || !P.Crec || !P.prior || np < 1 || np > kFurtherMaxPrior) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
#define SOAR_X(DP, BN, CH) e = launch_further_dp<DP, BN, CH>(P, np, st)
  switch (dp) { SOAR_F32F_SHAPES(SOAR_X) }
#undef SOAR_X
  if (e != hipSuccess) return e;
  const size_t smem =
      ((size_t)(1 + 2 * np) * P.d + (P.K <= FS_LDS_K ? (size_t)P.K : 0)) * sizeof(float);
  switch (np) {
    case 1: hipLaunchKernelGGL(full_scan_further_kernel<1>, dim3(256), dim3(FS_THREADS), smem, st, P); break;
    case 2: hipLaunchKernelGGL(full_scan_further_kernel<2>, dim3(256), dim3(FS_THREADS), smem, st, P); break;
    default: hipLaunchKernelGGL(full_scan_further_kernel<3>, dim3(256), dim3(FS_THREADS), smem, st, P); break;
  }
  return hipGetLastError();
}

}  // namespace soar
