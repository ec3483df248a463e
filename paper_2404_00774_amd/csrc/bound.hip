// The nearest centroids of every centroid, for a bound that confines a row's spill to a few
// columns so that the row needs no spill sweep.
//
// Let x have primary p and residual r = x - c_p (Section 3.1), and let L(j) be its spill loss
// ||x - c_j||^2 + lambda <r, x - c_j>^2 / ||r||^2 (Section 3.4, Theorem 3.1).  The penalty term
// lies between 0 and lambda ||x - c_j||^2 (Cauchy-Schwarz), so for the spill j* and any other
// centroid j2 != p
//     ||x - c_j*||^2 <= L(j*) <= L(j2) <= (1 + lambda) ||x - c_j2||^2 =: U,
// and by the triangle inequality ||c_p - c_j*|| <= ||r|| + sqrt(U).  If every centroid outside
// the M nearest of c_p lies farther from c_p than that, j* is one of those M, and an exact
// re-score of them decides the spill.  This file computes, for every centroid p, its M nearest
// other centroids and a lower bound on the distance from c_p to every other centroid, and
// decides the rows.  The table costs 2 K^2 d FP32 flop, so it is built only where it pays: the
// same kernels first run over 256 sample rows (their two nearest centroids, then the table
// entries of their nearest centroids), and a one-workgroup kernel scales the sample's decided
// share to n and sets a device flag that the full table's kernels and the decision kernel read
// (no host round trip; an enqueue-only call stays one).
//
// Distances come from the expansion ||a||^2 + ||b||^2 - 2 <a, b> in FP32.  Its error is at most
// (d + 2) u (||a|| + ||b||)^2 (u = 2^-24: the dot product's and the norms' accumulations and
// the two final roundings), so each value is lowered by twice that before it is ranked: the
// ranked quantity is a proven lower bound of the squared distance, and the (M + 1)-th smallest
// of them bounds every centroid left out.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace soar {

namespace {

constexpr int KT = 64;        // centroids per tile, on both sides (four 16-column blocks)

// One workgroup of four waves per 64 centroids p (16 per wave) and part blockIdx.y of the
// codebook; the part's centroids stream through LDS in tiles of 64 and chunks of DPC = 4 DQ
// dimensions, both sides' chunks through LDS (the p side is read once when one chunk covers the
// rows), each chunk loaded into registers one step ahead so that its loads overlap the MFMAs of
// the step before.  The products <c_p, c_j> run on v_mfma_f32_16x16x4_f32 with the contraction
// permuted: at step s, lane (q, i) supplies element q DQ + s of the chunk for row i of the
// wave's p rows (A) and of block b's j rows (B).  In the output layout lane (q, c16) holds p rows
// 4 q + v (v = 0..3) at column c16 of every block, and keeps, for each of its four p rows, the
// M + 1 smallest lower values it saw (ascending); the 16 lanes of group q merge theirs and write
// the part's M + 1 smallest to tv / tj ([K][parts][M + 1]) for knn_merge_kernel.
// The p side (A) is rows of A (the codebook itself, or rows of X for the sample estimate):
// every row (plist null, np = arows) or the rows plist[0 .. np) (entries outside [0, arows) are
// skipped); outputs are indexed by position in that list.  A row's squared norm is anorm[k] for
// list position k, or cnorm of the row when anorm is null.  self: A is the codebook, and a
// centroid is not its own neighbour.  With enable set and *enable == 0 the kernel does nothing.
// LIST = false is the codebook against itself (A = C, every row, self); the general form only
// runs on the samples.
template <int DQ, int M, bool LIST>
__global__ __launch_bounds__(256) void centroid_knn_kernel(
    const float* __restrict__ A, int64_t arows, const float* __restrict__ anorm, int self,
    const float* __restrict__ C, int K, int d, const float* __restrict__ cnorm,
    const int32_t* __restrict__ plist, int np, const int32_t* enable, float* __restrict__ tv,
    int32_t* __restrict__ tj) {
  if (enable && *enable == 0) return;
  constexpr int DPC = 4 * DQ;       // dimensions per chunk
  constexpr int LDW = DPC + 4;      // LDS row stride (floats): 16-byte aligned
  constexpr int F4 = KT * DPC / 4;  // float4 per side per chunk
  constexpr int NF = (F4 + 255) / 256;   // of them per thread
  __shared__ __attribute__((aligned(16))) float sA[KT * LDW];
  __shared__ __attribute__((aligned(16))) float sB[KT * LDW];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63, q = lane >> 4, c16 = lane & 15;
  const int p0 = blockIdx.x * KT;
  const int nch = (d + DPC - 1) / DPC;
  const int ntiles = (K + KT - 1) / KT, parts = gridDim.y;
  const int tb = (int)((int64_t)ntiles * blockIdx.y / parts);
  const int te = (int)((int64_t)ntiles * (blockIdx.y + 1) / parts);
  const bool v4 = (d & 3) == 0 && reinterpret_cast<uintptr_t>(C) % 16 == 0 &&
                  reinterpret_cast<uintptr_t>(A) % 16 == 0;
  const float eb = 2.f * (float)(d + 4) * kU32;
  // A row of list position k (-1: none)
  auto pid = [&](int k) __attribute__((always_inline)) -> int64_t {
    if constexpr (!LIST) {
      return k < K ? k : -1;
    } else {
      if (k >= np) return -1;
      const int64_t g = plist ? (int64_t)plist[k] : (int64_t)k;
      return g >= 0 && g < arows ? g : -1;
    }
  };
  float pc[4], pn[4];
  int64_t pg[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int k = p0 + 16 * w + 4 * q + v;
    pg[v] = pid(k);
    pc[v] = pg[v] < 0 ? 0.f : (LIST && anorm) ? anorm[k] : cnorm[pg[v]];
    pn[v] = sqrtf(pc[v]);
  }
  float lv[4][M + 1];
  int lj[4][M + 1];
  // thr[v]: a value at or above it cannot be among the p row's M + 1 smallest: the lane's own
  // (M + 1)-th smallest, and the 16 lanes' (M + 1)-th smallest as of the last refresh
  float thr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    thr[v] = kInf;
#pragma unroll
    for (int k = 0; k <= M; ++k) { lv[v][k] = kInf; lj[v][k] = 0x7fffffff; }
  }
  // the (M + 1)-th smallest value held by the 16 lanes of the group, for every p row: M + 1
  // rounds of the group minimum of the lanes' heads (a lane whose head equals it moves on; lanes
  // tying on a value all move, which can only raise the result, so it stays a valid threshold)
  auto refresh = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int head = 0;
      float m = kInf;
#pragma unroll
      for (int k = 0; k <= M; ++k) {
        float h = kInf;
#pragma unroll
        for (int e = 0; e <= M; ++e)
          if (head == e) h = lv[v][e];
        m = h;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) m = fminf(m, __shfl_xor(m, o));
        head += h == m ? 1 : 0;
      }
      thr[v] = fminf(m, lv[v][M]);
    }
  };

  // registers <- one side's chunk: rows r0 .. r0 + 63, dimensions kc .. kc + DPC - 1 (zeros
  // past d and K); LDS <- those registers
  auto load = [&](v4f (&rg)[NF], bool aside, int r0, int kc) __attribute__((always_inline)) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int e = t + 256 * f, row = e / (DPC / 4), c4 = e % (DPC / 4);
      const int64_t g = aside ? pid(r0 + row) : (r0 + row < K ? r0 + row : -1);
      const int k = kc + 4 * c4;
      v4f v = {0.f, 0.f, 0.f, 0.f};
      if (e < F4 && g >= 0) {
        const float* src = (LIST && aside ? A : C) + g * d + k;
        if (v4) {
          if (k < d) v = *reinterpret_cast<const v4f*>(src);
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (k + u < d) v[u] = src[u];
        }
      }
      rg[f] = v;
    }
  };
  auto store = [&](const v4f (&rg)[NF], float* dst) __attribute__((always_inline)) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int e = t + 256 * f, row = e / (DPC / 4), c4 = e % (DPC / 4);
      if (e < F4) *reinterpret_cast<v4f*>(dst + row * LDW + 4 * c4) = rg[f];
    }
  };
  const int steps = (te - tb) * nch;     // (tile, chunk) pairs of the part, tile-major
  v4f ra[NF], rb[NF];
  // squared norms of the lane's columns of a tile (16 b + c16), loaded with its first chunk
  float cn[4], cnext[4];
  auto load_norms = [&](float (&dst)[4], int j0n) __attribute__((always_inline)) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0n + 16 * b + c16;
      dst[b] = j < K ? cnorm[j] : 0.f;
    }
  };
  if (steps > 0) {
    load(ra, true, p0, 0);
    load(rb, false, tb * KT, 0);
    load_norms(cnext, tb * KT);
  }
  float a[DQ];                      // A operand: row 16 w + c16, elements q DQ .. q DQ + DQ - 1
  v4f acc[4];
  for (int u = 0; u < steps; ++u) {
    const int ti = tb + u / nch, ch = u % nch, j0 = ti * KT;
    const bool a_here = nch > 1 || u == 0;          // this step brings a new A chunk
    if (ch == 0) {
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    if (a_here) store(ra, sA);
    store(rb, sB);
    __syncthreads();
    if (a_here) {
#pragma unroll
      for (int m = 0; m < DQ / 4; ++m) {
        const v4f v = *reinterpret_cast<const v4f*>(sA + (16 * w + c16) * LDW + q * DQ + 4 * m);
        a[4 * m] = v.x; a[4 * m + 1] = v.y; a[4 * m + 2] = v.z; a[4 * m + 3] = v.w;
      }
    }
    if (ch == 0) {
#pragma unroll
      for (int b = 0; b < 4; ++b) cn[b] = cnext[b];
    }
    if (u + 1 < steps) {            // the next step's chunks, in flight during these MFMAs
      const int tn = tb + (u + 1) / nch, cc = (u + 1) % nch;
      if (nch > 1) load(ra, true, p0, cc * DPC);
      load(rb, false, tn * KT, cc * DPC);
      if (cc == 0) load_norms(cnext, tn * KT);
    }
#pragma unroll
    for (int m = 0; m < DQ / 4; ++m) {
      v4f bv[4];
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bv[b] = *reinterpret_cast<const v4f*>(sB + (16 * b + c16) * LDW + q * DQ + 4 * m);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * m + e], bv[b][e], acc[b], 0, 0, 0);
    }
    __syncthreads();
    if (ch + 1 < nch) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + 16 * b + c16;
      if (j >= K) continue;
      const float cj = cn[b], nj = sqrtf(cj);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (pg[v] < 0 || ((!LIST || self) && j == pg[v])) continue;
        const float s = pn[v] + nj;
        const float lo = (pc[v] + cj) - 2.f * acc[b][v] - eb * s * s;
        if (lo < thr[v]) {
          // insertion into the ascending list (j increases along the scan, so equal values
          // keep the lower index first)
          float cv = lo;
          int cx = j;
#pragma unroll
          for (int k = 0; k <= M; ++k) {
            const bool sw = cv < lv[v][k];
            const float tvv = sw ? lv[v][k] : cv;
            const int tx = sw ? lj[v][k] : cx;
            lv[v][k] = sw ? cv : lv[v][k];
            lj[v][k] = sw ? cx : lj[v][k];
            cv = tvv;
            cx = tx;
          }
          thr[v] = fminf(thr[v], lv[v][M]);
        }
      }
    }
    if ((ti - tb) % 8 == 7) refresh();   // every 8 tiles (the whole group takes part)
  }

  // merge the 16 lists of each p row: M + 1 rounds, each taking the least (value, index) head
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int p = p0 + 16 * w + 4 * q + v;      // list position
    int head = 0;
#pragma unroll
    for (int k = 0; k <= M; ++k) {
      float h = kInf;
      int hj = 0x7fffffff;
#pragma unroll
      for (int e = 0; e <= M; ++e)
        if (head == e) { h = lv[v][e]; hj = lj[v][e]; }
      float m = h;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) m = fminf(m, __shfl_xor(m, o));
      int mj = h == m ? hj : 0x7fffffff;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) mj = min(mj, __shfl_xor(mj, o));
      head += (h == m && hj == mj) ? 1 : 0;
      if (c16 == 0 && p < np) {
        const int64_t o = ((int64_t)p * parts + blockIdx.y) * (M + 1) + k;
        const bool ok = m < kInf && mj < K;
        tv[o] = ok ? m : kInf;
        tj[o] = ok ? mj : 0x7fffffff;
      }
    }
  }
}

// Per centroid p: the M + 1 smallest (lower value, index) pairs of its parts' lists, by
// insertion; the first M are the neighbours, the (M + 1)-th gives the bound.
// first (nullable): the square root of the smallest lower value, per list position.
template <int M>
__global__ __launch_bounds__(256) void knn_merge_kernel(const float* __restrict__ tv,
                                                        const int32_t* __restrict__ tj, int np,
                                                        int K, int parts, const int32_t* enable,
                                                        int32_t* __restrict__ nbr,
                                                        float* __restrict__ nbr_lb,
                                                        float* __restrict__ first) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= np || (enable && *enable == 0)) return;
  float lv[M + 1];
  int lj[M + 1];
#pragma unroll
  for (int k = 0; k <= M; ++k) { lv[k] = kInf; lj[k] = 0x7fffffff; }
  for (int e = 0; e < parts * (M + 1); ++e) {
    float cv = tv[(int64_t)p * parts * (M + 1) + e];
    int cx = tj[(int64_t)p * parts * (M + 1) + e];
#pragma unroll
    for (int k = 0; k <= M; ++k) {
      const bool sw = cv < lv[k] || (cv == lv[k] && cx < lj[k]);
      const float tvv = sw ? lv[k] : cv;
      const int tx = sw ? lj[k] : cx;
      lv[k] = sw ? cv : lv[k];
      lj[k] = sw ? cx : lj[k];
      cv = tvv;
      cx = tx;
    }
  }
#pragma unroll
  for (int k = 0; k < M; ++k) nbr[(int64_t)p * M + k] = lv[k] < kInf && lj[k] < K ? lj[k] : -1;
  nbr_lb[p] = lv[M] < kInf && lj[M] < K ? sqrtf(fmaxf(lv[M], 0.f)) * (1.f - 4.f * kU32) : kInf;
  if (first) first[p] = lv[0] < kInf && lj[0] < K ? sqrtf(fmaxf(lv[0], 0.f)) : kInf;
}

// Rows of the sample: kBoundSample rows spread evenly over the n (all of them when n is
// smaller), and their squared norms.
__global__ __launch_bounds__(256) void bound_sample_kernel(const float* __restrict__ X, int64_t n,
                                                           int d, int ns,
                                                           int32_t* __restrict__ rows,
                                                           float* __restrict__ xnorm) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= ns) return;
  // (the rows are listed as int32: beyond 2^31 - 1 rows the sample spans the first 2^31 - 1)
  const int64_t span = n < 2147483647 ? n : 2147483647;
  const int64_t i = (int64_t)k * span / ns;
  const float* x = X + i * d;
  float s0 = 0.f;
  for (int m = 0; m < d; ++m) s0 = fmaf(x[m], x[m], s0);
  rows[k] = (int32_t)i;
  xnorm[k] = s0;
}

// The device's decision: build the table when the sample's decided share, scaled to n, exceeds
// payoff rows per centroid (what the table costs in spill-sweep rows).  A sample row counts as
// decided when d1 + sqrt(1 + lambda) d2 (its nearest and second-nearest centroid distances, as
// lowered by the table's rounding margin: an estimate, not a proof) lies below the bound of its
// nearest centroid.
__global__ __launch_bounds__(1024) void bound_estimate_kernel(const float* __restrict__ d1,
                                                              const float* __restrict__ d2,
                                                              const int32_t* __restrict__ near,
                                                              const float* __restrict__ slb,
                                                              int ns, int64_t n, int K, float lam,
                                                              int payoff, int32_t* enable) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int c = 0;
  for (int k = threadIdx.x; k < ns; k += 1024) {
    const int p = near[k];
    c += (p >= 0 && p < K && d1[k] + sqrtf(1.f + lam) * d2[k] < slb[k]) ? 1 : 0;
  }
  atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) enable[0] = (double)cnt * (double)n / ns > (double)payoff * K ? 1 : 0;
}

__global__ void bound_enable_kernel(int32_t* enable) {
  if (threadIdx.x == 0) enable[0] = 1;
}

// Every row: bounded (the primary's neighbours as spill candidates, group key -1) when the table
// was built and the row's radius lies below its primary's bound; else the primary as group key.
template <int M>
__global__ __launch_bounds__(256) void bound_decide_kernel(const int32_t* __restrict__ primary,
                                                           const float* __restrict__ radius,
                                                           int64_t n, int K,
                                                           const int32_t* __restrict__ nbr,
                                                           const float* __restrict__ nbr_lb,
                                                           const int32_t* enable,
                                                           int32_t* __restrict__ cand,
                                                           int32_t* __restrict__ gkey) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int p = primary[i];
  if (p < 0 || p >= K) { gkey[i] = -1; return; }
  if (*enable && radius[i] < nbr_lb[p]) {
#pragma unroll
    for (int k = 0; k < M; ++k) cand[i * M + k] = nbr[(int64_t)p * M + k];
    gkey[i] = -1;
  } else {
    gkey[i] = p;
  }
}

// Parts of the codebook per block of 64 list positions: about 2,048 workgroups in all, at most
// one part per tile, and at most 16 parts for the whole codebook's table (its merge reads
// 16 (M + 1) entries per centroid) or 64 for a sample's (a few hundred positions, so the merge
// stays short, while each workgroup walks few tiles one after another).
int knn_parts(int np, int K) {
  const int ntiles = (K + KT - 1) / KT, nblk = (np + KT - 1) / KT;
  int parts = (2048 + nblk - 1) / nblk;
  if (parts > ntiles) parts = ntiles;
  const int cap = np <= kBoundSample ? 64 : 16;
  if (parts > cap) parts = cap;
  return parts < 1 ? 1 : parts;
}

template <int DQ>
void launch_knn_dq(const float* A, int64_t arows, const float* anorm, int self, const float* C,
                   int K, int d, const float* cnorm, int M, const int32_t* plist, int np,
                   const int32_t* enable, float* tv, int32_t* tj, hipStream_t st) {
  const int parts = knn_parts(np, K);
  const dim3 grid((unsigned)((np + KT - 1) / KT), (unsigned)parts), block(256);
  const bool whole = A == C && !plist && !anorm && self && np == K;
  switch (M) {
#define SOAR_KNN(m)                                                                           \
  case m:                                                                                     \
    if (whole)                                                                                \
      hipLaunchKernelGGL((centroid_knn_kernel<DQ, m, false>), grid, block, 0, st, A, arows,    \
                         anorm, self, C, K, d, cnorm, plist, np, enable, tv, tj);             \
    else                                                                                      \
      hipLaunchKernelGGL((centroid_knn_kernel<DQ, m, true>), grid, block, 0, st, A, arows,     \
                         anorm, self, C, K, d, cnorm, plist, np, enable, tv, tj);             \
    break;
    SOAR_KNN(1) SOAR_KNN(2) SOAR_KNN(3) SOAR_KNN(4) SOAR_KNN(5) SOAR_KNN(6) SOAR_KNN(7)
    SOAR_KNN(8)
#undef SOAR_KNN
    default:
      break;
  }
}

// Nearest centroids of the A rows plist[0 .. np) (plist null: every row), merged into nbr /
// nbr_lb (and the nearest distance into first, when given).
template <int M>
void launch_table(const float* A, int64_t arows, const float* anorm, int self, const float* C,
                  int K, int d, const float* cnorm, const int32_t* plist, int np,
                  const int32_t* enable, float* tv, int32_t* tj, int32_t* nbr, float* nbr_lb,
                  float* first, hipStream_t st) {
  if (d <= 32)
    launch_knn_dq<8>(A, arows, anorm, self, C, K, d, cnorm, M, plist, np, enable, tv, tj, st);
  else if (d <= 64)
    launch_knn_dq<16>(A, arows, anorm, self, C, K, d, cnorm, M, plist, np, enable, tv, tj, st);
  else if (d <= 96)
    launch_knn_dq<24>(A, arows, anorm, self, C, K, d, cnorm, M, plist, np, enable, tv, tj, st);
  else
    launch_knn_dq<32>(A, arows, anorm, self, C, K, d, cnorm, M, plist, np, enable, tv, tj, st);
  hipLaunchKernelGGL(knn_merge_kernel<M>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, tv,
                     tj, np, K, knn_parts(np, K), enable, nbr, nbr_lb, first);
}

template <int M>
void launch_bound_table_m(const float* X, int64_t n, const float* C, int K, int d,
                          const float* cnorm, float lam, const BoundLayout& B, int payoff,
                          hipStream_t st) {
  if (payoff <= 0) {
    // no estimate: the table is built
    hipLaunchKernelGGL(bound_enable_kernel, dim3(1), dim3(64), 0, st, B.enable);
    launch_table<M>(C, K, nullptr, 1, C, K, d, cnorm, nullptr, K, nullptr, B.scratch_v,
                    B.scratch_j, B.nbr, B.nbr_lb, nullptr, st);
    return;
  }
  const int ns = n < kBoundSample ? (int)n : kBoundSample;
  // the sample rows' two nearest centroids, then the bound of the nearest, then the decision
  hipLaunchKernelGGL(bound_sample_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, X,
                     n, d, ns, B.xrows, B.xnorm);
  launch_table<1>(X, n, B.xnorm, 0, C, K, d, cnorm, B.xrows, ns, nullptr, B.scratch_v,
                  B.scratch_j, B.xnear, B.xd2, B.xd1, st);
  launch_table<M>(C, K, nullptr, 1, C, K, d, cnorm, B.xnear, ns, nullptr, B.scratch_v,
                  B.scratch_j, B.snbr, B.slb, nullptr, st);
  hipLaunchKernelGGL(bound_estimate_kernel, dim3(1), dim3(1024), 0, st, B.xd1, B.xd2, B.xnear,
                     B.slb, ns, n, K, lam, payoff, B.enable);
  launch_table<M>(C, K, nullptr, 1, C, K, d, cnorm, nullptr, K, B.enable, B.scratch_v,
                  B.scratch_j, B.nbr, B.nbr_lb, nullptr, st);
}

// Rows left out of the grouping (off[K] of them were grouped): the decided ones and the rows
// without a primary (those have no spill to sweep for either).
__global__ void bound_count_kernel(const int32_t* __restrict__ off, int K, int64_t n,
                                   unsigned* counters) {
  if (threadIdx.x == 0) counters[CNT_BOUNDED] = (unsigned)(n - (int64_t)off[K]);
}

}  // namespace

BoundLayout bound_layout(void* ws, int K, int M) {
  char* b = static_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? b + off : nullptr;
    off = (off + bytes + 255) / 256 * 256;
    return p;
  };
  const size_t ent = (size_t)(M + 1) *
      std::max((size_t)K * knn_parts(K, K), (size_t)kBoundSample * knn_parts(kBoundSample, K));
  BoundLayout L;
  L.nbr = static_cast<int32_t*>(take((size_t)K * M * 4));
  L.nbr_lb = static_cast<float*>(take((size_t)K * 4));
  L.xrows = static_cast<int32_t*>(take((size_t)kBoundSample * 4));
  L.xnorm = static_cast<float*>(take((size_t)kBoundSample * 4));
  L.xnear = static_cast<int32_t*>(take((size_t)kBoundSample * 4));
  L.xd1 = static_cast<float*>(take((size_t)kBoundSample * 4));
  L.xd2 = static_cast<float*>(take((size_t)kBoundSample * 4));
  L.snbr = static_cast<int32_t*>(take((size_t)kBoundSample * M * 4));
  L.slb = static_cast<float*>(take((size_t)kBoundSample * 4));
  L.scratch_v = static_cast<float*>(take(ent * 4));
  L.scratch_j = static_cast<int32_t*>(take(ent * 4));
  L.enable = static_cast<int32_t*>(take(4));
  L.bytes = off;
  return L;
}

hipError_t launch_bound_table(const float* X, int64_t n, const float* C, int K, int d,
                              const float* cnorm, int M, float lam, const BoundLayout& B,
                              int payoff, hipStream_t st) {
  switch (M) {
#define SOAR_BOUND(m)                                                                  \
  case m:                                                                              \
    launch_bound_table_m<m>(X, n, C, K, d, cnorm, lam, B, payoff, st);                 \
    break;
    SOAR_BOUND(1) SOAR_BOUND(2) SOAR_BOUND(3) SOAR_BOUND(4) SOAR_BOUND(5) SOAR_BOUND(6)
    SOAR_BOUND(7) SOAR_BOUND(8)
#undef SOAR_BOUND
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bound_decide(int M, int64_t n, int K, const int32_t* primary,
                               const float* radius, const BoundLayout& B, int32_t* cand,
                               int32_t* gkey, hipStream_t st) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (M) {
#define SOAR_DECIDE(m)                                                                         \
  case m:                                                                                      \
    hipLaunchKernelGGL(bound_decide_kernel<m>, grid, block, 0, st, primary, radius, n, K, B.nbr, \
                       B.nbr_lb, B.enable, cand, gkey);                                        \
    break;
    SOAR_DECIDE(1) SOAR_DECIDE(2) SOAR_DECIDE(3) SOAR_DECIDE(4) SOAR_DECIDE(5) SOAR_DECIDE(6)
    SOAR_DECIDE(7) SOAR_DECIDE(8)
#undef SOAR_DECIDE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bound_count(const int32_t* group_off, int K, int64_t n, unsigned* counters,
                              hipStream_t st) {
  hipLaunchKernelGGL(bound_count_kernel, dim3(1), dim3(64), 0, st, group_off, K, n, counters);
  return hipGetLastError();
}

}  // namespace soar
