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
// other centroids and a lower bound on the distance from c_p to every other centroid.
//
// Distances come from the expansion ||a||^2 + ||b||^2 - 2 <a, b> in FP32.  Its error is at most
// (d + 2) u (||a|| + ||b||)^2 (u = 2^-24: the dot product's and the norms' accumulations and
// the two final roundings), so each value is lowered by twice that before it is ranked: the
// ranked quantity is a proven lower bound of the squared distance, and the (M + 1)-th smallest
// of them bounds every centroid left out.
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
template <int DQ, int M>
__global__ __launch_bounds__(256) void centroid_knn_kernel(const float* __restrict__ C, int K,
                                                           int d, const float* __restrict__ cnorm,
                                                           float* __restrict__ tv,
                                                           int32_t* __restrict__ tj) {
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
  const bool v4 = (d & 3) == 0 && reinterpret_cast<uintptr_t>(C) % 16 == 0;
  const float eb = 2.f * (float)(d + 4) * kU32;
  float pc[4], pn[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int p = p0 + 16 * w + 4 * q + v;
    pc[v] = p < K ? cnorm[p] : 0.f;
    pn[v] = sqrtf(pc[v]);
  }
  float lv[4][M + 1];
  int lj[4][M + 1];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int k = 0; k <= M; ++k) { lv[v][k] = kInf; lj[v][k] = 0x7fffffff; }

  // registers <- one side's chunk: rows r0 .. r0 + 63, dimensions kc .. kc + DPC - 1 (zeros
  // past d and K); LDS <- those registers
  auto load = [&](v4f (&rg)[NF], int r0, int kc) __attribute__((always_inline)) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int e = t + 256 * f, row = e / (DPC / 4), c4 = e % (DPC / 4), g = r0 + row;
      const int k = kc + 4 * c4;
      v4f v = {0.f, 0.f, 0.f, 0.f};
      if (e < F4 && g < K) {
        const float* src = C + (int64_t)g * d + k;
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
  if (steps > 0) {
    load(ra, p0, 0);
    load(rb, tb * KT, 0);
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
    if (u + 1 < steps) {            // the next step's chunks, in flight during these MFMAs
      const int tn = tb + (u + 1) / nch, cn = (u + 1) % nch;
      if (nch > 1) load(ra, p0, cn * DPC);
      load(rb, tn * KT, cn * DPC);
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
      const float cj = cnorm[j], nj = sqrtf(cj);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = p0 + 16 * w + 4 * q + v;
        if (p >= K || j == p) continue;
        const float s = pn[v] + nj;
        const float lo = (pc[v] + cj) - 2.f * acc[b][v] - eb * s * s;
        if (lo < lv[v][M]) {
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
        }
      }
    }
  }

  // merge the 16 lists of each p row: M + 1 rounds, each taking the least (value, index) head
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int p = p0 + 16 * w + 4 * q + v;
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
      if (c16 == 0 && p < K) {
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
template <int M>
__global__ __launch_bounds__(256) void knn_merge_kernel(const float* __restrict__ tv,
                                                        const int32_t* __restrict__ tj, int K,
                                                        int parts, int32_t* __restrict__ nbr,
                                                        float* __restrict__ nbr_lb) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= K) return;
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
}

template <int DQ>
void launch_knn_dq(const float* C, int K, int d, const float* cnorm, int M, float* tv,
                   int32_t* tj, int parts, hipStream_t st) {
  const dim3 grid((unsigned)((K + KT - 1) / KT), (unsigned)parts), block(256);
  switch (M) {
#define SOAR_KNN(m)                                                                         \
  case m:                                                                                   \
    hipLaunchKernelGGL((centroid_knn_kernel<DQ, m>), grid, block, 0, st, C, K, d, cnorm, tv, tj); \
    break;
    SOAR_KNN(1) SOAR_KNN(2) SOAR_KNN(3) SOAR_KNN(4) SOAR_KNN(5) SOAR_KNN(6) SOAR_KNN(7)
    SOAR_KNN(8)
#undef SOAR_KNN
    default:
      break;
  }
}

// Rows left out of the grouping (off[K] of them were grouped) are the bounded ones, except rows
// without a primary, which the caller counts as bounded too (they have no spill to sweep for).
__global__ void bound_count_kernel(const int32_t* __restrict__ off, int K, int64_t n,
                                   unsigned* counters) {
  if (threadIdx.x == 0) counters[CNT_BOUNDED] = (unsigned)(n - (int64_t)off[K]);
}

}  // namespace

hipError_t launch_bound_count(const int32_t* group_off, int K, int64_t n, unsigned* counters,
                              hipStream_t st) {
  hipLaunchKernelGGL(bound_count_kernel, dim3(1), dim3(64), 0, st, group_off, K, n, counters);
  return hipGetLastError();
}

int knn_parts(int K) {
  // enough (p block, part) workgroups to fill the chip a few times over: about 2,048 of them,
  // at most one part per tile and 32 parts
  const int ntiles = (K + KT - 1) / KT;
  int parts = (2048 + ntiles - 1) / ntiles;
  if (parts > ntiles) parts = ntiles;
  return parts < 1 ? 1 : (parts > 32 ? 32 : parts);
}

size_t knn_scratch_entries(int K) { return (size_t)K * knn_parts(K) * (kBoundMaxM + 1); }

hipError_t launch_centroid_knn(const float* C, int K, int d, const float* cnorm, int M,
                               float* scratch_v, int32_t* scratch_j, int32_t* nbr, float* nbr_lb,
                               hipStream_t st) {
  if (M < 1 || M > kBoundMaxM) return hipErrorInvalidValue;
  const int parts = knn_parts(K);
  // chunk width: the row padded to 32, 64 or 96 dimensions, else chunks of 128
  if (d <= 32) launch_knn_dq<8>(C, K, d, cnorm, M, scratch_v, scratch_j, parts, st);
  else if (d <= 64) launch_knn_dq<16>(C, K, d, cnorm, M, scratch_v, scratch_j, parts, st);
  else if (d <= 96) launch_knn_dq<24>(C, K, d, cnorm, M, scratch_v, scratch_j, parts, st);
  else launch_knn_dq<32>(C, K, d, cnorm, M, scratch_v, scratch_j, parts, st);
  const dim3 grid((unsigned)((K + 255) / 256)), block(256);
  switch (M) {
#define SOAR_MERGE(m)                                                                        \
  case m:                                                                                    \
    hipLaunchKernelGGL(knn_merge_kernel<m>, grid, block, 0, st, scratch_v, scratch_j, K, parts, \
                       nbr, nbr_lb);                                                         \
    break;
    SOAR_MERGE(1) SOAR_MERGE(2) SOAR_MERGE(3) SOAR_MERGE(4) SOAR_MERGE(5) SOAR_MERGE(6)
    SOAR_MERGE(7) SOAR_MERGE(8)
#undef SOAR_MERGE
    default:
      break;
  }
  return hipGetLastError();
}

}  // namespace soar
