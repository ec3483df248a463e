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

constexpr int KT = 64;        // centroids per tile, on both sides
constexpr int KC = 32;        // dimensions per LDS chunk
constexpr int KCP = KC + 4;   // padded LDS row (floats): 16-byte aligned, fewer bank conflicts

// One workgroup per 64 centroids p; the codebook streams through LDS in tiles of 64 centroids j
// and chunks of 32 dimensions.  Thread (tp, tj) computes the 4 x 4 products of p rows 4 tp + a
// and j rows 4 tj + b, and keeps, for each of its four p, the M + 1 smallest lower values it saw
// (ascending).  The 16 threads of one tp are one 16-lane group; their lists are merged at the end.
template <int M>
__global__ __launch_bounds__(256) void centroid_knn_kernel(const float* __restrict__ C, int K,
                                                           int d, const float* __restrict__ cnorm,
                                                           int32_t* __restrict__ nbr,
                                                           float* __restrict__ nbr_lb) {
  __shared__ __attribute__((aligned(16))) float sp[KT * KCP];
  __shared__ __attribute__((aligned(16))) float sj[KT * KCP];
  const int t = threadIdx.x, tj = t & 15, tp = t >> 4;
  const int p0 = blockIdx.x * KT;
  const float eb = 2.f * (float)(d + 4) * kU32;
  float pc[4], pn[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int p = p0 + 4 * tp + a;
    pc[a] = p < K ? cnorm[p] : 0.f;
    pn[a] = sqrtf(pc[a]);
  }
  float lv[4][M + 1];
  int lj[4][M + 1];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q <= M; ++q) { lv[a][q] = kInf; lj[a][q] = 0x7fffffff; }

  const bool v4 = (d & 3) == 0 && reinterpret_cast<uintptr_t>(C) % 16 == 0;
  for (int j0 = 0; j0 < K; j0 += KT) {
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
    for (int k0 = 0; k0 < d; k0 += KC) {
      // 64 rows x 8 float4 per side: two per thread; eight threads read one row's 128 bytes
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = t + 256 * h, row = e >> 3, k = k0 + 4 * (e & 7);
        const int gp = p0 + row, gj = j0 + row;
        v4f vp = {0.f, 0.f, 0.f, 0.f}, vj = {0.f, 0.f, 0.f, 0.f};
        if (v4) {
          if (gp < K && k < d) vp = *reinterpret_cast<const v4f*>(C + (int64_t)gp * d + k);
          if (gj < K && k < d) vj = *reinterpret_cast<const v4f*>(C + (int64_t)gj * d + k);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (gp < K && k + q < d) vp[q] = C[(int64_t)gp * d + k + q];
            if (gj < K && k + q < d) vj[q] = C[(int64_t)gj * d + k + q];
          }
        }
        *reinterpret_cast<v4f*>(sp + row * KCP + 4 * (e & 7)) = vp;
        *reinterpret_cast<v4f*>(sj + row * KCP + 4 * (e & 7)) = vj;
      }
      __syncthreads();
#pragma unroll
      for (int k4 = 0; k4 < KC / 4; ++k4) {
        v4f av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          av[a] = *reinterpret_cast<const v4f*>(sp + (4 * tp + a) * KCP + 4 * k4);
#pragma unroll
        for (int b = 0; b < 4; ++b)
          bv[b] = *reinterpret_cast<const v4f*>(sj + (4 * tj + b) * KCP + 4 * k4);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            acc[a][b] = fmaf(av[a].x, bv[b].x, acc[a][b]);
            acc[a][b] = fmaf(av[a].y, bv[b].y, acc[a][b]);
            acc[a][b] = fmaf(av[a].z, bv[b].z, acc[a][b]);
            acc[a][b] = fmaf(av[a].w, bv[b].w, acc[a][b]);
          }
      }
      __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = j0 + 4 * tj + b;
      if (j >= K) continue;
      const float cj = cnorm[j], nj = sqrtf(cj);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int p = p0 + 4 * tp + a;
        if (p >= K || j == p) continue;
        const float s = pn[a] + nj;
        const float lo = (pc[a] + cj) - 2.f * acc[a][b] - eb * s * s;
        if (lo < lv[a][M]) {
          // insertion into the ascending list (j increases along the scan, so equal values
          // keep the lower index first)
          float cv = lo;
          int cx = j;
#pragma unroll
          for (int q = 0; q <= M; ++q) {
            const bool sw = cv < lv[a][q];
            const float tv = sw ? lv[a][q] : cv;
            const int tx = sw ? lj[a][q] : cx;
            lv[a][q] = sw ? cv : lv[a][q];
            lj[a][q] = sw ? cx : lj[a][q];
            cv = tv;
            cx = tx;
          }
        }
      }
    }
  }

  // merge the 16 lists of each p: M + 1 rounds, each taking the least (value, index) head
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int p = p0 + 4 * tp + a;
    int head = 0;
#pragma unroll
    for (int k = 0; k <= M; ++k) {
      float h = kInf;
      int hj = 0x7fffffff;
#pragma unroll
      for (int q = 0; q <= M; ++q)
        if (head == q) { h = lv[a][q]; hj = lj[a][q]; }
      float m = h;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) m = fminf(m, __shfl_xor(m, o));
      int mj = h == m ? hj : 0x7fffffff;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) mj = min(mj, __shfl_xor(mj, o));
      head += (h == m && hj == mj) ? 1 : 0;
      if (tj == 0 && p < K) {
        const bool ok = m < kInf && mj < K;
        if (k < M) nbr[(int64_t)p * M + k] = ok ? mj : -1;
        else nbr_lb[p] = ok ? sqrtf(fmaxf(m, 0.f)) * (1.f - 4.f * kU32) : kInf;
      }
    }
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

hipError_t launch_centroid_knn(const float* C, int K, int d, const float* cnorm, int M,
                               int32_t* nbr, float* nbr_lb, hipStream_t st) {
  const dim3 grid((unsigned)((K + KT - 1) / KT)), block(256);
  switch (M) {
#define SOAR_KNN(m)                                                                            \
  case m:                                                                                      \
    hipLaunchKernelGGL(centroid_knn_kernel<m>, grid, block, 0, st, C, K, d, cnorm, nbr, nbr_lb); \
    break;
    SOAR_KNN(1) SOAR_KNN(2) SOAR_KNN(3) SOAR_KNN(4) SOAR_KNN(5) SOAR_KNN(6) SOAR_KNN(7)
    SOAR_KNN(8)
#undef SOAR_KNN
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace soar
