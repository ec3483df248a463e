// Grouping of rows by their primary partition, for the grouped form of the spill sweep.
//
// The spill loss of row i against centroid j needs <r_i, c_j> = <x_i, c_j> - <c_pi, c_j>
// (Section 3.4, with r = x - c_pi).  When the 16 rows of an MFMA tile share their primary p, the
// second term is one more row of the same product: the tile takes 15 rows of partition p and, as
// its 16th row, c_p itself, so one MFMA stream yields both <x_i, c_j> and <c_p, c_j>.  This file
// builds that layout:
//   cnt[p]     rows with primary p (rows without a valid primary are left out)
//   off[p]     exclusive prefix of cnt: partition p's rows are perm[off[p] .. off[p] + cnt[p])
//   perm[]     row ids grouped by primary (order inside a partition is not specified; no result
//              depends on it, since every row's values are computed independently)
//   sbeg[p]    exclusive prefix of ceil(cnt[p] / 15): partition p's first stripe
//   stripes[s] {p, first position in perm, rows (1..15)}
//   meta[0]    number of stripes
#include "common.h"
#include "kernels.h"

namespace soar {

namespace {

__global__ void group_fill_kernel(int32_t* p, int64_t count, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void group_hist_kernel(const int32_t* __restrict__ prim,
                                                         int64_t cap, const int64_t* live,
                                                         int K, int32_t* cnt) {
  const int64_t n = live_rows(cap, live);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = prim[i];
    if (p >= 0 && p < K) atomicAdd(&cnt[p], 1);
  }
}

// Exclusive scans of cnt and of ceil(cnt / 15), in chunks of 1024 (one workgroup).
__global__ __launch_bounds__(1024) void group_scan_kernel(const int32_t* __restrict__ cnt, int K,
                                                          int32_t* off, int32_t* sbeg,
                                                          int32_t* meta) {
  __shared__ int32_t a[1024], b[1024];
  __shared__ int32_t carry_a, carry_b;
  const int t = threadIdx.x;
  if (t == 0) { carry_a = 0; carry_b = 0; }
  __syncthreads();
  for (int base = 0; base < K; base += 1024) {
    const int c = base + t < K ? cnt[base + t] : 0;
    a[t] = c;
    b[t] = (c + GROUP_ROWS - 1) / GROUP_ROWS;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scans
      const int32_t va = t >= o ? a[t - o] : 0, vb = t >= o ? b[t - o] : 0;
      __syncthreads();
      a[t] += va;
      b[t] += vb;
      __syncthreads();
    }
    if (base + t < K) {
      off[base + t] = carry_a + a[t] - c;
      sbeg[base + t] = carry_b + b[t] - (c + GROUP_ROWS - 1) / GROUP_ROWS;
    }
    __syncthreads();
    if (t == 1023) { carry_a += a[1023]; carry_b += b[1023]; }
    __syncthreads();
  }
  if (t == 0) {
    off[K] = carry_a;
    sbeg[K] = carry_b;
    meta[0] = carry_b;
  }
}

__global__ __launch_bounds__(256) void group_scatter_kernel(const int32_t* __restrict__ prim,
                                                            int64_t cap, const int64_t* live,
                                                            int K, const int32_t* __restrict__ off,
                                                            int32_t* cursor, int32_t* perm) {
  const int64_t n = live_rows(cap, live);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = prim[i];
    if (p >= 0 && p < K) perm[off[p] + atomicAdd(&cursor[p], 1)] = (int32_t)i;
  }
}

// One thread per stripe; its partition is the last p with sbeg[p] <= s (binary search).
__global__ __launch_bounds__(256) void group_stripes_kernel(const int32_t* __restrict__ cnt,
                                                            const int32_t* __restrict__ off,
                                                            const int32_t* __restrict__ sbeg,
                                                            int K, const int32_t* meta,
                                                            int64_t max_stripes, int4* stripes) {
  const int ns = meta[0];
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < ns && s < max_stripes;
       s += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = K - 1;               // sbeg[lo] <= s < sbeg[hi + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sbeg[mid] <= s) lo = mid; else hi = mid - 1;
    }
    const int p = lo, k = (int)(s - sbeg[p]), c = cnt[p];
    const int rows = c - k * GROUP_ROWS < GROUP_ROWS ? c - k * GROUP_ROWS : GROUP_ROWS;
    stripes[s] = int4{p, off[p] + k * GROUP_ROWS, rows, 0};
  }
}

// Histogram and scatter with per-block counts in LDS (K <= GROUP_LDS_K): one global atomic per
// block and partition instead of one per row, so rows piling onto a few partitions do not
// serialize on their counters.
constexpr int GROUP_LDS_K = 16384;
constexpr int GROUP_ROWS_PER_BLOCK = 8192;

__global__ __launch_bounds__(1024) void group_hist_lds_kernel(const int32_t* __restrict__ prim,
                                                              int64_t cap, const int64_t* live,
                                                              int K, int32_t* cnt) {
  __shared__ int32_t h[GROUP_LDS_K];
  const int64_t n = live_rows(cap, live);
  const int64_t r0 = (int64_t)blockIdx.x * GROUP_ROWS_PER_BLOCK;
  if (r0 >= n) return;
  for (int p = threadIdx.x; p < K; p += 1024) h[p] = 0;
  __syncthreads();
  const int64_t r1 = r0 + GROUP_ROWS_PER_BLOCK < n ? r0 + GROUP_ROWS_PER_BLOCK : n;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 1024) {
    const int p = prim[i];
    if (p >= 0 && p < K) atomicAdd(&h[p], 1);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < K; p += 1024)
    if (h[p]) atomicAdd(&cnt[p], h[p]);
}

__global__ __launch_bounds__(1024) void group_scatter_lds_kernel(
    const int32_t* __restrict__ prim, int64_t cap, const int64_t* live, int K,
    const int32_t* __restrict__ off, int32_t* cursor, int32_t* perm) {
  __shared__ int32_t h[GROUP_LDS_K];      // block counts, then the block's first position
  __shared__ int32_t c2[GROUP_LDS_K];     // running position inside the block's range
  const int64_t n = live_rows(cap, live);
  const int64_t r0 = (int64_t)blockIdx.x * GROUP_ROWS_PER_BLOCK;
  if (r0 >= n) return;
  for (int p = threadIdx.x; p < K; p += 1024) { h[p] = 0; c2[p] = 0; }
  __syncthreads();
  const int64_t r1 = r0 + GROUP_ROWS_PER_BLOCK < n ? r0 + GROUP_ROWS_PER_BLOCK : n;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 1024) {
    const int p = prim[i];
    if (p >= 0 && p < K) atomicAdd(&h[p], 1);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < K; p += 1024)
    if (h[p]) h[p] = off[p] + atomicAdd(&cursor[p], h[p]);
  __syncthreads();
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 1024) {
    const int p = prim[i];
    if (p >= 0 && p < K) perm[h[p] + atomicAdd(&c2[p], 1)] = (int32_t)i;
  }
}

inline unsigned grid_rows(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

int64_t group_max_stripes(int64_t n, int K) {
  return (n + GROUP_ROWS - 1) / GROUP_ROWS + (n < K ? n : (int64_t)K);
}

GroupLayout group_layout(void* ws, int64_t n, int K) {
  char* b = static_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? b + off : nullptr;
    off = (off + bytes + 255) / 256 * 256;
    return p;
  };
  GroupLayout L;
  L.cnt = static_cast<int32_t*>(take((size_t)K * 4));
  L.cursor = static_cast<int32_t*>(take((size_t)K * 4));
  L.off = static_cast<int32_t*>(take((size_t)(K + 1) * 4));
  L.sbeg = static_cast<int32_t*>(take((size_t)(K + 1) * 4));
  L.meta = static_cast<int32_t*>(take(64));
  L.perm = static_cast<int32_t*>(take((size_t)n * 4));
  L.stripes = static_cast<int4*>(take((size_t)group_max_stripes(n, K) * 16));
  L.bytes = off;
  return L;
}

hipError_t launch_group_by_primary(const int32_t* prim, int64_t cap, const int64_t* live_n, int K,
                                   const GroupLayout& L, hipStream_t st) {
  const unsigned gk = (unsigned)((K + 255) / 256);
  hipLaunchKernelGGL(group_fill_kernel, dim3(gk), dim3(256), 0, st, L.cnt, (int64_t)K, 0);
  hipLaunchKernelGGL(group_fill_kernel, dim3(gk), dim3(256), 0, st, L.cursor, (int64_t)K, 0);
  const bool lds = K <= GROUP_LDS_K;
  const unsigned gb = (unsigned)((cap + GROUP_ROWS_PER_BLOCK - 1) / GROUP_ROWS_PER_BLOCK);
  if (lds)
    hipLaunchKernelGGL(group_hist_lds_kernel, dim3(gb > 0 ? gb : 1), dim3(1024), 0, st, prim, cap,
                       live_n, K, L.cnt);
  else
    hipLaunchKernelGGL(group_hist_kernel, dim3(grid_rows(cap)), dim3(256), 0, st, prim, cap,
                       live_n, K, L.cnt);
  hipLaunchKernelGGL(group_scan_kernel, dim3(1), dim3(1024), 0, st, L.cnt, K, L.off, L.sbeg,
                     L.meta);
  if (lds)
    hipLaunchKernelGGL(group_scatter_lds_kernel, dim3(gb > 0 ? gb : 1), dim3(1024), 0, st, prim,
                       cap, live_n, K, L.off, L.cursor, L.perm);
  else
    hipLaunchKernelGGL(group_scatter_kernel, dim3(grid_rows(cap)), dim3(256), 0, st, prim, cap,
                       live_n, K, L.off, L.cursor, L.perm);
  const int64_t ms = group_max_stripes(cap, K);
  hipLaunchKernelGGL(group_stripes_kernel, dim3(grid_rows(ms)), dim3(256), 0, st, L.cnt, L.off,
                     L.sbeg, K, L.meta, ms, L.stripes);
  return hipGetLastError();
}

}  // namespace soar
