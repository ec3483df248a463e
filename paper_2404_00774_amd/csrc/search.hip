// Query-side probing over the SOAR inverted lists (Section 2.2's VQ search; the spilled copies of
// Section 3.5 are listed in a second partition and counted once).
//
//   lists   CSR inverted lists from the assignment arrays: offsets[K + 1], ids[] (a point spilled
//           into a second partition appears in both lists).  Counting sort on the GPU.
//   probe   per query, <q, c_j> for every partition in FP64 (products of FP32 inputs are exact in
//           FP64), then a stable descending segmented radix sort: the best t partitions, equal
//           scores to the lower index.
//   rerank  one workgroup per query walks the t probed lists; every candidate gets its exact
//           <q, x> (FP64 accumulation, one fixed order, so a point reached through two lists gets
//           the same value twice); each thread keeps its k best (score, then id) without
//           repeats, and k rounds of a workgroup arg-max over the threads' lists yield the k
//           best distinct ids.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "../../include/soar.h"
#include "common.h"

namespace soar {
namespace {

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

constexpr int kSearchMaxK = 16;      // results per query
constexpr int kRerankThreads = 256;

__global__ void list_hist_kernel(const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                                 int64_t n, int K, int64_t* cnt, unsigned* bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = a[i];
    if (p >= 0 && p < K) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[p]), 1ull);
    else atomicOr(bad, 1u);
    if (b) {
      const int s = b[i];
      if (s >= 0 && s < K) atomicAdd(reinterpret_cast<unsigned long long*>(&cnt[s]), 1ull);
      else atomicOr(bad, 1u);
    }
  }
}

// Exclusive scan of cnt[0..K) into off[0..K], one workgroup of 1024 threads, chunk by chunk.
__global__ __launch_bounds__(1024) void list_scan_kernel(const int64_t* __restrict__ cnt, int K,
                                                         int64_t* off, int64_t* cursor) {
  __shared__ int64_t s[1024];
  int64_t carry = 0;
  for (int base = 0; base < K; base += 1024) {
    const int j = base + (int)threadIdx.x;
    const int64_t v = j < K ? cnt[j] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t add = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    if (j < K) {
      off[j] = carry + s[threadIdx.x] - v;
      cursor[j] = off[j];
    }
    carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) off[K] = carry;
}

__global__ void list_fill_kernel(const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                                 int64_t n, int K, int64_t* cursor, int32_t* ids) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = a[i];
    if (p >= 0 && p < K)
      ids[atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[p]), 1ull)] = (int32_t)i;
    if (b) {
      const int s = b[i];
      if (s >= 0 && s < K)
        ids[atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[s]), 1ull)] = (int32_t)i;
    }
  }
}

__global__ void zero_i64_kernel(int64_t* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// <q, c_j> in FP64 for the queries of a chunk: keys[(q - q0) * K + j], vals[...] = j, and the
// segment bounds of the sort.  A workgroup takes kPQ queries x kPC centroids; both go through LDS
// kPD dimensions at a time in whole-row coalesced loads, and every (query, centroid) pair is
// accumulated by one thread in dimension order: the sequential FP64 sum of the definition.
constexpr int kPQ = 16, kPC = 64, kPD = 64;

__global__ __launch_bounds__(256) void probe_scores_kernel(const float* __restrict__ Q, int64_t q0,
                                                           int nqc, int d,
                                                           const float* __restrict__ C, int K,
                                                           double* keys, int32_t* vals, int* seg) {
  __shared__ float sq[kPQ][kPD + 1];
  __shared__ float sc[kPC][kPD + 1];
  const int tid = threadIdx.x;
  const int j0 = blockIdx.x * kPC, qb = blockIdx.y * kPQ;
  if (blockIdx.x == 0 && tid < kPQ) {
    const int qq = qb + tid;
    if (qq < nqc) seg[qq] = qq * K;
    if (qq == nqc - 1) seg[nqc] = nqc * K;
  }
  const int ql = tid >> 4, cl = tid & 15;   // query ql, centroids cl + 16 m
  double acc[kPC / 16];
#pragma unroll
  for (int m = 0; m < kPC / 16; ++m) acc[m] = 0.0;
  for (int k0 = 0; k0 < d; k0 += kPD) {
    const int kw = min(kPD, d - k0);
    for (int i = tid; i < kPQ * kPD; i += 256) {
      const int r = i / kPD, c = i % kPD, qq = qb + r;
      sq[r][c] = (qq < nqc && c < kw) ? Q[(q0 + qq) * (int64_t)d + k0 + c] : 0.f;
    }
    for (int i = tid; i < kPC * kPD; i += 256) {
      const int r = i / kPD, c = i % kPD, jj = j0 + r;
      sc[r][c] = (jj < K && c < kw) ? C[(int64_t)jj * d + k0 + c] : 0.f;
    }
    __syncthreads();
    for (int c = 0; c < kw; ++c) {
      const double qv = (double)sq[ql][c];
#pragma unroll
      for (int m = 0; m < kPC / 16; ++m) acc[m] = fma(qv, (double)sc[cl + 16 * m][c], acc[m]);
    }
    __syncthreads();
  }
  const int qq = qb + ql;
  if (qq >= nqc) return;
#pragma unroll
  for (int m = 0; m < kPC / 16; ++m) {
    const int jj = j0 + cl + 16 * m;
    if (jj < K) {
      keys[(int64_t)qq * K + jj] = acc[m] + 0.0;   // -0 becomes +0, so equal scores sort as equal
      vals[(int64_t)qq * K + jj] = jj;
    }
  }
}

// (score, id) order of the results: higher score first, then lower id.
__device__ __forceinline__ bool better(double s, int i, double t, int j) {
  return s > t || (s == t && i < j);
}

// One workgroup per query of the chunk: scan the t probed lists, keep the k best distinct ids.
// The lists are taken kRerankThreads points at a time; their rows go through LDS kRD dimensions
// at a time (coalesced), and each thread accumulates its point's <q, x> in dimension order (FP64),
// so a point reached through two lists gets the same value twice.  Each thread keeps its
// kSearchMaxK best without repeats; k rounds of a workgroup arg-max then take the k best distinct
// ids (a point held by two threads is taken once: every holder moves past it).
constexpr int kRD = 32;

__device__ __forceinline__ void wave_best(double& s, int& i) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double os = __shfl_xor(s, off);
    const int oi = __shfl_xor(i, off);
    if (better(os, oi, s, i)) { s = os; i = oi; }
  }
}

__global__ __launch_bounds__(kRerankThreads) void rerank_kernel(
    const float* __restrict__ Q, int64_t q0, int d, const float* __restrict__ X,
    const int64_t* __restrict__ off, const int32_t* __restrict__ ids,
    const int32_t* __restrict__ order, int K, int t, int k, int32_t* out_ids, double* out_scores,
    int64_t* searched) {
  __shared__ float s_rows[kRerankThreads][kRD + 1];
  __shared__ float s_q[kRD];
  __shared__ double s_ws[kRerankThreads / 64];
  __shared__ int s_wi[kRerankThreads / 64];
  const int qi = blockIdx.x;
  const int64_t qg = q0 + qi;
  const float* q = Q + qg * (int64_t)d;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int64_t count = 0;
  // the thread's kSearchMaxK best, best first (empty places: -inf and id INT_MAX)
  double sc[kSearchMaxK];
  int id_[kSearchMaxK];
#pragma unroll
  for (int m = 0; m < kSearchMaxK; ++m) { sc[m] = -__builtin_inf(); id_[m] = 0x7fffffff; }
  for (int r = 0; r < t; ++r) {
    const int p = order[(int64_t)qi * K + r];
    const int64_t b = off[p], e = off[p + 1];
    count += e - b;
    for (int64_t base = b; base < e; base += kRerankThreads) {
      const int nb = (int)min<int64_t>(kRerankThreads, e - base);
      const bool mine = tid < nb;
      const int x = mine ? ids[base + tid] : 0;
      double s = 0.0;
      for (int k0 = 0; k0 < d; k0 += kRD) {
        const int kw = min(kRD, d - k0);
        // rows of the batch: 8 lanes per row, 4 floats each (zeros past d and past the batch)
        for (int i = tid; i < kRerankThreads * (kRD / 4); i += kRerankThreads) {
          const int rr = i / (kRD / 4), c4 = (i % (kRD / 4)) * 4;
          float v[4] = {0.f, 0.f, 0.f, 0.f};
          if (rr < nb) {
            const float* xr = X + (int64_t)ids[base + rr] * d + k0;
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (c4 + u < kw) v[u] = xr[c4 + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) s_rows[rr][c4 + u] = v[u];
        }
        if (tid < kRD) s_q[tid] = tid < kw ? q[k0 + tid] : 0.f;
        __syncthreads();
        for (int c = 0; c < kw; ++c) s = fma((double)s_q[c], (double)s_rows[tid][c], s);
        __syncthreads();
      }
      s += 0.0;
      // enters only if better than the current last and not already held
      if (!mine || !better(s, x, sc[kSearchMaxK - 1], id_[kSearchMaxK - 1])) continue;
      bool held = false;
#pragma unroll
      for (int m = 0; m < kSearchMaxK; ++m) held |= id_[m] == x;
      if (held) continue;
      double cs = s;
      int ci = x;
#pragma unroll
      for (int m = 0; m < kSearchMaxK; ++m) {
        if (better(cs, ci, sc[m], id_[m])) {
          const double ts = sc[m];
          const int ti = id_[m];
          sc[m] = cs;
          id_[m] = ci;
          cs = ts;
          ci = ti;
        }
      }
    }
  }
  // k rounds of a workgroup arg-max over the threads' heads
  int h = 0;
  for (int r = 0; r < k; ++r) {
    double bs = -__builtin_inf();
    int bi = 0x7fffffff;
#pragma unroll
    for (int m = 0; m < kSearchMaxK; ++m)
      if (h == m) { bs = sc[m]; bi = id_[m]; }
    wave_best(bs, bi);
    if (lane == 0) { s_ws[w] = bs; s_wi[w] = bi; }
    __syncthreads();
    double ws = s_ws[0];
    int wi = s_wi[0];
#pragma unroll
    for (int v = 1; v < kRerankThreads / 64; ++v)
      if (better(s_ws[v], s_wi[v], ws, wi)) { ws = s_ws[v]; wi = s_wi[v]; }
    __syncthreads();
    int hid = 0x7fffffff;
#pragma unroll
    for (int m = 0; m < kSearchMaxK; ++m)
      if (h == m) hid = id_[m];
    if (wi != 0x7fffffff && hid == wi) ++h;
    if (tid == 0) {
      const bool got = wi != 0x7fffffff && ws > -__builtin_inf();
      out_ids[qg * k + r] = got ? wi : -1;
      out_scores[qg * k + r] = got ? ws : -__builtin_inf();
    }
  }
  if (tid == 0 && searched) searched[qg] = count;
}

struct SearchLayout {
  double* keys_in;
  double* keys_out;
  int32_t* vals_in;
  int32_t* vals_out;
  int* seg;
  void* temp;
  size_t temp_bytes;
  size_t bytes;
  int nqc;
};

SearchLayout search_layout(void* ws, int64_t nq, int K) {
  SearchLayout L{};
  // queries per chunk: about 256 MB of sort keys and values
  const int64_t per_q = (int64_t)K * 24;
  L.nqc = (int)std::max<int64_t>(
      1, std::min<int64_t>(std::min<int64_t>(nq, 65535), ((int64_t)256 << 20) / per_q));
  const int64_t items = (int64_t)L.nqc * K;
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t b) { char* p = base ? base + off : nullptr; off = al(off + b); return p; };
  L.keys_in = reinterpret_cast<double*>(take(items * 8));
  L.keys_out = reinterpret_cast<double*>(take(items * 8));
  L.vals_in = reinterpret_cast<int32_t*>(take(items * 4));
  L.vals_out = reinterpret_cast<int32_t*>(take(items * 4));
  L.seg = reinterpret_cast<int*>(take((size_t)(L.nqc + 1) * 4));
  size_t tb = 0;
  (void)hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
      nullptr, tb, L.keys_in, L.keys_out, L.vals_in, L.vals_out, (int)items, L.nqc, L.seg,
      L.seg + 1);
  L.temp_bytes = tb;
  L.temp = take(tb);
  L.bytes = off;
  return L;
}

}  // namespace
}  // namespace soar

using namespace soar;

extern "C" {

soar_status soar_lists_workspace_size(int64_t n, int32_t K, size_t* bytes) {
  if (!bytes || n < 1 || K < 1) return SOAR_E_INVAL;
  *bytes = al((size_t)K * 8) * 2 + al(64);
  return SOAR_OK;
}

soar_status soar_lists_build(const int32_t* primary, const int32_t* spill, int64_t n, int32_t K,
                             int64_t* offsets, int32_t* ids, void* workspace, size_t ws_bytes,
                             void* stream) {
  size_t need = 0;
  if (!primary || !offsets || !ids || !workspace ||
      soar_lists_workspace_size(n, K, &need) != SOAR_OK || ws_bytes < need ||
      n > INT32_MAX)
    return SOAR_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(workspace);
  int64_t* cnt = reinterpret_cast<int64_t*>(w);
  int64_t* cursor = reinterpret_cast<int64_t*>(w + al((size_t)K * 8));
  unsigned* bad = reinterpret_cast<unsigned*>(w + 2 * al((size_t)K * 8));
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(zero_i64_kernel, dim3((K + 255) / 256 + 1), dim3(256), 0, st, cnt,
                     (int64_t)K);
  hipLaunchKernelGGL(zero_i64_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<int64_t*>(bad),
                     (int64_t)1);
  hipLaunchKernelGGL(list_hist_kernel, dim3(g), dim3(256), 0, st, primary, spill, n, K, cnt, bad);
  hipLaunchKernelGGL(list_scan_kernel, dim3(1), dim3(1024), 0, st, cnt, K, offsets, cursor);
  hipLaunchKernelGGL(list_fill_kernel, dim3(g), dim3(256), 0, st, primary, spill, n, K, cursor,
                     ids);
  unsigned hbad = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SOAR_E_DEVICE;
  return hbad ? SOAR_E_INVAL : SOAR_OK;
}

soar_status soar_search_workspace_size(int64_t nq, int32_t d, int32_t K, size_t* bytes) {
  if (!bytes || nq < 1 || d < 1 || K < 1) return SOAR_E_INVAL;
  *bytes = search_layout(nullptr, nq, K).bytes;
  return SOAR_OK;
}

soar_status soar_search(const float* Q, int64_t nq, int32_t d, const float* C, int32_t K,
                        const float* X, int64_t n, const int64_t* offsets, const int32_t* ids,
                        int32_t t, int32_t k, int32_t* out_ids, double* out_scores,
                        int64_t* searched, void* workspace, size_t ws_bytes, void* stream) {
  size_t need = 0;
  if (!Q || !C || !X || !offsets || !ids || !out_ids || !out_scores || !workspace || n < 1 ||
      t < 1 || k < 1 || k > kSearchMaxK || soar_search_workspace_size(nq, d, K, &need) != SOAR_OK ||
      ws_bytes < need)
    return SOAR_E_INVAL;
  t = std::min(t, K);
  hipStream_t st = static_cast<hipStream_t>(stream);
  SearchLayout L = search_layout(workspace, nq, K);
  for (int64_t q0 = 0; q0 < nq; q0 += L.nqc) {
    const int nqc = (int)std::min<int64_t>(L.nqc, nq - q0);
    hipLaunchKernelGGL(probe_scores_kernel, dim3((K + kPC - 1) / kPC, (nqc + kPQ - 1) / kPQ),
                       dim3(256), 0, st, Q, q0, nqc, d, C, K, L.keys_in, L.vals_in, L.seg);
    size_t tb = L.temp_bytes;
    if (hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
            L.temp, tb, L.keys_in, L.keys_out, L.vals_in, L.vals_out, nqc * K, nqc, L.seg,
            L.seg + 1, 0, 64, st) != hipSuccess)
      return SOAR_E_DEVICE;
    hipLaunchKernelGGL(rerank_kernel, dim3(nqc), dim3(kRerankThreads), 0, st, Q, q0, d, X,
                       offsets, ids, L.vals_out, K, t, k, out_ids, out_scores, searched);
    if (hipGetLastError() != hipSuccess) return SOAR_E_DEVICE;
  }
  return hipStreamSynchronize(st) == hipSuccess ? SOAR_OK : SOAR_E_DEVICE;
}

}  // extern "C"
