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
//           repeats, and a bitonic sort of the workgroup's lists in LDS yields the k best
//           distinct ids.
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
// segment bounds of the sort.
__global__ void probe_scores_kernel(const float* __restrict__ Q, int64_t q0, int nqc, int d,
                                    const float* __restrict__ C, int K, double* keys,
                                    int32_t* vals, int* seg) {
  const int qi = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) {
    seg[qi] = qi * K;
    if (qi == nqc - 1) seg[nqc] = nqc * K;
  }
  if (j >= K) return;
  const float* q = Q + (q0 + qi) * (int64_t)d;
  const float* c = C + (int64_t)j * d;
  double s = 0.0;
  for (int k = 0; k < d; ++k) s = fma((double)q[k], (double)c[k], s);
  keys[(int64_t)qi * K + j] = s + 0.0;   // -0 becomes +0, so equal scores sort as equal
  vals[(int64_t)qi * K + j] = j;
}

// (score, id) order of the results: higher score first, then lower id.
__device__ __forceinline__ bool better(double s, int i, double t, int j) {
  return s > t || (s == t && i < j);
}

// One workgroup per query of the chunk: scan the t probed lists, keep the k best distinct ids.
__global__ __launch_bounds__(kRerankThreads) void rerank_kernel(
    const float* __restrict__ Q, int64_t q0, int d, const float* __restrict__ X,
    const int64_t* __restrict__ off, const int32_t* __restrict__ ids,
    const int32_t* __restrict__ order, int K, int t, int k, int32_t* out_ids, double* out_scores,
    int64_t* searched) {
  __shared__ double s_sc[kRerankThreads * kSearchMaxK];
  __shared__ int s_id[kRerankThreads * kSearchMaxK];
  __shared__ int64_t s_count;
  const int qi = blockIdx.x;
  const int64_t qg = q0 + qi;
  const float* q = Q + qg * (int64_t)d;
  const int tid = threadIdx.x;
  if (tid == 0) s_count = 0;
  // the thread's k best, best first (empty places: -inf and id INT_MAX)
  double sc[kSearchMaxK];
  int id_[kSearchMaxK];
#pragma unroll
  for (int m = 0; m < kSearchMaxK; ++m) { sc[m] = -__builtin_inf(); id_[m] = 0x7fffffff; }
  __syncthreads();
  for (int r = 0; r < t; ++r) {
    const int p = order[(int64_t)qi * K + r];
    const int64_t b = off[p], e = off[p + 1];
    if (tid == 0) s_count += e - b;
    for (int64_t i = b + tid; i < e; i += kRerankThreads) {
      const int x = ids[i];
      const float* xr = X + (int64_t)x * d;
      double s = 0.0;
      for (int kk = 0; kk < d; ++kk) s = fma((double)q[kk], (double)xr[kk], s);
      s += 0.0;
      // (every thread keeps its kSearchMaxK best; the first k of the merge are returned)
      // enters only if better than the current last and not already held
      if (!better(s, x, sc[kSearchMaxK - 1], id_[kSearchMaxK - 1])) continue;
      bool held = false;
#pragma unroll
      for (int m = 0; m < kSearchMaxK; ++m) held |= id_[m] == x;
      if (held) continue;
      // insert: shift the worse entries down by one
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
  // the workgroup's candidates: kRerankThreads * kSearchMaxK entries, bitonic sort, best first
#pragma unroll
  for (int m = 0; m < kSearchMaxK; ++m) {
    s_sc[tid * kSearchMaxK + m] = sc[m];
    s_id[tid * kSearchMaxK + m] = id_[m];
  }
  __syncthreads();
  constexpr int N = kRerankThreads * kSearchMaxK;
  for (int size = 2; size <= N; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < N; i += kRerankThreads) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;   // this pair's run is sorted best first
          const bool swap = up ? better(s_sc[j], s_id[j], s_sc[i], s_id[i])
                               : better(s_sc[i], s_id[i], s_sc[j], s_id[j]);
          if (swap) {
            const double ts = s_sc[i];
            const int ti = s_id[i];
            s_sc[i] = s_sc[j];
            s_id[i] = s_id[j];
            s_sc[j] = ts;
            s_id[j] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    int got = 0;
    int last = -1;
    for (int i = 0; i < N && got < k; ++i) {
      const int x = s_id[i];
      if (x == 0x7fffffff) break;
      if (x == last) continue;         // a point met through both of its lists
      out_ids[qg * k + got] = x;
      out_scores[qg * k + got] = s_sc[i];
      last = x;
      ++got;
    }
    for (; got < k; ++got) {
      out_ids[qg * k + got] = -1;
      out_scores[qg * k + got] = -__builtin_inf();
    }
    if (searched) searched[qg] = s_count;
  }
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
    hipLaunchKernelGGL(probe_scores_kernel, dim3((K + 255) / 256, nqc), dim3(256), 0, st, Q, q0,
                       nqc, d, C, K, L.keys_in, L.vals_in, L.seg);
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
