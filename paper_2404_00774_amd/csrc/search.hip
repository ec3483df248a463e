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
#include <functional>
#include <vector>

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

// The t best partitions of each query of a chunk (t <= kSelMax) in the order a stable
// descending sort gives them (higher score, then lower index), without sorting all K: per query
// one workgroup finds the t-th largest score T by a radix select over an order-preserving 64-bit
// image of the scores (six passes of at most 11 bits, counts in LDS), takes every score above T
// and the lowest-indexed scores equal to T, and sorts those t entries in LDS (bitonic).  The
// first t places of keys_out / vals_out are written as the sort would write them.
constexpr int kSelMax = 256;
constexpr int kSelBins = 2048;
constexpr int kSelStage = 4096;        // up to this many scores per query are read once, into LDS

__device__ __forceinline__ uint64_t order_key(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

template <bool STAGE>
__global__ __launch_bounds__(256) void probe_select_kernel(const double* __restrict__ keys,
                                                           int K, int t, double* keys_out,
                                                           int32_t* vals_out) {
  __shared__ double s_keys[STAGE ? kSelStage : 1];
  __shared__ unsigned hist[kSelBins];
  __shared__ unsigned part[256];
  __shared__ uint64_t s_prefix;
  __shared__ int s_need, s_cnt, s_taken;
  __shared__ double sel_s[kSelMax];
  __shared__ int sel_j[kSelMax];
  const int tid = threadIdx.x, qi = blockIdx.x;
  const double* kg = keys + (int64_t)qi * K;
  if constexpr (STAGE)
    for (int j = tid; j < K; j += 256) s_keys[j] = kg[j];
  const double* kq = STAGE ? s_keys : kg;
  if (tid == 0) { s_prefix = 0; s_need = t; }
  __syncthreads();
  // radix select: digits of 11 bits from the top (bits 53..63, 42..52, 31..41, 20..30, 9..19),
  // then the last 9 bits
  for (int pass = 0; pass < 6; ++pass) {
    const int base_shift = pass < 5 ? 53 - 11 * pass : 0;
    const int bits = pass < 5 ? 11 : 9;
    const uint64_t high_mask = base_shift + bits >= 64 ? 0ull : ~0ull << (base_shift + bits);
    const uint64_t prefix = s_prefix;
    const int need = s_need;
    for (int i = tid; i < kSelBins; i += 256) hist[i] = 0u;
    __syncthreads();
    for (int j = tid; j < K; j += 256) {
      const uint64_t key = order_key(kq[j]);
      if ((key & high_mask) == prefix)
        atomicAdd(&hist[(key >> base_shift) & ((1u << bits) - 1u)], 1u);
    }
    __syncthreads();
    // counts from the top digit down: thread i sums the 8 digits nb - 8 i - 1 .. nb - 8 i - 8
    const int nb = 1 << bits;
    unsigned mine = 0;
    for (int u = 0; u < 8; ++u) {
      const int dgt = nb - 1 - (8 * tid + u);
      if (dgt >= 0) mine += hist[dgt];
    }
    part[tid] = mine;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const unsigned add = tid >= o ? part[tid - o] : 0u;
      __syncthreads();
      part[tid] += add;
      __syncthreads();
    }
    const unsigned before = tid > 0 ? part[tid - 1] : 0u;
    if (before < (unsigned)need && part[tid] >= (unsigned)need) {
      unsigned c = before;
      for (int u = 0; u < 8; ++u) {
        const int dgt = nb - 1 - (8 * tid + u);
        if (dgt < 0) break;
        if (c + hist[dgt] >= (unsigned)need) {
          s_prefix = prefix | ((uint64_t)dgt << base_shift);
          s_need = need - (int)c;
          break;
        }
        c += hist[dgt];
      }
    }
    __syncthreads();
  }
  const uint64_t T = s_prefix;
  const int need_eq = s_need;                   // entries equal to T to take, lowest index first
  if (tid == 0) { s_cnt = 0; s_taken = 0; }
  __syncthreads();
  // every key above T
  for (int j = tid; j < K; j += 256) {
    const double v = kq[j];
    if (order_key(v) > T) {
      const int pos = atomicAdd(&s_cnt, 1);
      sel_s[pos] = v;
      sel_j[pos] = j;
    }
  }
  __syncthreads();
  const int above = s_cnt;
  // the need_eq lowest-indexed keys equal to T, in index order
  for (int j0 = 0; j0 < K && s_taken < need_eq; j0 += 256) {
    const int j = j0 + tid;
    const bool eq = j < K && order_key(kq[j]) == T;
    part[tid] = eq ? 1u : 0u;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const unsigned add = tid >= o ? part[tid - o] : 0u;
      __syncthreads();
      part[tid] += add;
      __syncthreads();
    }
    const int rank = s_taken + (int)part[tid] - 1;
    if (eq && rank < need_eq) {
      sel_s[above + rank] = kq[j];
      sel_j[above + rank] = j;
    }
    __syncthreads();
    if (tid == 0) s_taken += (int)part[255];
    __syncthreads();
  }
  // bitonic sort of the t selected entries (padded to kSelMax): higher score, then lower index
  if (tid >= t) { sel_s[tid] = -__builtin_inf(); sel_j[tid] = 0x7fffffff; }
  __syncthreads();
  for (int k = 2; k <= kSelMax; k <<= 1) {
    for (int h = k >> 1; h > 0; h >>= 1) {
      const int o = tid ^ h;
      if (o > tid) {
        const bool up = (tid & k) == 0;        // this half ascends in the sort order
        const double a = sel_s[tid], b = sel_s[o];
        const int ia = sel_j[tid], ib = sel_j[o];
        const bool a_first = a > b || (a == b && ia < ib);
        if (up ? !a_first : a_first) {
          sel_s[tid] = b; sel_s[o] = a;
          sel_j[tid] = ib; sel_j[o] = ia;
        }
      }
      __syncthreads();
    }
  }
  if (tid < t) {
    keys_out[(int64_t)qi * K + tid] = sel_s[tid];
    vals_out[(int64_t)qi * K + tid] = sel_j[tid];
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

// A thread's kSearchMaxK best (score, id), best first; (s, x) enters if better than the last
// and not already held.
__device__ __forceinline__ void keep_best(double (&sc)[kSearchMaxK], int (&id_)[kSearchMaxK],
                                          double s, int x) {
  if (!better(s, x, sc[kSearchMaxK - 1], id_[kSearchMaxK - 1])) return;
  bool held = false;
#pragma unroll
  for (int m = 0; m < kSearchMaxK; ++m) held |= id_[m] == x;
  if (held) return;
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

// k rounds of a workgroup arg-max over the threads' heads (a workgroup of kRerankThreads): the k
// best distinct ids (an id held by two threads is taken once: every holder moves past it);
// -1 and -inf where fewer than k were held.
__device__ __forceinline__ void emit_best(const double (&sc)[kSearchMaxK],
                                          const int (&id_)[kSearchMaxK], int k, int32_t* out_ids,
                                          double* out_scores, double* s_ws, int* s_wi) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
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
      out_ids[r] = got ? wi : -1;
      out_scores[r] = got ? ws : -__builtin_inf();
    }
  }
}

// Exact <q, x> of the rows idp[0 .. nb) (nb <= kRerankThreads), thread tid taking row tid (0
// for threads past nb): the rows go through LDS kRD dimensions at a time, each thread
// accumulating its row in dimension order (FP64), so a row's value does not depend on the batch
// it is in.  Loads: 8 lanes per row piece of kRD floats, each lane 4 floats (one 16-byte load
// when d % 4 == 0); a thread's 8 pieces of a chunk are issued together, and the next chunk's are
// in flight while the current one is summed.  Every thread of the workgroup calls it.
constexpr int kRowPieces = kRerankThreads * (kRD / 4) / kRerankThreads;   // per thread per chunk

// VEC: d % 4 == 0, so every piece is one aligned 16-byte load (chunk widths are multiples of 4).
template <bool VEC>
__device__ __forceinline__ double score_rows(const float* q, int d, const float* X,
                                             const int32_t* idp, int nb,
                                             float (*s_rows)[kRD + 1], float* s_q) {
  const int tid = threadIdx.x;
  // the thread's pieces: row rr = (tid + 256 u) / 8, columns c4 .. c4 + 3 with c4 = (tid % 8) * 4
  const float* rowp[kRowPieces];
  bool live[kRowPieces];
#pragma unroll
  for (int u = 0; u < kRowPieces; ++u) {
    const int rr = (tid + kRerankThreads * u) >> 3;
    live[u] = rr < nb;
    rowp[u] = X + (int64_t)idp[live[u] ? rr : 0] * d;    // nb >= 1: row 0 exists
  }
  const int c4 = (tid & 7) * 4;
  float4 v[kRowPieces];
  auto load = [&](int k0) __attribute__((always_inline)) {
    const int kw = min(kRD, d - k0);
#pragma unroll
    for (int u = 0; u < kRowPieces; ++u) {
      float4 w = {0.f, 0.f, 0.f, 0.f};
      const float* src = rowp[u] + k0 + c4;
      if constexpr (VEC) {
        if (live[u] && c4 < kw) w = *reinterpret_cast<const float4*>(src);
      } else {
        if (live[u]) {
          if (c4 < kw) w.x = src[0];
          if (c4 + 1 < kw) w.y = src[1];
          if (c4 + 2 < kw) w.z = src[2];
          if (c4 + 3 < kw) w.w = src[3];
        }
      }
      v[u] = w;
    }
  };
  double s = 0.0;
  load(0);
  for (int k0 = 0; k0 < d; k0 += kRD) {
    const int kw = min(kRD, d - k0);
#pragma unroll
    for (int u = 0; u < kRowPieces; ++u) {
      const int rr = (tid + kRerankThreads * u) >> 3;
      s_rows[rr][c4] = v[u].x;
      s_rows[rr][c4 + 1] = v[u].y;
      s_rows[rr][c4 + 2] = v[u].z;
      s_rows[rr][c4 + 3] = v[u].w;
    }
    if (tid < kRD) s_q[tid] = tid < kw ? q[k0 + tid] : 0.f;
    __syncthreads();
    if (k0 + kRD < d) load(k0 + kRD);
    for (int c = 0; c < kw; ++c) s = fma((double)s_q[c], (double)s_rows[tid][c], s);
    __syncthreads();
  }
  return s + 0.0;
}

template <bool VEC>
__global__ __launch_bounds__(kRerankThreads) void rerank_kernel(
    const float* __restrict__ Q, int64_t q0, int d, const float* __restrict__ X,
    const int64_t* __restrict__ off, const int32_t* __restrict__ ids,
    const int32_t* __restrict__ order, const double* __restrict__ oscore, int K, int t, int k,
    int32_t* out_ids, double* out_scores, int64_t* searched) {
  __shared__ float s_rows[kRerankThreads][kRD + 1];
  __shared__ float s_q[kRD];
  __shared__ double s_ws[kRerankThreads / 64];
  __shared__ int s_wi[kRerankThreads / 64];
  const int qi = blockIdx.x;
  const int64_t qg = q0 + qi;
  const float* q = Q + qg * (int64_t)d;
  const int tid = threadIdx.x;
  int64_t count = 0;
  // the thread's kSearchMaxK best, best first (empty places: -inf and id INT_MAX)
  double sc[kSearchMaxK];
  int id_[kSearchMaxK];
#pragma unroll
  for (int m = 0; m < kSearchMaxK; ++m) { sc[m] = -__builtin_inf(); id_[m] = 0x7fffffff; }
  for (int r = 0; r < t; ++r) {
    if (oscore && oscore[(int64_t)qi * K + r] == -__builtin_inf()) break;   // nothing listed
    const int p = order[(int64_t)qi * K + r];
    const int64_t b = off[p], e = off[p + 1];
    count += e - b;
    for (int64_t base = b; base < e; base += kRerankThreads) {
      const int nb = (int)min<int64_t>(kRerankThreads, e - base);
      const double s = score_rows<VEC>(q, d, X, ids + base, nb, s_rows, s_q);
      if (tid < nb) keep_best(sc, id_, s, ids[base + tid]);
    }
  }
  emit_best(sc, id_, k, out_ids + qg * k, out_scores + qg * k, s_ws, s_wi);
  if (tid == 0 && searched) searched[qg] = count;
}


// ---- Lists with PQ-coded copies (Section 3.5's index layout) and their search ----
// A list entry is a copy of a point in one partition; it carries the PQ code of that copy's own
// residual x - c_p.  The codes are stored in list order, code_bytes = M / 2 per entry.
constexpr int kPQMaxSub = 512;        // subspaces: the FP64 table (16 per subspace) in 64 KB LDS
constexpr int kPQMaxRerank = 4096;    // points re-scored exactly per query

// Codes in list order: entry pos of list p is point ids[pos] through its first assignment j with
// assign[ids[pos] * m + j] == p, and takes that assignment's code.  One workgroup per list; the
// longest list's length goes to *max_list.
__global__ __launch_bounds__(256) void list_codes_kernel(
    const int64_t* __restrict__ off, const int32_t* __restrict__ ids, int64_t n,
    const int32_t* __restrict__ assign, int m, const uint8_t* __restrict__ codes, int nb,
    uint8_t* __restrict__ out, unsigned long long* max_list, unsigned* bad) {
  const int p = blockIdx.x;
  const int64_t b = off[p], e = off[p + 1];
  if (threadIdx.x == 0) atomicMax(max_list, (unsigned long long)(e - b));
  for (int64_t pos = b + threadIdx.x; pos < e; pos += blockDim.x) {
    const int64_t i = ids[pos];
    int j = -1;
    if (i >= 0 && i < n)
      for (int u = m - 1; u >= 0; --u)
        if (assign[i * m + u] == p) j = u;
    uint8_t* o = out + pos * nb;
    if (j < 0) {
      atomicOr(bad, 1u);
      for (int c = 0; c < nb; ++c) o[c] = 0;
      continue;
    }
    const uint8_t* src = codes + (i * m + j) * nb;
    for (int c = 0; c < nb; ++c) o[c] = src[c];
  }
}

// Per query of the chunk: where each probed list's copies start inside the query's candidate
// segment, the query's copy count, and (scored) that count for the caller.
__global__ void pq_slots_kernel(const int64_t* __restrict__ off, const int32_t* __restrict__ order,
                                int K, int nqc, int t, int64_t* slot, int64_t* cnt,
                                int64_t* scored, int64_t q0) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= nqc) return;
  int64_t acc = 0;
  for (int r = 0; r < t; ++r) {
    const int p = order[(int64_t)qi * K + r];
    slot[(int64_t)qi * t + r] = acc;
    acc += off[p + 1] - off[p];
  }
  cnt[qi] = acc;
  if (scored) scored[q0 + qi] = acc;
}

// Exclusive scan of the chunk's copy counts into the segment bounds seg[0 .. nqc] (one
// workgroup of 1024 threads; the layout keeps the total below 2^31).
__global__ __launch_bounds__(1024) void pq_seg_kernel(const int64_t* __restrict__ cnt, int nqc,
                                                      int* seg) {
  __shared__ int64_t sh[1024];
  int64_t carry = 0;
  for (int base = 0; base < nqc; base += 1024) {
    const int j = base + (int)threadIdx.x;
    const int64_t v = j < nqc ? cnt[j] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (j < nqc) seg[j] = (int)(carry + sh[threadIdx.x] - v);
    carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) seg[nqc] = (int)carry;
}

// Approximate scores of the copies in probed list r of query qi (one workgroup each): the
// query's table LUT[m][c] = <q_m, P[m][c]> (FP64, the s dimensions in order) in LDS, then per
// copy <q, c_p> + LUT[0][code_0] + LUT[1][code_1] + ... added in subspace order, written with
// the copy's id at its place in the query's candidate segment.
__global__ __launch_bounds__(256) void pq_score_kernel(
    const float* __restrict__ Q, int64_t q0, int d, const float* __restrict__ P, int s, int M,
    const int64_t* __restrict__ off, const int32_t* __restrict__ ids,
    const uint8_t* __restrict__ lcodes, const double* __restrict__ pscore,
    const int32_t* __restrict__ order, int K, int t, const int64_t* __restrict__ slot,
    const int* __restrict__ seg, int32_t* cid, double* cval) {
  extern __shared__ double lut[];        // [M][16]
  const int r = blockIdx.x, qi = blockIdx.y;
  const float* q = Q + (q0 + qi) * (int64_t)d;
  for (int e = threadIdx.x; e < M * 16; e += blockDim.x) {
    const int m = e >> 4;
    const float* pv = P + (int64_t)e * s;
    double a = 0.0;
    for (int u = 0; u < s; ++u) a = fma((double)q[m * s + u], (double)pv[u], a);
    lut[e] = a;
  }
  __syncthreads();
  const int p = order[(int64_t)qi * K + r];
  const double sp = pscore[(int64_t)qi * K + r];
  const int64_t b = off[p], e = off[p + 1];
  const int64_t dst = (int64_t)seg[qi] + slot[(int64_t)qi * t + r] - b;
  const int nb = M / 2;
  for (int64_t pos = b + threadIdx.x; pos < e; pos += blockDim.x) {
    double a = sp;
    if ((nb & 3) == 0) {
      const uint32_t* c4 = reinterpret_cast<const uint32_t*>(lcodes + pos * nb);
      for (int w4 = 0; w4 < nb / 4; ++w4) {
        const uint32_t w = c4[w4];
#pragma unroll
        for (int u = 0; u < 8; ++u) a += lut[(w4 * 8 + u) * 16 + ((w >> (4 * u)) & 15)];
      }
    } else {
      const uint8_t* c = lcodes + pos * nb;
      for (int j = 0; j < nb; ++j) {
        const unsigned byte = c[j];
        a += lut[(2 * j) * 16 + (byte & 15)];
        a += lut[(2 * j + 1) * 16 + (byte >> 4)];
      }
    }
    cid[dst + pos] = ids[pos];
    cval[dst + pos] = a;
  }
}

// A threshold on the estimates per query that keeps every copy the selection can need: with
// at most two copies per point, the R best points all have their best copy among the 2 R best
// copies, so every copy whose estimate is at least the (2 R)-th largest suffices (a point with
// one copy kept has its best copy kept too).  The estimates are binned linearly between the
// query's smallest and largest (a monotone map, so the bins are ordered like the estimates),
// and the kept set is every copy in the highest bins whose counts reach 2 R.  A query with at
// most 2 R copies keeps them all.
constexpr int kPQBins = 1024;

__device__ __forceinline__ int pq_bin(double v, double lo, double scale) {
  return min(kPQBins - 1, (int)((v - lo) * scale));
}

__global__ __launch_bounds__(256) void pq_thresh_kernel(const int* __restrict__ seg,
                                                        const double* __restrict__ cv, int need,
                                                        int64_t* cnt, double* lo_out,
                                                        double* scale_out, int* bin_out) {
  __shared__ unsigned hist[kPQBins];
  __shared__ double s_lo[4], s_hi[4];
  const int qi = blockIdx.x, tid = threadIdx.x;
  const int b = seg[qi], e = seg[qi + 1];
  if (e - b <= need) {
    if (tid == 0) { cnt[qi] = e - b; lo_out[qi] = 0.0; scale_out[qi] = 0.0; bin_out[qi] = 0; }
    return;
  }
  double lo = __builtin_inf(), hi = -__builtin_inf();
  for (int i = b + tid; i < e; i += 256) {
    const double v = cv[i];
    lo = v < lo ? v : lo;
    hi = v > hi ? v : hi;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ol = __shfl_xor(lo, off), oh = __shfl_xor(hi, off);
    lo = ol < lo ? ol : lo;
    hi = oh > hi ? oh : hi;
  }
  if ((tid & 63) == 0) { s_lo[tid >> 6] = lo; s_hi[tid >> 6] = hi; }
  for (int i = tid; i < kPQBins; i += 256) hist[i] = 0u;
  __syncthreads();
  lo = s_lo[0];
  hi = s_hi[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    lo = s_lo[w] < lo ? s_lo[w] : lo;
    hi = s_hi[w] > hi ? s_hi[w] : hi;
  }
  const double scale = hi > lo ? kPQBins / (hi - lo) : 0.0;
  for (int i = b + tid; i < e; i += 256) atomicAdd(&hist[pq_bin(cv[i], lo, scale)], 1u);
  __syncthreads();
  if (tid == 0) {
    int64_t c = 0;
    int bb = kPQBins - 1;
    for (; bb > 0; --bb) {
      c += hist[bb];
      if (c >= need) break;
    }
    if (bb == 0) c += hist[0];
    cnt[qi] = c;
    lo_out[qi] = lo;
    scale_out[qi] = scale;
    bin_out[qi] = bb;
  }
}

// The kept copies of each query, compacted into the segment seg2[qi] .. (order not kept: the
// sorts that follow do not depend on it).
__global__ __launch_bounds__(256) void pq_compact_kernel(
    const int* __restrict__ seg, const int32_t* __restrict__ cid, const double* __restrict__ cv,
    const double* __restrict__ lo, const double* __restrict__ scale, const int* __restrict__ bin,
    const int* __restrict__ seg2, int32_t* cid_o, double* cv_o) {
  __shared__ int cursor;
  const int qi = blockIdx.x;
  if (threadIdx.x == 0) cursor = 0;
  __syncthreads();
  const int b = seg[qi], e = seg[qi + 1], o = seg2[qi];
  const double l = lo[qi], sc = scale[qi];
  const int bb = bin[qi];
  for (int i = b + threadIdx.x; i < e; i += 256) {
    const double v = cv[i];
    if (pq_bin(v, l, sc) >= bb) {
      const int pos = atomicAdd(&cursor, 1);
      cid_o[o + pos] = cid[i];
      cv_o[o + pos] = v;
    }
  }
}

// After the copies of each query are sorted by id: the first copy of every id takes the largest
// estimate of its copies, the others -inf (so they sort last and are never re-scored).
__global__ __launch_bounds__(256) void pq_dedup_kernel(const int* __restrict__ seg,
                                                       const int32_t* __restrict__ cid,
                                                       const double* __restrict__ cval,
                                                       double* out) {
  const int qi = blockIdx.x;
  const int b = seg[qi], e = seg[qi + 1];
  for (int i = b + threadIdx.x; i < e; i += blockDim.x) {
    const int id = cid[i];
    if (i > b && cid[i - 1] == id) {
      out[i] = -__builtin_inf();
      continue;
    }
    double v = cval[i];
    for (int j = i + 1; j < e && cid[j] == id; ++j) v = cval[j] > v ? cval[j] : v;
    out[i] = v;
  }
}

// The R best points of a query (its segment sorted by estimate, descending, ties by id) are
// scored exactly and the k best returned.
template <bool VEC>
__global__ __launch_bounds__(kRerankThreads) void pq_rerank_kernel(
    const float* __restrict__ Q, int64_t q0, int d, const float* __restrict__ X,
    const int* __restrict__ seg, const double* __restrict__ cval, const int32_t* __restrict__ cid,
    int R, int k, int32_t* out_ids, double* out_scores) {
  __shared__ float s_rows[kRerankThreads][kRD + 1];
  __shared__ float s_q[kRD];
  __shared__ double s_ws[kRerankThreads / 64];
  __shared__ int s_wi[kRerankThreads / 64];
  const int qi = blockIdx.x;
  const int64_t qg = q0 + qi;
  const float* q = Q + qg * (int64_t)d;
  const int tid = threadIdx.x;
  const int b = seg[qi];
  const int e = b + min(R, seg[qi + 1] - b);
  double sc[kSearchMaxK];
  int id_[kSearchMaxK];
#pragma unroll
  for (int m = 0; m < kSearchMaxK; ++m) { sc[m] = -__builtin_inf(); id_[m] = 0x7fffffff; }
  for (int base = b; base < e; base += kRerankThreads) {
    const int nb = min(kRerankThreads, e - base);
    const double s = score_rows<VEC>(q, d, X, cid + base, nb, s_rows, s_q);
    if (tid < nb && cval[base + tid] > -__builtin_inf()) keep_best(sc, id_, s, cid[base + tid]);
  }
  emit_best(sc, id_, k, out_ids + qg * k, out_scores + qg * k, s_ws, s_wi);
}

// Second level of a two-level probe: for each of a query's t2 best upper centroids (one
// workgroup each), every partition listed under it gets its score <q, c_p> at place p of the
// query's K scores (FP64 in dimension order from zero, as probe_scores_kernel forms it); the
// places of partitions not listed stay -inf.
__global__ __launch_bounds__(256) void probe_second_kernel(
    const float* __restrict__ Q, int64_t q0, int d, const float* __restrict__ C, int K,
    const int64_t* __restrict__ uoff, const int32_t* __restrict__ uids,
    const int32_t* __restrict__ uorder, int K2, double* keys) {
  __shared__ float sq[1024];
  const int r = blockIdx.x, qi = blockIdx.y;
  const float* q = Q + (q0 + qi) * (int64_t)d;
  for (int j = threadIdx.x; j < d; j += blockDim.x) sq[j] = q[j];
  __syncthreads();
  const int u = uorder[(int64_t)qi * K2 + r];
  for (int64_t pos = uoff[u] + threadIdx.x; pos < uoff[u + 1]; pos += blockDim.x) {
    const int p = uids[pos];
    if (p < 0 || p >= K) continue;
    const float* c = C + (int64_t)p * d;
    double acc = 0.0;
    for (int j = 0; j < d; ++j) acc = fma((double)sq[j], (double)c[j], acc);
    keys[(int64_t)qi * K + p] = acc + 0.0;
  }
}

// Segment bounds q K of nqc queries of K scores, and the index of every place (the inputs a
// segmented sort of the scores needs when the probe depth is beyond the selection's).
__global__ void seg_bounds_kernel(int nqc, int K, int* seg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= nqc) seg[i] = i * K;
}

__global__ void iota_rows_kernel(int32_t* vals, int nqc, int K) {
  const int64_t cells = (int64_t)nqc * K;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cells;
       i += (int64_t)gridDim.x * blockDim.x)
    vals[i] = (int32_t)(i % K);
}

__global__ void fill_f64_kernel(double* p, int64_t count, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

bool launch_rerank(const float* Q, int64_t q0, int d, const float* X, const int64_t* offsets,
                   const int32_t* ids, const int32_t* order, const double* oscore, int K, int t,
                   int k, int32_t* out_ids, double* out_scores, int64_t* searched, int nqc,
                   hipStream_t st) {
  if ((d & 3) == 0)
    hipLaunchKernelGGL(rerank_kernel<true>, dim3(nqc), dim3(kRerankThreads), 0, st, Q, q0, d, X,
                       offsets, ids, order, oscore, K, t, k, out_ids, out_scores, searched);
  else
    hipLaunchKernelGGL(rerank_kernel<false>, dim3(nqc), dim3(kRerankThreads), 0, st, Q, q0, d, X,
                       offsets, ids, order, oscore, K, t, k, out_ids, out_scores, searched);
  return hipGetLastError() == hipSuccess;
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

// Queries per chunk for K scores each: about 256 MB of sort keys and values.
int search_chunk(int64_t nq, int K) {
  const int64_t per_q = (int64_t)K * 24;
  return (int)std::max<int64_t>(
      1, std::min<int64_t>(std::min<int64_t>(nq, 65535), ((int64_t)256 << 20) / per_q));
}

// The probe arrays of nqc queries of K scores, placed at *off in ws (nullptr: sizes only).
SearchLayout search_layout_at(char* base, size_t* off, int nqc, int K) {
  SearchLayout L{};
  L.nqc = nqc;
  const int64_t items = (int64_t)nqc * K;
  auto take = [&](size_t b) { char* p = base ? base + *off : nullptr; *off = al(*off + b); return p; };
  L.keys_in = reinterpret_cast<double*>(take(items * 8));
  L.keys_out = reinterpret_cast<double*>(take(items * 8));
  L.vals_in = reinterpret_cast<int32_t*>(take(items * 4));
  L.vals_out = reinterpret_cast<int32_t*>(take(items * 4));
  L.seg = reinterpret_cast<int*>(take((size_t)(nqc + 1) * 4));
  size_t tb = 0;
  (void)hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
      nullptr, tb, L.keys_in, L.keys_out, L.vals_in, L.vals_out, (int)items, nqc, L.seg,
      L.seg + 1);
  L.temp_bytes = tb;
  L.temp = take(tb);
  L.bytes = *off;
  return L;
}

SearchLayout search_layout(void* ws, int64_t nq, int K) {
  size_t off = 0;
  return search_layout_at(static_cast<char*>(ws), &off, search_chunk(nq, K), K);
}

// The first t places of keys_out / vals_out per query: the selection kernel for t <= kSelMax,
// else a stable descending segmented sort of all K scores.
bool probe_top(const SearchLayout& L, int nqc, int K, int t, hipStream_t st) {
  if (t <= kSelMax) {
    if (K <= kSelStage)
      hipLaunchKernelGGL(probe_select_kernel<true>, dim3(nqc), dim3(256), 0, st, L.keys_in, K, t,
                         L.keys_out, L.vals_out);
    else
      hipLaunchKernelGGL(probe_select_kernel<false>, dim3(nqc), dim3(256), 0, st, L.keys_in, K,
                         t, L.keys_out, L.vals_out);
    return hipGetLastError() == hipSuccess;
  }
  size_t tb = L.temp_bytes;
  return hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
             L.temp, tb, L.keys_in, L.keys_out, L.vals_in, L.vals_out, nqc * K, nqc, L.seg,
             L.seg + 1, 0, 64, st) == hipSuccess;
}

// Workspace of soar_search_two_level: the probe arrays of both levels for one chunk of queries.
struct TwoLevelLayout {
  SearchLayout upper, lower;
  size_t bytes;
  int nqc;
};

TwoLevelLayout two_level_layout(void* ws, int64_t nq, int K, int K2) {
  TwoLevelLayout L{};
  L.nqc = std::min(search_chunk(nq, K), search_chunk(nq, K2));
  size_t off = 0;
  char* base = static_cast<char*>(ws);
  L.upper = search_layout_at(base, &off, L.nqc, K2);
  L.lower = search_layout_at(base, &off, L.nqc, K);
  L.bytes = off;
  return L;
}

// Workspace of soar_search_pq: the probe's sort arrays for nqc queries and the candidate arrays
// (ids and estimates, twice each, and the sorts' temporary storage) for nqc queries of at most
// max_probed copies each (the most that t probed lists can hold).
struct SearchPQLayout {
  SearchLayout probe;
  int64_t* slot;
  int64_t* cnt;
  int* seg;
  int64_t* cnt2;                       // copies kept per query, and their segments
  int* seg2;
  double* lo;
  double* scale;
  int* bin;
  int32_t* cid_a;
  int32_t* cid_b;
  double* cv_a;
  double* cv_b;
  void* temp;
  size_t temp_bytes;
  int64_t cap;
  size_t bytes;
  int nqc;
};

constexpr int64_t kPQCandidates = (int64_t)1 << 28;   // copies per chunk of queries (about 6.4 GB)

SearchPQLayout search_pq_layout(void* ws, int64_t nq, int K, int t, int64_t max_probed) {
  SearchPQLayout L{};
  const int64_t per_q = std::max<int64_t>(1, max_probed);
  const int64_t probe_q = search_chunk(nq, K);
  L.nqc = (int)std::max<int64_t>(1, std::min<int64_t>(probe_q, kPQCandidates / per_q));
  L.cap = (int64_t)L.nqc * per_q;
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t b) { char* p = base ? base + off : nullptr; off = al(off + b); return p; };
  // the probe arrays first, sized for this layout's nqc
  const int64_t items = (int64_t)L.nqc * K;
  L.probe.nqc = L.nqc;
  L.probe.keys_in = reinterpret_cast<double*>(take(items * 8));
  L.probe.keys_out = reinterpret_cast<double*>(take(items * 8));
  L.probe.vals_in = reinterpret_cast<int32_t*>(take(items * 4));
  L.probe.vals_out = reinterpret_cast<int32_t*>(take(items * 4));
  L.probe.seg = reinterpret_cast<int*>(take((size_t)(L.nqc + 1) * 4));
  L.slot = reinterpret_cast<int64_t*>(take((size_t)L.nqc * t * 8));
  L.cnt = reinterpret_cast<int64_t*>(take((size_t)L.nqc * 8));
  L.seg = reinterpret_cast<int*>(take((size_t)(L.nqc + 1) * 4));
  L.cnt2 = reinterpret_cast<int64_t*>(take((size_t)L.nqc * 8));
  L.seg2 = reinterpret_cast<int*>(take((size_t)(L.nqc + 1) * 4));
  L.lo = reinterpret_cast<double*>(take((size_t)L.nqc * 8));
  L.scale = reinterpret_cast<double*>(take((size_t)L.nqc * 8));
  L.bin = reinterpret_cast<int*>(take((size_t)L.nqc * 4));
  L.cid_a = reinterpret_cast<int32_t*>(take(L.cap * 4));
  L.cid_b = reinterpret_cast<int32_t*>(take(L.cap * 4));
  L.cv_a = reinterpret_cast<double*>(take(L.cap * 8));
  L.cv_b = reinterpret_cast<double*>(take(L.cap * 8));
  size_t tb = 0, t1 = 0, t2 = 0;
  (void)hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
      nullptr, tb, L.probe.keys_in, L.probe.keys_out, L.probe.vals_in, L.probe.vals_out,
      (int)items, L.nqc, L.probe.seg, L.probe.seg + 1);
  (void)hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, t1, L.cid_b, L.cid_a, L.cv_b, L.cv_a,
                                                    (int)L.cap, L.nqc, L.seg2, L.seg2 + 1);
  (void)hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
      nullptr, t2, L.cv_b, L.cv_a, L.cid_a, L.cid_b, (int)L.cap, L.nqc, L.seg2, L.seg2 + 1);
  L.temp_bytes = std::max(tb, std::max(t1, t2));
  L.temp = take(L.temp_bytes);
  L.probe.temp = L.temp;
  L.probe.temp_bytes = L.temp_bytes;
  L.bytes = off;
  return L;
}

// The most copies any t lists hold: the sum of the t longest list lengths (offsets read back).
soar_status probe_bound(const int64_t* offsets, int K, int t, hipStream_t st, int64_t* bound) {
  std::vector<int64_t> off((size_t)K + 1);
  if (hipMemcpyAsync(off.data(), offsets, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost,
                     st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SOAR_E_DEVICE;
  std::vector<int64_t> len((size_t)K);
  for (int p = 0; p < K; ++p) {
    len[p] = off[p + 1] - off[p];
    if (len[p] < 0) return SOAR_E_INVAL;
  }
  const int tt = std::min(t, K);
  std::nth_element(len.begin(), len.begin() + (tt - 1), len.end(), std::greater<int64_t>());
  int64_t b = 0;
  for (int i = 0; i < tt; ++i) b += len[i];
  *bound = b;
  return SOAR_OK;
}

int id_bits(int64_t n) {
  int b = 1;
  while (b < 32 && ((int64_t)1 << b) < n) ++b;
  return b;
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
    if (!probe_top(L, nqc, K, t, st)) return SOAR_E_DEVICE;
    if (!launch_rerank(Q, q0, d, X, offsets, ids, L.vals_out, nullptr, K, t, k, out_ids,
                       out_scores, searched, nqc, st))
      return SOAR_E_DEVICE;
    if (hipGetLastError() != hipSuccess) return SOAR_E_DEVICE;
  }
  return hipStreamSynchronize(st) == hipSuccess ? SOAR_OK : SOAR_E_DEVICE;
}


soar_status soar_lists_codes(const int64_t* offsets, const int32_t* ids, int32_t K, int64_t n,
                             const int32_t* assign, int32_t m, const uint8_t* codes,
                             int32_t code_bytes, uint8_t* list_codes, int64_t* max_list,
                             void* workspace, size_t ws_bytes, void* stream) {
  if (!offsets || !ids || !assign || !codes || !list_codes || !workspace || ws_bytes < 256 ||
      K < 1 || n < 1 || m < 1 || code_bytes < 1)
    return SOAR_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int64_t* w = static_cast<int64_t*>(workspace);    // [0] longest list, [1] bad-entry flag
  hipLaunchKernelGGL(zero_i64_kernel, dim3(1), dim3(64), 0, st, w, (int64_t)2);
  hipLaunchKernelGGL(list_codes_kernel, dim3(K), dim3(256), 0, st, offsets, ids, n, assign, m,
                     codes, code_bytes, list_codes, reinterpret_cast<unsigned long long*>(w),
                     reinterpret_cast<unsigned*>(w + 1));
  int64_t h[2] = {0, 0};
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(h, w, 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SOAR_E_DEVICE;
  if (max_list) *max_list = h[0];
  return h[1] ? SOAR_E_INVAL : SOAR_OK;
}

soar_status soar_lists_probe_bound(const int64_t* offsets, int32_t K, int32_t t, int64_t* bound,
                                   void* stream) {
  if (!offsets || !bound || K < 1 || t < 1) return SOAR_E_INVAL;
  return probe_bound(offsets, K, t, static_cast<hipStream_t>(stream), bound);
}

soar_status soar_search_pq_workspace_size(int64_t nq, int32_t d, int32_t K, int32_t t,
                                          int64_t max_probed, size_t* bytes) {
  if (!bytes || nq < 1 || d < 1 || K < 1 || t < 1 || max_probed < 0) return SOAR_E_INVAL;
  t = std::min(t, K);
  if (max_probed >= ((int64_t)1 << 31)) return SOAR_E_UNSUPPORTED;
  *bytes = search_pq_layout(nullptr, nq, K, t, max_probed).bytes;
  return SOAR_OK;
}

soar_status soar_search_pq(const float* Q, int64_t nq, int32_t d, const float* C, int32_t K,
                           const float* X, int64_t n, const int64_t* offsets, const int32_t* ids,
                           const uint8_t* list_codes, const float* P, int32_t s, int32_t t,
                           int32_t R, int32_t k, int64_t max_probed, int32_t* out_ids,
                           double* out_scores, int64_t* scored, void* workspace, size_t ws_bytes,
                           void* stream) {
  size_t need = 0;
  if (!Q || !C || !X || !offsets || !ids || !list_codes || !P || !out_ids || !out_scores ||
      !workspace || n < 1 || t < 1 || k < 1 || k > kSearchMaxK || R < k || R > kPQMaxRerank ||
      s < 1 || d % (2 * s) != 0 || (reinterpret_cast<uintptr_t>(list_codes) & 3) != 0)
    return SOAR_E_INVAL;
  const int M = d / s;
  if (M > kPQMaxSub) return SOAR_E_UNSUPPORTED;
  const soar_status sz = soar_search_pq_workspace_size(nq, d, K, t, max_probed, &need);
  if (sz != SOAR_OK) return sz;
  if (ws_bytes < need) return SOAR_E_INVAL;
  t = std::min(t, K);
  hipStream_t st = static_cast<hipStream_t>(stream);
  SearchPQLayout L = search_pq_layout(workspace, nq, K, t, max_probed);
  // any t lists must fit the bound the workspace was sized for
  int64_t actual = 0;
  const soar_status bs = probe_bound(offsets, K, t, st, &actual);
  if (bs != SOAR_OK) return bs;
  if (actual > max_probed) return SOAR_E_INVAL;
  const size_t lut_bytes = (size_t)M * 16 * sizeof(double);
  const int bits = id_bits(n);
  for (int64_t q0 = 0; q0 < nq; q0 += L.nqc) {
    const int nqc = (int)std::min<int64_t>(L.nqc, nq - q0);
    SearchLayout& PL = L.probe;
    hipLaunchKernelGGL(probe_scores_kernel, dim3((K + kPC - 1) / kPC, (nqc + kPQ - 1) / kPQ),
                       dim3(256), 0, st, Q, q0, nqc, d, C, K, PL.keys_in, PL.vals_in, PL.seg);
    if (!probe_top(PL, nqc, K, t, st)) return SOAR_E_DEVICE;
    size_t tb = L.temp_bytes;
    hipLaunchKernelGGL(pq_slots_kernel, dim3((nqc + 255) / 256), dim3(256), 0, st, offsets,
                       PL.vals_out, K, nqc, t, L.slot, L.cnt, scored, q0);
    hipLaunchKernelGGL(pq_seg_kernel, dim3(1), dim3(1024), 0, st, L.cnt, nqc, L.seg);
    hipLaunchKernelGGL(pq_score_kernel, dim3(t, nqc), dim3(256), lut_bytes, st, Q, q0, d, P, s,
                       M, offsets, ids, list_codes, PL.keys_out, PL.vals_out, K, t, L.slot,
                       L.seg, L.cid_a, L.cv_a);
    // the copies that can matter (at least the 2 R best of each query), compacted
    hipLaunchKernelGGL(pq_thresh_kernel, dim3(nqc), dim3(256), 0, st, L.seg, L.cv_a, 2 * R,
                       L.cnt2, L.lo, L.scale, L.bin);
    hipLaunchKernelGGL(pq_seg_kernel, dim3(1), dim3(1024), 0, st, L.cnt2, nqc, L.seg2);
    hipLaunchKernelGGL(pq_compact_kernel, dim3(nqc), dim3(256), 0, st, L.seg, L.cid_a, L.cv_a,
                       L.lo, L.scale, L.bin, L.seg2, L.cid_b, L.cv_b);
    // by id (so a point's copies are adjacent), best copy kept, then by estimate: descending,
    // equal estimates in id order (both sorts are stable)
    const int items = (int)L.cap;
    tb = L.temp_bytes;
    if (hipcub::DeviceSegmentedRadixSort::SortPairs(L.temp, tb, L.cid_b, L.cid_a, L.cv_b, L.cv_a,
                                                    items, nqc, L.seg2, L.seg2 + 1, 0, bits,
                                                    st) != hipSuccess)
      return SOAR_E_DEVICE;
    hipLaunchKernelGGL(pq_dedup_kernel, dim3(nqc), dim3(256), 0, st, L.seg2, L.cid_a, L.cv_a,
                       L.cv_b);
    tb = L.temp_bytes;
    if (hipcub::DeviceSegmentedRadixSort::SortPairsDescending(
            L.temp, tb, L.cv_b, L.cv_a, L.cid_a, L.cid_b, items, nqc, L.seg2, L.seg2 + 1, 0, 64,
            st) != hipSuccess)
      return SOAR_E_DEVICE;
    if ((d & 3) == 0)
      hipLaunchKernelGGL(pq_rerank_kernel<true>, dim3(nqc), dim3(kRerankThreads), 0, st, Q, q0,
                         d, X, L.seg2, L.cv_a, L.cid_b, R, k, out_ids, out_scores);
    else
      hipLaunchKernelGGL(pq_rerank_kernel<false>, dim3(nqc), dim3(kRerankThreads), 0, st, Q, q0,
                         d, X, L.seg2, L.cv_a, L.cid_b, R, k, out_ids, out_scores);
    if (hipGetLastError() != hipSuccess) return SOAR_E_DEVICE;
  }
  return hipStreamSynchronize(st) == hipSuccess ? SOAR_OK : SOAR_E_DEVICE;
}


soar_status soar_search_two_level_workspace_size(int64_t nq, int32_t d, int32_t K, int32_t K2,
                                                 size_t* bytes) {
  if (!bytes || nq < 1 || d < 1 || K < 1 || K2 < 1) return SOAR_E_INVAL;
  *bytes = two_level_layout(nullptr, nq, K, K2).bytes;
  return SOAR_OK;
}

soar_status soar_search_two_level(const float* Q, int64_t nq, int32_t d, const float* U,
                                  int32_t K2, const int64_t* upper_offsets,
                                  const int32_t* upper_ids, int32_t t2, const float* C, int32_t K,
                                  const float* X, int64_t n, const int64_t* offsets,
                                  const int32_t* ids, int32_t t, int32_t k, int32_t* out_ids,
                                  double* out_scores, int64_t* searched, void* workspace,
                                  size_t ws_bytes, void* stream) {
  size_t need = 0;
  if (!Q || !U || !upper_offsets || !upper_ids || !C || !X || !offsets || !ids || !out_ids ||
      !out_scores || !workspace || n < 1 || t < 1 || t2 < 1 || k < 1 || k > kSearchMaxK ||
      soar_search_two_level_workspace_size(nq, d, K, K2, &need) != SOAR_OK || ws_bytes < need)
    return SOAR_E_INVAL;
  if (d > 1024) return SOAR_E_UNSUPPORTED;
  t = std::min(t, K);
  t2 = std::min(t2, K2);
  hipStream_t st = static_cast<hipStream_t>(stream);
  TwoLevelLayout L = two_level_layout(workspace, nq, K, K2);
  for (int64_t q0 = 0; q0 < nq; q0 += L.nqc) {
    const int nqc = (int)std::min<int64_t>(L.nqc, nq - q0);
    // upper level: <q, u> for every upper centroid, the t2 best
    hipLaunchKernelGGL(probe_scores_kernel, dim3((K2 + kPC - 1) / kPC, (nqc + kPQ - 1) / kPQ),
                       dim3(256), 0, st, Q, q0, nqc, d, U, K2, L.upper.keys_in, L.upper.vals_in,
                       L.upper.seg);
    if (!probe_top(L.upper, nqc, K2, t2, st)) return SOAR_E_DEVICE;
    // lower level: the partitions listed under those, scored; the rest stay -inf
    const int64_t cells = (int64_t)nqc * K;
    hipLaunchKernelGGL(fill_f64_kernel,
                       dim3((unsigned)std::min<int64_t>((cells + 255) / 256, 4096)), dim3(256), 0,
                       st, L.lower.keys_in, cells, -__builtin_inf());
    hipLaunchKernelGGL(probe_second_kernel, dim3(t2, nqc), dim3(256), 0, st, Q, q0, d, C, K,
                       upper_offsets, upper_ids, L.upper.vals_out, K2, L.lower.keys_in);
    if (t > kSelMax) {   // the segmented sort's inputs: segment bounds and place indices
      hipLaunchKernelGGL(seg_bounds_kernel, dim3((nqc + 256) / 256), dim3(256), 0, st, nqc, K,
                         L.lower.seg);
      hipLaunchKernelGGL(iota_rows_kernel,
                         dim3((unsigned)std::min<int64_t>((cells + 255) / 256, 4096)), dim3(256),
                         0, st, L.lower.vals_in, nqc, K);
    }
    if (!probe_top(L.lower, nqc, K, t, st)) return SOAR_E_DEVICE;
    if (!launch_rerank(Q, q0, d, X, offsets, ids, L.lower.vals_out, L.lower.keys_out, K, t, k,
                       out_ids, out_scores, searched, nqc, st))
      return SOAR_E_DEVICE;
  }
  return hipStreamSynchronize(st) == hipSuccess ? SOAR_OK : SOAR_E_DEVICE;
}

}  // extern "C"
