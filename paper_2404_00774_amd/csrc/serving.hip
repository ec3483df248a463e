// Serving: a resident codebook plus inverted lists (Section 2.2: for each partition the ids of
// the points assigned to it; with SOAR a point sits in the lists of pi(x) and pi'(x)), fed by
// streaming insert requests.
//
// Continuous batching.  A scheduler thread builds device steps of at most max_step_rows rows from
// the queued requests and launches each into a free step slot as soon as one is free (a request
// may span steps, a step may hold many requests).  Rows are shared out max-min fairly: every
// queued request gets up to an equal share of the step, and what a request does not need goes to
// the others, so a small request that arrives behind a large one joins the very next step.  Each
// slot has its own stream, buffers, pre-captured HIP graphs and a waiter thread, so steps overlap
// on the GPU and each one's results are delivered the moment its own work is done.  A step is
//   H2D (live row count, rows, ids) -> compute graph (the SOAR assignment kernels, which read the
//   live row count from device memory) -> D2H of the indices [results delivered here] ->
//   [waits for the previous step's list append] -> append graph (count, reserve chunks, scatter
//   ids) -> D2H of the step's list status [slot freed here].
// Admission by memory: a step is admitted only if the list arena can take its worst-case growth
// on top of what the steps in flight may take.
//
// Lists live in the caller's arena as chains of chunks of CH ids: partition p has len[p] ids in
// the chain head[p] -> next[] -> tail[p].  The appends of one step: count per partition; one
// thread per touched partition takes the chunks it needs from the pool (a compare-and-swap bump
// that never takes more than the pool holds) and links them behind its tail; then every
// assignment takes a position by an atomic cursor and finds its chunk from the step's first new
// chunk.  The order of ids inside a list is therefore not fixed; its content is.  Appends of
// consecutive steps are ordered by events, so these per-step arrays are shared by all slots.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/soar.h"
#include "common.h"
#include "kernels.h"
#include "train.h"

namespace soar {

constexpr int LIST_CH = 64;        // ids per chunk
constexpr int kSlots = 2;          // step slots (steps in flight at once)

struct ListDev {
  int32_t* len;      // [K] ids in the list
  int32_t* head;     // [K] first chunk (-1: empty list)
  int32_t* tail;     // [K] last chunk
  int32_t* next;     // [chunks] next chunk of the same list (-1: last)
  int64_t* pool;     // [chunks * LIST_CH] ids
  // per-step state (appends of consecutive steps are serialized)
  int32_t* cnt;      // [K] appends of the current step (-1: could not reserve)
  int32_t* cursor;   // [K] append cursor (old length + appends taken so far)
  int32_t* olen;     // [K] length before the step
  int32_t* otail;    // [K] tail before the step
  int32_t* first;    // [K] first new chunk of the step
  int32_t* meta;     // [0] chunks in use
  int32_t chunks;    // pool capacity in chunks
  int32_t K;
};

__global__ void fill_i32(int32_t* p, int64_t count, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void list_count_kernel(const int32_t* __restrict__ prim, const int32_t* __restrict__ spl,
                                  const int64_t* live, int64_t cap, ListDev L) {
  const int64_t n = live_rows(cap, live);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int a = prim[i], b = spl[i];
    if (a >= 0 && a < L.K) atomicAdd(&L.cnt[a], 1);
    if (b >= 0 && b < L.K) atomicAdd(&L.cnt[b], 1);
  }
}

// One thread per partition with appends: reserve its new chunks and link them behind its tail.
// A workgroup's partitions reserve their chunks together (a prefix sum of their needs and one
// compare-and-swap on the pool cursor for the total), so the cursor sees one update per 256
// partitions instead of one per partition.  If the pool cannot hold the workgroup's total, each
// partition tries alone; a reservation that the pool cannot hold takes nothing, leaves the list
// as it was and sets bit 0 of the step's status word.
constexpr int kReserveThreads = 256;

__device__ __forceinline__ bool reserve_chunks(int32_t* cursor, int chunks, int k, int* base) {
  int cur = atomicAdd(cursor, 0);
  for (;;) {
    if (cur > chunks - k) return false;
    const int seen = atomicCAS(cursor, cur, cur + k);
    if (seen == cur) break;
    cur = seen;
  }
  *base = cur;
  return true;
}

__global__ __launch_bounds__(kReserveThreads) void list_reserve_kernel(ListDev L,
                                                                       unsigned* status) {
  __shared__ int s_k[kReserveThreads];
  __shared__ int s_base;
  const int tid = threadIdx.x;
  const int p = blockIdx.x * kReserveThreads + tid;
  const int c = p < L.K ? L.cnt[p] : 0;
  const int old = c > 0 ? L.len[p] : 0, nw = old + (c > 0 ? c : 0);
  const int have = (old + LIST_CH - 1) / LIST_CH, need = (nw + LIST_CH - 1) / LIST_CH;
  const int k = c > 0 ? need - have : 0;
  // inclusive prefix sum of the chunk needs over the workgroup
  s_k[tid] = k;
  __syncthreads();
  for (int o = 1; o < kReserveThreads; o <<= 1) {
    const int add = tid >= o ? s_k[tid - o] : 0;
    __syncthreads();
    s_k[tid] += add;
    __syncthreads();
  }
  const int total = s_k[kReserveThreads - 1];
  if (tid == 0) {
    int b = -1;
    if (total > 0 && !reserve_chunks(&L.meta[0], L.chunks, total, &b)) b = -1;
    s_base = b;
  }
  __syncthreads();
  if (c <= 0) return;
  int base = -1;
  if (k > 0) {
    if (s_base >= 0) {
      base = s_base + s_k[tid] - k;
    } else if (!reserve_chunks(&L.meta[0], L.chunks, k, &base)) {
      L.cnt[p] = -1;
      atomicOr(status, 1u);
      return;
    }
    for (int i = 0; i < k; ++i) L.next[base + i] = i + 1 < k ? base + i + 1 : -1;
    if (old == 0) L.head[p] = base;
    else L.next[L.tail[p]] = base;
  }
  L.olen[p] = old;
  L.otail[p] = old == 0 ? -1 : L.tail[p];
  L.first[p] = base;
  if (k > 0) L.tail[p] = base + k - 1;
  L.cursor[p] = old;
  L.len[p] = nw;
}

__global__ void list_scatter_kernel(const int32_t* __restrict__ prim,
                                    const int32_t* __restrict__ spl,
                                    const int64_t* __restrict__ ids, const int64_t* live,
                                    int64_t cap, ListDev L) {
  const int64_t n = live_rows(cap, live);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int ab[2] = {prim[i], spl[i]};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int p = ab[k];
      if (p < 0 || p >= L.K || L.cnt[p] < 0) continue;
      const int pos = atomicAdd(&L.cursor[p], 1);
      // positions up to the old tail chunk's end stay in it; the rest go to the new chunks
      const int ofull = (L.olen[p] + LIST_CH - 1) / LIST_CH * LIST_CH;
      const int chunk = pos < ofull ? L.otail[p] : L.first[p] + (pos - ofull) / LIST_CH;
      L.pool[(int64_t)chunk * LIST_CH + pos % LIST_CH] = ids[i];
    }
  }
}

// --------------------------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------------------------
namespace {

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0, first_id = 0;
  std::vector<float> X;
  std::vector<int32_t> prim, spill;
  int64_t next_row = 0;    // rows handed to steps
  int64_t done_rows = 0;   // rows whose results arrived
  soar_status status = SOAR_OK;
  bool complete = false;
};

struct Part {
  std::shared_ptr<Request> req;
  int64_t row0, rows, slot_off;
};

struct Slot {
  hipStream_t st = nullptr;
  hipGraphExec_t g_compute = nullptr, g_append = nullptr;
  hipEvent_t ev_results = nullptr, ev_append = nullptr, ev_done = nullptr;
  // device
  float* X = nullptr;
  int64_t* ids = nullptr;
  int64_t* live = nullptr;
  int32_t* prim = nullptr;
  int32_t* spill = nullptr;
  unsigned* status = nullptr;    // list status of the step (bit 0: a reservation failed)
  void* ws = nullptr;            // assignment workspace of this slot
  unsigned* counters = nullptr;
  // pinned host staging
  char* h_in = nullptr;          // [live int64][ids cap int64][X cap*d float]
  char* h_out = nullptr;         // [prim cap][spill cap][counters 8][status, chunks used]
  bool busy = false;     // the worker has taken the slot for a step (set before its launch)
  bool ready = false;    // the step is fully enqueued, its events recorded: the waiter may go
  int64_t rows = 0, worst_chunks = 0;
  std::vector<Part> parts;
  std::thread waiter;
  std::condition_variable cv;    // a step was launched into this slot, or shutdown
};

}  // namespace

}  // namespace soar

using namespace soar;

struct soar_index {
  int32_t K = 0, d = 0, precision = 0, cap = 0, fmt = 0;
  float lambda = 0.f;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  // codebook (device, inside the arena)
  float* C = nullptr;
  float* cnorm = nullptr;
  void* crec = nullptr;          // packed codebook records of the sweeps
  ListDev L{};
  Slot slots[kSlots];
  hipEvent_t last_append = nullptr;   // append event of the latest launched step
  // scheduling state (guarded by mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
  uint64_t next_ticket = 1;
  int64_t chunks_used = 0;       // known from the last completed step
  int64_t chunks_reserved = 0;   // worst case of the steps in flight
  bool shutdown = false;
  bool device_error = false;
  bool list_error = false;       // an append could not be reserved (never with admission)
  int paused = 0;
  int in_flight = 0;
  soar_index_stats stats{};
  std::thread worker;
};

namespace {

// Codebook splits of a serving step's sweeps.  A step of few rows fills few workgroups, and
// each would sweep every centroid tile in turn; splitting the codebook into S parts runs S
// workgroups per row group, each over an S-th of the tiles, and a merge keeps the best
// candidates (BF16/FP8) or joins the splits' exact answers (FP32, rows of up to 256 dimensions).  One split per 4096 centroids, at most 8, so every split covers at least 4096
// columns.  Fixed per index, so a row's result does not depend on the step it runs in.
int serving_ksplit(int K) { return std::max(1, std::min(8, K / 4096)); }

size_t step_ws_bytes(int64_t cap, int d, int K, bool lowp, int fmt) {
  if (!lowp) {
    // counters + full-scan rows; with codebook splits per split: index, value, full-scan rows
    const int S = fp32_split_supported(d) ? serving_ksplit(K) : 1;
    return al(CNT_ALLOC_WORDS * 4) + al((size_t)cap * 4) +
           (S > 1 ? 3 * al((size_t)cap * S * 4) + al(64 * 4) : 0);
  }
  const int dp = lowp_padded_dim(fmt, d);
  const size_t eb = fmt == LOWP_BF16 ? 2 : 1;
  const int S = serving_ksplit(K);
  return al(CNT_ALLOC_WORDS * 4) + 2 * al((size_t)cap * dp * eb) + al((size_t)cap * 4) +
         al((size_t)cap * 16) + al((size_t)cap * 8 * 4) +
         (S > 1 ? 2 * al((size_t)cap * S * 8 * 4) : 0);
}

// Bytes of one list chunk: its ids and its link.
constexpr size_t kChunkBytes = LIST_CH * 8 + 4;

struct ArenaPlan {
  size_t C, cnorm, crec, L_len, L_head, L_tail, L_cnt, L_cursor, L_olen, L_otail, L_first, L_meta;
  size_t slot[kSlots], next, pool;
  size_t slot_bytes, fixed, total;
  int64_t chunks;
};

ArenaPlan plan_arena(int K, int d, int precision, int cap, size_t arena_bytes) {
  ArenaPlan P{};
  const bool lowp = precision != SOAR_FP32;
  const int fmt = precision == SOAR_BF16 ? LOWP_BF16 : LOWP_FP8;
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off = al(off + b); return o; };
  P.C = take((size_t)K * d * 4);
  P.cnorm = take((size_t)K * 4);
  P.crec = take(lowp ? lowp_codebook_bytes(fmt, d, K) : fp32_codebook_bytes(d, K));
  P.L_len = take((size_t)K * 4);
  P.L_head = take((size_t)K * 4);
  P.L_tail = take((size_t)K * 4);
  P.L_cnt = take((size_t)K * 4);
  P.L_cursor = take((size_t)K * 4);
  P.L_olen = take((size_t)K * 4);
  P.L_otail = take((size_t)K * 4);
  P.L_first = take((size_t)K * 4);
  P.L_meta = take(64);
  P.slot_bytes = al((size_t)cap * d * 4) + al((size_t)cap * 8) + al(8) + 2 * al((size_t)cap * 4) +
                 al(64) + step_ws_bytes(cap, d, K, lowp, fmt);
  for (int k = 0; k < kSlots; ++k) P.slot[k] = take(P.slot_bytes);
  P.fixed = off + 2 * kAl;        // the link and id arrays start aligned
  int64_t chunks = arena_bytes > P.fixed ? (int64_t)((arena_bytes - P.fixed) / kChunkBytes) : 0;
  if (chunks > INT32_MAX) chunks = INT32_MAX;
  P.chunks = chunks;
  P.next = take((size_t)chunks * 4);
  P.pool = take((size_t)chunks * LIST_CH * 8);
  P.total = off;
  return P;
}

// Most chunks the appends of a step of `rows` rows can take: its ids fill whole chunks, plus at
// most one partly filled new chunk per touched partition.
int64_t worst_chunks(int64_t rows, int K) {
  const int64_t a = 2 * rows;
  return (a + LIST_CH - 1) / LIST_CH + std::min<int64_t>(a, K);
}

// Launch the assignment kernels of one step on st (captured into the slot's compute graph).
hipError_t enqueue_compute(soar_index* ix, Slot& s) {
  const bool lowp = ix->precision != SOAR_FP32;
  hipError_t e = launch_reset_step_counters(s.counters, s.st);
  if (e != hipSuccess) return e;
  if (!lowp) {
    AssignParams P;
    P.X = s.X; P.n = ix->cap; P.d = ix->d; P.C = ix->C; P.K = ix->K;
    P.Crec = static_cast<const char*>(ix->crec);
    P.cnorm = ix->cnorm; P.counters = s.counters;
    P.lam = ix->lambda;
    P.tie_rel = tie_threshold(ix->d, ix->lambda, 0.f);
    P.band_p = band_coef_primary(ix->d);
    P.band_s = band_coef_spill(ix->d, ix->lambda);
    P.primary = s.prim; P.spill = s.spill; P.pdist = nullptr; P.sloss = nullptr;
    char* w = static_cast<char*>(s.ws) + al(CNT_ALLOC_WORDS * 4);
    P.full_rows = reinterpret_cast<int32_t*>(w);
    w += al((size_t)ix->cap * 4);
    P.live_n = s.live;
    const int S = fp32_split_supported(ix->d) ? serving_ksplit(ix->K) : 1;
    if (S > 1) {
      P.split_idx = reinterpret_cast<int32_t*>(w); w += al((size_t)ix->cap * S * 4);
      P.split_val = reinterpret_cast<float*>(w); w += al((size_t)ix->cap * S * 4);
      P.split_rows = reinterpret_cast<int32_t*>(w); w += al((size_t)ix->cap * S * 4);
      P.split_cnt = reinterpret_cast<unsigned*>(w);
      return launch_assign_fp32_split(P, S, ix->d % 4 == 0, s.st);
    }
    return launch_assign_fp32(P, true, ix->d % 4 == 0, s.st);
  }
  const int fmt = ix->fmt, dp = lowp_padded_dim(fmt, ix->d);
  const size_t eb = fmt == LOWP_BF16 ? 2 : 1;
  char* w = static_cast<char*>(s.ws) + al(CNT_ALLOC_WORDS * 4);
  LowpParams P;
  P.n = ix->cap; P.d = ix->d; P.dp = dp; P.K = ix->K; P.topk = 8;
  P.lam = ix->lambda;
  P.tie_rel = tie_threshold(ix->d, ix->lambda, 0.f);
  P.X = s.X; P.C = ix->C;
  P.Xq = w; w += al((size_t)ix->cap * dp * eb);
  P.Rq = w; P.Rq_out = w; w += al((size_t)ix->cap * dp * eb);
  P.xs = reinterpret_cast<float*>(w); w += al((size_t)ix->cap * 4);
  P.rowc = reinterpret_cast<float4*>(w); P.rowc_out = reinterpret_cast<float4*>(w);
  w += al((size_t)ix->cap * 16);
  P.cand = reinterpret_cast<int32_t*>(w); w += al((size_t)ix->cap * 8 * 4);
  P.ksplit = serving_ksplit(ix->K);
  if (P.ksplit > 1) {
    P.cand_split = reinterpret_cast<int32_t*>(w); w += al((size_t)ix->cap * P.ksplit * 8 * 4);
    P.cand_val = reinterpret_cast<float*>(w); w += al((size_t)ix->cap * P.ksplit * 8 * 4);
  }
  P.Cq = ix->crec; P.cs = nullptr; P.cnorm = ix->cnorm;
  P.primary = s.prim; P.spill = s.spill; P.pdist = nullptr; P.sloss = nullptr;
  P.counters = s.counters;
  P.live_n = s.live;
  e = launch_lowp_quantize(fmt, s.X, ix->cap, ix->d, dp, false, const_cast<void*>(P.Xq),
                           const_cast<float*>(P.xs), s.counters, s.st, s.live);
  if (e == hipSuccess) e = launch_lowp_sweep(fmt, P, false, s.st);
  if (e == hipSuccess) e = launch_lowp_merge(P, s.st);
  if (e == hipSuccess) e = launch_lowp_rescore(fmt, P, false, s.st);
  if (e == hipSuccess) e = launch_lowp_sweep(fmt, P, true, s.st);
  if (e == hipSuccess) e = launch_lowp_merge(P, s.st);
  if (e == hipSuccess) e = launch_lowp_rescore(fmt, P, true, s.st);
  return e;
}

hipError_t enqueue_append(soar_index* ix, Slot& s) {
  const ListDev& L = ix->L;
  // fill kernels, not memsets: these run inside a replayed graph
  hipLaunchKernelGGL(fill_i32, dim3((L.K + 255) / 256), dim3(256), 0, s.st, L.cnt, (int64_t)L.K, 0);
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s.st, reinterpret_cast<int32_t*>(s.status),
                     (int64_t)1, 0);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((ix->cap + 255) / 256, 1024));
  hipLaunchKernelGGL(list_count_kernel, dim3(g), dim3(256), 0, s.st, s.prim, s.spill, s.live,
                     (int64_t)ix->cap, L);
  hipLaunchKernelGGL(list_reserve_kernel, dim3((L.K + kReserveThreads - 1) / kReserveThreads),
                     dim3(kReserveThreads), 0, s.st, L,
                     s.status);
  hipLaunchKernelGGL(list_scatter_kernel, dim3(g), dim3(256), 0, s.st, s.prim, s.spill, s.ids,
                     s.live, (int64_t)ix->cap, L);
  return hipGetLastError();
}

template <typename F>
hipError_t capture(hipStream_t st, hipGraphExec_t* out, F&& body) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t eb = body();
  e = hipStreamEndCapture(st, &g);
  if (eb != hipSuccess) { if (g) (void)hipGraphDestroy(g); return eb; }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

// Host layout of a slot's results buffer.
struct OutView {
  int32_t* prim;
  int32_t* spill;
  unsigned* cnt;
  unsigned* list;     // [0] step status, [1] chunks in use after the step
};
OutView out_view(const soar_index* ix, const Slot& s) {
  OutView v;
  v.prim = reinterpret_cast<int32_t*>(s.h_out);
  v.spill = v.prim + ix->cap;
  v.cnt = reinterpret_cast<unsigned*>(v.spill + ix->cap);
  v.list = v.cnt + CNT_WORDS;
  return v;
}

// The rows of `limit` a step takes from each queued request: max-min fair shares (a request
// needing less than an equal share gets all it needs, the rest is split evenly), handed out in
// queue order.
std::vector<Part> plan_step(soar_index* ix, int64_t limit) {
  std::vector<int64_t> need;
  for (auto& r : ix->queue) need.push_back(r->n - r->next_row);
  std::vector<int64_t> sorted = need;
  std::sort(sorted.begin(), sorted.end());
  // the largest share s with sum_i min(need_i, s) <= limit
  const size_t m = sorted.size();
  int64_t left = limit, share = m ? sorted[m - 1] : 0;
  for (size_t i = 0; i < m; ++i) {
    const int64_t eq = left / (int64_t)(m - i);
    if (sorted[i] > eq) { share = eq; break; }
    left -= sorted[i];
  }
  int64_t extra = limit;
  for (int64_t v : need) extra -= std::min(v, share);
  std::vector<Part> parts;
  int64_t rows = 0;
  size_t i = 0;
  for (auto it = ix->queue.begin(); it != ix->queue.end(); ++it, ++i) {
    int64_t take = std::min(need[i], share);
    const int64_t more = std::max<int64_t>(0, std::min(need[i] - take, extra));
    take += more;
    extra -= more;
    if (take <= 0) continue;
    parts.push_back(Part{*it, (*it)->next_row, take, rows});
    rows += take;
  }
  return parts;
}

// Fill slot s from the queue and launch it (lock held; released around the copies).
bool try_launch(soar_index* ix, Slot& s, std::unique_lock<std::mutex>& lk) {
  // admission by memory: the most rows whose worst-case list growth fits the free chunks
  const int64_t free_chunks = ix->L.chunks - ix->chunks_used - ix->chunks_reserved;
  int64_t limit = ix->cap;
  while (limit > 0 && worst_chunks(limit, ix->K) > free_chunks) limit /= 2;
  if (limit == 0) {
    if (ix->in_flight == 0) {
      // nothing in flight will release memory: the request at the head can never be placed
      Request& r = *ix->queue.front();
      r.status = SOAR_E_NOMEM;
      r.complete = true;
      ix->queue.pop_front();
      ix->cv_done.notify_all();
    }
    return false;
  }
  std::vector<Part> parts = plan_step(ix, limit);
  int64_t rows = 0;
  for (Part& p : parts) rows += p.rows;
  if (rows == 0) return false;
  for (Part& p : parts) p.req->next_row += p.rows;
  for (auto it = ix->queue.begin(); it != ix->queue.end();)
    it = (*it)->next_row == (*it)->n ? ix->queue.erase(it) : it + 1;
  s.parts = std::move(parts);
  s.rows = rows;
  s.worst_chunks = worst_chunks(rows, ix->K);
  s.busy = true;
  ix->chunks_reserved += s.worst_chunks;
  ++ix->in_flight;
  ix->stats.steps += 1;
  ix->stats.rows += rows;
  ix->stats.max_steps_in_flight = std::max<int64_t>(ix->stats.max_steps_in_flight, ix->in_flight);
  hipEvent_t prev_append = ix->last_append;
  ix->last_append = s.ev_append;
  ++ix->paused;                       // no soar_index_list while this slot is being launched
  lk.unlock();
  // stage the rows (pinned), then the step
  int64_t* hlive = reinterpret_cast<int64_t*>(s.h_in);
  int64_t* hids = hlive + 1;
  float* hX = reinterpret_cast<float*>(hids + ix->cap);
  hlive[0] = rows;
  for (Part& p : s.parts) {
    const Request& r = *p.req;
    std::memcpy(hX + p.slot_off * ix->d, r.X.data() + p.row0 * ix->d, p.rows * ix->d * 4);
    for (int64_t i = 0; i < p.rows; ++i) hids[p.slot_off + i] = r.first_id + p.row0 + i;
  }
  const OutView o = out_view(ix, s);
  hipError_t e = hipMemcpyAsync(s.live, hlive, 8, hipMemcpyHostToDevice, s.st);
  if (e == hipSuccess) e = hipMemcpyAsync(s.ids, hids, rows * 8, hipMemcpyHostToDevice, s.st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.X, hX, rows * ix->d * 4, hipMemcpyHostToDevice, s.st);
  if (e == hipSuccess) e = hipGraphLaunch(s.g_compute, s.st);
  if (e == hipSuccess) e = hipMemcpyAsync(o.prim, s.prim, rows * 4, hipMemcpyDeviceToHost, s.st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o.spill, s.spill, rows * 4, hipMemcpyDeviceToHost, s.st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o.cnt, s.counters, CNT_WORDS * 4, hipMemcpyDeviceToHost, s.st);
  if (e == hipSuccess) e = hipEventRecord(s.ev_results, s.st);
  if (e == hipSuccess && prev_append) e = hipStreamWaitEvent(s.st, prev_append, 0);
  if (e == hipSuccess) e = hipGraphLaunch(s.g_append, s.st);
  if (e == hipSuccess) e = hipEventRecord(s.ev_append, s.st);
  if (e == hipSuccess) e = hipMemcpyAsync(o.list, s.status, 4, hipMemcpyDeviceToHost, s.st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o.list + 1, ix->L.meta, 4, hipMemcpyDeviceToHost, s.st);
  if (e == hipSuccess) e = hipEventRecord(s.ev_done, s.st);
  lk.lock();
  --ix->paused;
  if (e != hipSuccess) ix->device_error = true;
  // only now are this step's events recorded: a waiter that woke while `busy` alone was set
  // would have synchronized on the previous step's events and taken its stale results
  s.ready = true;
  s.cv.notify_one();                  // the slot's waiter takes it from here
  ix->cv_done.notify_all();
  return true;
}

// Waiter thread of one slot: results to the requests as soon as the step's indices are in host
// memory; the slot (and its worst-case list memory) free once its list append is done.
void slot_loop(soar_index* ix, Slot& s) {
  std::unique_lock<std::mutex> lk(ix->mu);
  for (;;) {
    s.cv.wait(lk, [&] { return s.ready || (ix->shutdown && ix->in_flight == 0 &&
                                           ix->queue.empty()); });
    if (!s.ready) break;
    s.ready = false;
    const bool launch_failed = ix->device_error;
    lk.unlock();
    const hipError_t e1 = hipEventSynchronize(s.ev_results);
    lk.lock();
    const OutView o = out_view(ix, s);
    soar_status st = SOAR_OK;
    if (e1 != hipSuccess || launch_failed) { st = SOAR_E_DEVICE; ix->device_error = true; }
    else if (o.cnt[CNT_NONFINITE]) st = SOAR_E_NONFINITE;
    for (Part& p : s.parts) {
      Request& r = *p.req;
      std::memcpy(r.prim.data() + p.row0, o.prim + p.slot_off, p.rows * 4);
      std::memcpy(r.spill.data() + p.row0, o.spill + p.slot_off, p.rows * 4);
      if (st != SOAR_OK && r.status == SOAR_OK) r.status = st;
      r.done_rows += p.rows;
      if (r.done_rows == r.n) {
        r.complete = true;
        r.X.clear();
        r.X.shrink_to_fit();
      }
    }
    s.parts.clear();
    ix->cv_done.notify_all();
    lk.unlock();
    const hipError_t e2 = hipEventSynchronize(s.ev_done);
    lk.lock();
    if (e2 != hipSuccess) ix->device_error = true;
    else {
      if (o.list[0] != 0) ix->list_error = true;
      // the pool cursor only grows; the two slots' waiters may get here in either order, and a
      // slot's copy may predate the other slot's later append, so keep the largest value seen
      ix->chunks_used = std::max<int64_t>(ix->chunks_used, (int64_t)o.list[1]);
    }
    ix->chunks_reserved -= s.worst_chunks;
    s.busy = false;
    --ix->in_flight;
    ix->cv_work.notify_all();
    ix->cv_done.notify_all();
  }
}

// Scheduler thread: launches queued rows into free slots as soon as both exist.
void worker_loop(soar_index* ix) {
  std::unique_lock<std::mutex> lk(ix->mu);
  for (;;) {
    if (ix->device_error && !ix->queue.empty()) {
      for (auto& r : ix->queue) { r->status = SOAR_E_DEVICE; r->complete = true; }
      ix->queue.clear();
      ix->cv_done.notify_all();
    }
    if (!ix->queue.empty() && ix->paused == 0 && !ix->device_error) {
      Slot* free_slot = nullptr;
      for (Slot& s : ix->slots)
        if (!s.busy) { free_slot = &s; break; }
      if (free_slot && try_launch(ix, *free_slot, lk)) continue;
    }
    if (ix->shutdown && ix->queue.empty()) break;
    ix->cv_work.wait(lk);
  }
  // wake the slot waiters so they can leave once the last steps are done
  for (Slot& s : ix->slots) s.cv.notify_all();
}

void free_index(soar_index* ix) {
  for (Slot& s : ix->slots) {
    if (s.g_compute) (void)hipGraphExecDestroy(s.g_compute);
    if (s.g_append) (void)hipGraphExecDestroy(s.g_append);
    if (s.ev_results) (void)hipEventDestroy(s.ev_results);
    if (s.ev_append) (void)hipEventDestroy(s.ev_append);
    if (s.ev_done) (void)hipEventDestroy(s.ev_done);
    if (s.st) (void)hipStreamDestroy(s.st);
    if (s.h_in) (void)hipHostFree(s.h_in);
    if (s.h_out) (void)hipHostFree(s.h_out);
  }
  delete ix;
}

}  // namespace

extern "C" {

soar_status soar_index_arena_size(int32_t K, int32_t d, int32_t precision, int32_t max_step_rows,
                                  int64_t list_capacity_ids, size_t* bytes) {
  if (!bytes || K < 2 || d < 1 || max_step_rows < 1 || list_capacity_ids < 0) return SOAR_E_INVAL;
  if (precision == SOAR_FP32 ? fp32_padded_dim(d) < 0
                             : lowp_padded_dim(precision == SOAR_BF16 ? LOWP_BF16 : LOWP_FP8, d) < 0)
    return SOAR_E_UNSUPPORTED;
  const ArenaPlan P = plan_arena(K, d, precision, max_step_rows, 0);
  const int64_t chunks = (list_capacity_ids + LIST_CH - 1) / LIST_CH + 2 * (int64_t)K;
  *bytes = P.fixed + (size_t)chunks * kChunkBytes;
  return SOAR_OK;
}

size_t soar_index_chunk_bytes(void) { return kChunkBytes; }

soar_status soar_index_create(const float* C, int32_t K, int32_t d, float lambda,
                              int32_t precision, void* arena, size_t arena_bytes,
                              int32_t max_step_rows, soar_index** out) {
  if (!C || !arena || !out || K < 2 || d < 1 || max_step_rows < 1 || !std::isfinite(lambda) ||
      lambda < 0.f || (reinterpret_cast<uintptr_t>(arena) % 256) != 0)
    return SOAR_E_INVAL;
  if (precision != SOAR_FP32 && precision != SOAR_BF16 && precision != SOAR_FP8_E4M3)
    return SOAR_E_INVAL;
  const int fmt = precision == SOAR_BF16 ? LOWP_BF16 : LOWP_FP8;
  if (precision == SOAR_FP32 ? fp32_padded_dim(d) < 0 : lowp_padded_dim(fmt, d) < 0)
    return SOAR_E_UNSUPPORTED;
  const ArenaPlan plan = plan_arena(K, d, precision, max_step_rows, arena_bytes);
  if (plan.chunks < 1 || plan.total > arena_bytes) return SOAR_E_NOMEM;
  soar_index* ix = new soar_index();
  ix->K = K; ix->d = d; ix->precision = precision; ix->cap = max_step_rows; ix->fmt = fmt;
  ix->lambda = lambda;
  ix->arena = static_cast<char*>(arena);
  ix->arena_bytes = arena_bytes;
  char* A = ix->arena;
  ix->C = reinterpret_cast<float*>(A + plan.C);
  ix->cnorm = reinterpret_cast<float*>(A + plan.cnorm);
  ix->crec = A + plan.crec;
  ListDev& L = ix->L;
  L.len = reinterpret_cast<int32_t*>(A + plan.L_len);
  L.head = reinterpret_cast<int32_t*>(A + plan.L_head);
  L.tail = reinterpret_cast<int32_t*>(A + plan.L_tail);
  L.cnt = reinterpret_cast<int32_t*>(A + plan.L_cnt);
  L.cursor = reinterpret_cast<int32_t*>(A + plan.L_cursor);
  L.olen = reinterpret_cast<int32_t*>(A + plan.L_olen);
  L.otail = reinterpret_cast<int32_t*>(A + plan.L_otail);
  L.first = reinterpret_cast<int32_t*>(A + plan.L_first);
  L.meta = reinterpret_cast<int32_t*>(A + plan.L_meta);
  L.next = reinterpret_cast<int32_t*>(A + plan.next);
  L.pool = reinterpret_cast<int64_t*>(A + plan.pool);
  L.chunks = (int32_t)plan.chunks;
  L.K = K;
  hipError_t e = hipSuccess;
  for (int k = 0; k < kSlots && e == hipSuccess; ++k) {
    Slot& s = ix->slots[k];
    char* b = A + plan.slot[k];
    s.X = reinterpret_cast<float*>(b); b += al((size_t)max_step_rows * d * 4);
    s.ids = reinterpret_cast<int64_t*>(b); b += al((size_t)max_step_rows * 8);
    s.live = reinterpret_cast<int64_t*>(b); b += al(8);
    s.prim = reinterpret_cast<int32_t*>(b); b += al((size_t)max_step_rows * 4);
    s.spill = reinterpret_cast<int32_t*>(b); b += al((size_t)max_step_rows * 4);
    s.status = reinterpret_cast<unsigned*>(b); b += al(64);
    s.ws = b;
    s.counters = reinterpret_cast<unsigned*>(b);
    e = hipStreamCreate(&s.st);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev_results, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev_append, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev_done, hipEventDisableTiming);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&s.h_in),
                        8 + (size_t)max_step_rows * 8 + (size_t)max_step_rows * d * 4, 0);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&s.h_out),
                        (size_t)max_step_rows * 8 + CNT_WORDS * 4 + 16, 0);
  }
  hipStream_t st0 = ix->slots[0].st;
  // resident codebook, its norms (and maximum norm in every slot's counters), packed records
  if (e == hipSuccess)
    e = hipMemcpyAsync(ix->C, C, (size_t)K * d * 4, hipMemcpyDefault, st0);
  for (int k = 0; k < kSlots && e == hipSuccess; ++k)
    e = launch_prep_codebook(ix->C, K, d, ix->cnorm, ix->slots[k].counters, st0);
  if (e == hipSuccess && precision != SOAR_FP32)
    e = launch_lowp_pack_codebook(fmt, ix->C, K, d, ix->cnorm, ix->crec, ix->slots[0].counters, st0);
  if (e == hipSuccess && precision == SOAR_FP32)
    e = launch_pack_fp32(ix->C, K, d, ix->cnorm, ix->crec, st0);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(fill_i32, dim3((K + 255) / 256), dim3(256), 0, st0, L.len, (int64_t)K, 0);
    hipLaunchKernelGGL(fill_i32, dim3((K + 255) / 256), dim3(256), 0, st0, L.head, (int64_t)K, -1);
    hipLaunchKernelGGL(fill_i32, dim3((K + 255) / 256), dim3(256), 0, st0, L.tail, (int64_t)K, -1);
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st0, L.meta, (int64_t)16, 0);
    e = hipGetLastError();
  }
  unsigned cflags[CNT_WORDS] = {0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(cflags, ix->slots[0].counters, CNT_WORDS * 4, hipMemcpyDeviceToHost, st0);
  if (e == hipSuccess) e = hipStreamSynchronize(st0);
  if (e != hipSuccess) { free_index(ix); return SOAR_E_DEVICE; }
  if (cflags[CNT_NONFINITE]) { free_index(ix); return SOAR_E_NONFINITE; }
  // graphs of the slots
  for (int k = 0; k < kSlots && e == hipSuccess; ++k) {
    Slot& s = ix->slots[k];
    e = capture(s.st, &s.g_compute, [&] { return enqueue_compute(ix, s); });
    if (e == hipSuccess) e = capture(s.st, &s.g_append, [&] { return enqueue_append(ix, s); });
  }
  if (e != hipSuccess) { free_index(ix); return SOAR_E_DEVICE; }
  for (Slot& s : ix->slots) s.waiter = std::thread(slot_loop, ix, std::ref(s));
  ix->worker = std::thread(worker_loop, ix);
  *out = ix;
  return SOAR_OK;
}

soar_status soar_insert(soar_index* ix, const float* X_host, int64_t n, int64_t first_id,
                        uint64_t* ticket) {
  if (!ix || !X_host || !ticket || n < 1) return SOAR_E_INVAL;
  if (worst_chunks(std::min<int64_t>(n, 1), ix->K) > ix->L.chunks ||
      (2 * n + LIST_CH - 1) / LIST_CH > (int64_t)ix->L.chunks)
    return SOAR_E_NOMEM;   // can never fit
  auto r = std::make_shared<Request>();
  r->n = n;
  r->first_id = first_id;
  r->X.assign(X_host, X_host + n * ix->d);
  r->prim.assign(n, -1);
  r->spill.assign(n, -1);
  {
    std::lock_guard<std::mutex> g(ix->mu);
    if (ix->shutdown) return SOAR_E_SHUTDOWN;
    if (ix->list_error) return SOAR_E_NOMEM;
    r->ticket = ix->next_ticket++;
    ix->tickets[r->ticket] = r;
    ix->queue.push_back(r);
    ix->stats.requests += 1;
  }
  ix->cv_work.notify_all();
  *ticket = r->ticket;
  return SOAR_OK;
}

soar_status soar_wait(soar_index* ix, uint64_t ticket, int32_t* primary_host, int32_t* spill_host,
                      double timeout_s) {
  if (!ix) return SOAR_E_INVAL;
  std::unique_lock<std::mutex> lk(ix->mu);
  auto it = ix->tickets.find(ticket);
  if (it == ix->tickets.end()) return SOAR_E_INVAL;
  std::shared_ptr<Request> r = it->second;
  auto done = [&] { return r->complete; };
  if (timeout_s < 0) ix->cv_done.wait(lk, done);
  else if (!ix->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
    return SOAR_E_TIMEOUT;
  if (primary_host) std::memcpy(primary_host, r->prim.data(), r->n * 4);
  if (spill_host) std::memcpy(spill_host, r->spill.data(), r->n * 4);
  const soar_status s = r->status;
  ix->tickets.erase(ticket);
  return s;
}

soar_status soar_index_list(soar_index* ix, int32_t part, int64_t* ids_host, int64_t cap,
                            int64_t* len) {
  if (!ix || !len || part < 0 || part >= ix->K || cap < 0 || (cap > 0 && !ids_host))
    return SOAR_E_INVAL;
  std::unique_lock<std::mutex> lk(ix->mu);
  // hold new steps and let the ones in flight (and their list appends) finish
  ++ix->paused;
  ix->cv_done.wait(lk, [&] { return ix->in_flight == 0; });
  hipStream_t st = ix->slots[0].st;
  int32_t meta[3] = {0, -1, 0};
  std::vector<int32_t> next;
  hipError_t e = hipMemcpyAsync(&meta[0], ix->L.len + part, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&meta[1], ix->L.head + part, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&meta[2], ix->L.meta, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const int32_t n = meta[0];
  const int64_t want = std::min<int64_t>(n, cap);
  if (e == hipSuccess && want > 0) {
    // the chunk links in use, then the chain from the head
    next.resize(std::max(1, meta[2]));
    e = hipMemcpyAsync(next.data(), ix->L.next, (size_t)meta[2] * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int32_t c = meta[1];
    for (int64_t k = 0; e == hipSuccess && k * LIST_CH < want && c >= 0 && c < meta[2]; ++k) {
      const int64_t m = std::min<int64_t>(LIST_CH, want - k * LIST_CH);
      e = hipMemcpyAsync(ids_host + k * LIST_CH, ix->L.pool + (int64_t)c * LIST_CH, m * 8,
                         hipMemcpyDeviceToHost, st);
      c = next[c];
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  const bool bad = ix->list_error;
  --ix->paused;
  lk.unlock();
  ix->cv_work.notify_all();
  *len = n;
  if (e != hipSuccess) return SOAR_E_DEVICE;
  return bad ? SOAR_E_NOMEM : SOAR_OK;
}

soar_status soar_index_get_stats(soar_index* ix, soar_index_stats* out) {
  if (!ix || !out || out->struct_size < sizeof(soar_index_stats)) return SOAR_E_INVAL;
  std::lock_guard<std::mutex> g(ix->mu);
  const uint32_t sz = out->struct_size;
  *out = ix->stats;
  out->struct_size = sz;
  out->chunks_used = ix->chunks_used;
  out->chunks_total = ix->L.chunks;
  return SOAR_OK;
}

void soar_index_destroy(soar_index* ix) {
  if (!ix) return;
  {
    std::lock_guard<std::mutex> g(ix->mu);
    ix->shutdown = true;
  }
  ix->cv_work.notify_all();
  if (ix->worker.joinable()) ix->worker.join();
  {
    // the queue is empty now; wait for the steps in flight, then release the waiters
    std::unique_lock<std::mutex> lk(ix->mu);
    ix->cv_done.wait(lk, [&] { return ix->in_flight == 0; });
    for (Slot& s : ix->slots) s.cv.notify_all();
  }
  for (Slot& s : ix->slots)
    if (s.waiter.joinable()) s.waiter.join();
  free_index(ix);
}

}  // extern "C"
