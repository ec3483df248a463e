// C-ABI entry points of the SOAR library: argument validation, workspace layout, launches and
// status reporting.  Every computation runs in the HIP kernels; this file only plans and orders
// them on the caller's stream.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/soar.h"
#include "common.h"
#include "kernels.h"
#include "train.h"

namespace {

using soar::AssignParams;

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carves a caller-provided workspace into aligned sub-buffers.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* p) : base(static_cast<char*>(p)) {}
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline soar_status dev_err(hipError_t e) { return e == hipSuccess ? SOAR_OK : SOAR_E_DEVICE; }

struct OptsView {
  float lambda = 1.f;
  int precision = SOAR_FP32;
  int topk = 0;
  float near_tie_rel = 0.f;
  uint32_t flags = 0;
};

bool read_opts(const soar_assign_opts* o, OptsView* v) {
  if (!o || o->struct_size < offsetof(soar_assign_opts, flags) + sizeof(uint32_t)) return false;
  v->lambda = o->lambda;
  v->precision = o->precision;
  v->topk = o->topk;
  v->near_tie_rel = o->near_tie_rel;
  v->flags = o->flags;
  return true;
}

soar_status validate_assign(int64_t n, int32_t d, int32_t K, const OptsView& o) {
  if (n < 1 || n > INT32_MAX || d < 1 || K < 2) return SOAR_E_INVAL;
  if (!std::isfinite(o.lambda) || o.lambda < 0.f) return SOAR_E_INVAL;
  if ((o.flags & SOAR_SPILL_GROUPED) && (o.flags & SOAR_SPILL_DIRECT)) return SOAR_E_INVAL;
  if ((o.flags & SOAR_NO_BOUND) && (o.flags & SOAR_BOUND_ALWAYS)) return SOAR_E_INVAL;
  if (!(o.near_tie_rel >= 0.f) || !std::isfinite(o.near_tie_rel)) return SOAR_E_INVAL;
  if (o.precision == SOAR_FP32) return soar::fp32_padded_dim(d) < 0 ? SOAR_E_UNSUPPORTED : SOAR_OK;
  if (o.precision != SOAR_BF16 && o.precision != SOAR_FP8_E4M3) return SOAR_E_INVAL;
  if (o.topk < 0 || o.topk > 16) return SOAR_E_INVAL;
  const int fmt = o.precision == SOAR_BF16 ? soar::LOWP_BF16 : soar::LOWP_FP8;
  if (soar::lowp_padded_dim(fmt, d) < 0) return SOAR_E_UNSUPPORTED;
  return SOAR_OK;
}

struct LowpLayout {
  unsigned* counters;
  float* cnorm;
  void* Xq;
  void* Cq;
  void* Rq;
  float* xs;
  float* cs;
  float4* rowc;
  int32_t* cand_p;      // [n x topk] candidates of the primary sweep
  int32_t* cand;        // [n x topk] candidates of the spill sweep
  void* Cp;             // codebook rows quantized like X (grouped spill form)
  float* cps;
  void* group;
  float* radius;        // [n] spill bound: each row's radius around its primary centroid
  int32_t* gkey;        // [n] group key of the spill sweep (-1: bounded row)
  void* bound;          // the bound's table, sample and flag (bound_layout)
  size_t bytes;
};

LowpLayout layout_lowp(void* ws, int64_t n, int32_t d, int32_t K, int fmt, int topk) {
  const int dp = soar::lowp_padded_dim(fmt, d);
  const size_t eb = fmt == soar::LOWP_BF16 ? 2 : 1;
  Carver c(ws);
  LowpLayout L;
  L.counters = c.take<unsigned>(soar::CNT_ALLOC_WORDS);
  L.cnorm = c.take<float>((size_t)K);
  L.Xq = c.take<char>((size_t)n * dp * eb);
  L.Cq = c.take<char>(soar::lowp_codebook_bytes(fmt, d, K));
  L.Rq = c.take<char>((size_t)n * dp * eb);
  L.xs = c.take<float>((size_t)n);
  L.cs = c.take<float>((size_t)K);
  L.rowc = c.take<float4>((size_t)n);
  L.cand_p = c.take<int32_t>((size_t)n * topk);
  L.cand = c.take<int32_t>((size_t)n * topk);
  L.Cp = c.take<char>((size_t)K * dp * eb);
  L.cps = c.take<float>((size_t)K);
  L.group = c.take<char>(soar::group_layout(nullptr, n, K).bytes);
  L.radius = c.take<float>((size_t)n);
  L.gkey = c.take<int32_t>((size_t)n);
  L.bound = c.take<char>(soar::bound_layout(nullptr, K, topk < soar::kBoundMaxM ? topk
                                                                         : soar::kBoundMaxM).bytes);
  L.bytes = c.off;
  return L;
}

inline int lowp_fmt(const OptsView& o) {
  return o.precision == SOAR_BF16 ? soar::LOWP_BF16 : soar::LOWP_FP8;
}
// Default candidates re-scored per row: the 8 smallest kept approximate values.
inline int lowp_topk(const OptsView& o, int) { return o.topk > 0 ? o.topk : 8; }

struct AssignLayout {
  unsigned* counters;
  float* cnorm;
  char* crec;
  float* gram;          // [K x K] when the spill sweep uses the Gram form
  int32_t* full_rows;
  void* group;          // grouping of rows by primary (grouped form of the spill sweep)
  size_t bytes;
};

AssignLayout layout_assign(void* ws, int64_t n, int32_t d, int32_t K) {
  Carver c(ws);
  AssignLayout L;
  L.counters = c.take<unsigned>(soar::CNT_ALLOC_WORDS);
  L.cnorm = c.take<float>((size_t)K);
  L.crec = c.take<char>(soar::fp32_codebook_bytes(d, K));
  L.gram = soar::fp32_uses_gram(d, K) ? c.take<float>((size_t)K * K) : nullptr;
  L.full_rows = c.take<int32_t>((size_t)n);
  L.group = c.take<char>(soar::group_layout(nullptr, n, K).bytes);
  L.bytes = c.off;
  return L;
}

struct FurtherLayout {
  unsigned* counters;
  float* cnorm;
  char* crec;
  int32_t* full_rows;
  size_t bytes;
};

FurtherLayout layout_further(void* ws, int64_t n, int32_t d, int32_t K) {
  Carver c(ws);
  FurtherLayout L;
  L.counters = c.take<unsigned>(soar::CNT_ALLOC_WORDS);
  L.cnorm = c.take<float>((size_t)K);
  L.crec = c.take<char>(soar::fp32_further_codebook_bytes(d, K));
  L.full_rows = c.take<int32_t>((size_t)n);
  L.bytes = c.off;
  return L;
}

soar_status validate_further(int64_t n, int32_t d, int32_t K, int32_t m, float lambda,
                             float near_tie_rel) {
  if (n < 1 || n > INT32_MAX || d < 1 || m < 1 || m > soar::kFurtherMaxPrior || K <= m)
    return SOAR_E_INVAL;
  if (!std::isfinite(lambda) || lambda < 0.f) return SOAR_E_INVAL;
  if (!(near_tie_rel >= 0.f) || !std::isfinite(near_tie_rel)) return SOAR_E_INVAL;
  return soar::fp32_further_padded_dim(d) < 0 ? SOAR_E_UNSUPPORTED : SOAR_OK;
}

}  // namespace

namespace soar {

// Screening bands: twice the rounding-error bound of centroid j's expanded ranking value, with a
// 10% margin.  With T_j = ||x|| + ||c_j||:
//   primary  |(||c||^2 - 2<x,c>)~ - exact| <= gamma_{d+2} T_j^2 (norm, dot product, fma);
//   spill    adds the penalty: lambda/||r||^2 * e^2 with |e| <= ||r|| ||x - c_j|| <= ||r|| T_j
//            and |e~ - e| <= gamma_{d+2} ||r|| T_j, so its error is <= 3 lambda gamma_{d+4} T_j^2,
//            plus the final roundings; in all <= (1 + 3 lambda) gamma_{d+5} T_j^2.
float band_coef_primary(int d) { return 2.2f * (float)(d + 2) * kU32; }
float band_coef_spill(int d, float lam) {
  return 2.2f * (1.f + 3.f * lam) * (float)(d + 5) * kU32;
}
// Gram form of the spill screen: <r, c_j> is formed as <x, c_j> - <c_pi, c_j>, whose error (with
// that of <r, x>) is gamma_{d+2} P T_j, P = ||x|| + ||c_pi|| (>= ||r||), instead of
// gamma_{d+2} ||r|| T_j.  Through lambda/||r||^2 * e^2 with |e| <= ||r|| T_j that adds
// 2 lambda gamma_{d+2} P T_j^2 / ||r|| and lambda gamma_{d+2}^2 P^2 T_j^2 / ||r||^2 to the error
// bound (again doubled, with a 10% margin).
float band_coef_gram1(int d, float lam) { return 2.2f * 2.f * lam * (float)(d + 2) * kU32; }
float band_coef_gram2(int d, float lam) {
  const float g = (float)(d + 2) * kU32;
  return 2.2f * lam * g * g;
}
float tie_threshold(int d, float lam, float near_tie_rel) {
  const float rel = near_tie_rel > 0.f ? near_tie_rel : 1e-5f;
  const float err = (1.f + 3.f * lam) * ((float)d / 16.f + 6.f) * kU32;
  return fmaxf(rel, 3.f * err);
}

// Shared by soar_assign and the training loop: primary-only (labels) or full SOAR.
// spill_form: 0 = chosen here, SOAR_SPILL_GROUPED or SOAR_SPILL_DIRECT.
soar_status run_assign_fp32(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                            float lam, float near_tie_rel, bool spill, int32_t* primary,
                            int32_t* spill_out, float* pdist, float* sloss, void* ws,
                            hipStream_t st, unsigned* counters_out_host, hipEvent_t* ev,
                            uint32_t spill_form) {
  AssignLayout L = layout_assign(ws, n, d, K);
  AssignParams P;
  P.X = X; P.n = n; P.d = d; P.C = C; P.K = K; P.Crec = L.crec;
  P.cnorm = L.cnorm; P.counters = L.counters;
  P.lam = lam;
  P.tie_rel = tie_threshold(d, lam, near_tie_rel);
  P.band_p = band_coef_primary(d);
  P.band_s = band_coef_spill(d, lam);
  P.primary = primary; P.spill = spill_out; P.pdist = pdist; P.sloss = sloss;
  P.full_rows = L.full_rows;
  const bool grouped = spill &&
                       (spill_form == SOAR_SPILL_GROUPED ||
                        (spill_form == 0 && grouped_spill_pays(n, K)));
  const bool gram = spill && !grouped && L.gram != nullptr;
  if (gram) P.G = L.gram;
  if (gram || grouped) {
    P.band_g1 = band_coef_gram1(d, lam);
    P.band_g2 = band_coef_gram2(d, lam);
  }
  const GroupLayout GL = group_layout(L.group, n, K);
  const bool vec = (d % 4 == 0) && aligned(X, 16) && aligned(C, 16);
  if (ev) (void)hipEventRecord(ev[0], st);
  hipError_t e = launch_prep_codebook(C, K, d, L.cnorm, L.counters, st);
  if (e == hipSuccess) e = launch_pack_fp32(C, K, d, L.cnorm, L.crec, st);
  if (e == hipSuccess && gram) e = launch_gram(C, K, d, L.gram, st);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess)
    e = launch_assign_fp32(P, spill, vec, st, ev ? ev + 2 : nullptr, grouped ? &GL : nullptr);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[6], st);
  if (e != hipSuccess) return SOAR_E_DEVICE;
  if (counters_out_host) {
    e = hipMemcpyAsync(counters_out_host, L.counters, CNT_WORDS * sizeof(unsigned),
                       hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return SOAR_E_DEVICE;
  }
  return SOAR_OK;
}

size_t assign_workspace_bytes(int64_t n, int32_t d, int32_t K) {
  return layout_assign(nullptr, n, d, K).bytes;
}

// A second stream per device (created on first use, kept for the process) on which the spill
// bound's table runs beside the quantization and the primary sweep: the table waits mostly on
// latency and fits beside the sweep's workgroups on a CU.  Default priority, non-blocking.
hipStream_t side_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}

// BF16 / FP8 pipeline: quantize, primary sweep + re-score, spill sweep + re-score.
soar_status run_assign_lowp(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                            float lam, float near_tie_rel, int fmt, int topk, int32_t* primary,
                            int32_t* spill_out, float* pdist, float* sloss, void* ws,
                            hipStream_t st, unsigned* counters_out_host, hipEvent_t* ev,
                            uint32_t flags) {
  LowpLayout L = layout_lowp(ws, n, d, K, fmt, topk);
  const uint32_t spill_form = flags & (SOAR_SPILL_GROUPED | SOAR_SPILL_DIRECT);
  // The grouped form trades the second MFMA stream for epilogue work.  Over residual rows
  // (lambda >= kGroupedResidualMinLam) that work is the direct form's one fma per element, so it
  // pays wherever grouping does: n=10M, d=96, K=40,000, BF16 149.5 vs 186.0 ms per call, FP8
  // 169.1 vs 178.5 ms; FP8 at d=768, n=500K, 7.5 vs 10.3 ms.  Over X rows (small lambda) the
  // form costs about two more VALU operations per element, which pays only where the direct
  // form's two B operands per LDS fetch bound it (FP8 rows of 512 dimensions and more).
  const bool grouped = spill_form == SOAR_SPILL_GROUPED ||
                       (spill_form == 0 && grouped_spill_pays(n, K) &&
                        (grouped_residual_rows(fmt, lam) ||
                         (fmt != LOWP_BF16 && lowp_padded_dim(fmt, d) >= 512)));
  const GroupLayout GL = group_layout(L.group, n, K);
  // The spill bound (bound.hip) serves the grouped form: rows it decides leave the grouping, and
  // the spill sweep runs over the rest.
  // The spill bound: a sample decides on the device whether its table pays, for calls of at
  // least 2^40 n K d (below that the sample's fixed cost, a few dependent launches, weighs more
  // than the sweep it could save); SOAR_BOUND_ALWAYS builds the table regardless.
  const bool always = (flags & SOAR_BOUND_ALWAYS) != 0;
  const bool bound = grouped && topk <= kBoundMaxM && !(flags & SOAR_NO_BOUND) &&
                     (always || (double)n * K * d >= 1099511627776.0);
  LowpParams P;
  P.n = n; P.d = d; P.dp = lowp_padded_dim(fmt, d); P.K = K; P.topk = topk;
  P.lam = lam;
  P.tie_rel = tie_threshold(d, lam, near_tie_rel);
  P.X = X; P.C = C; P.Xq = L.Xq; P.Cq = L.Cq; P.Rq = L.Rq;
  P.xs = L.xs; P.cs = L.cs; P.cnorm = L.cnorm; P.rowc = L.rowc; P.cand = L.cand_p;
  P.primary = primary; P.spill = spill_out; P.pdist = pdist; P.sloss = sloss;
  P.counters = L.counters; P.rowc_out = L.rowc;
  P.Rq_out = grouped && !grouped_residual_rows(fmt, lam) ? nullptr : L.Rq;
  if (grouped) {
    P.perm = GL.perm; P.stripes = GL.stripes; P.nstripes = GL.meta;
    P.Cp = L.Cp; P.cps = L.cps;
  }
  auto mark = [&](int k) { return ev ? hipEventRecord(ev[k], st) : hipSuccess; };
  hipError_t e = mark(0);
  if (e == hipSuccess) e = launch_prep_codebook(C, K, d, L.cnorm, L.counters, st);
  if (e == hipSuccess)
    e = launch_lowp_pack_codebook(fmt, C, K, d, L.cnorm, L.Cq, L.counters, st);
  if (e == hipSuccess && grouped)
    e = launch_lowp_quantize(fmt, C, K, d, P.dp, false, L.Cp, L.cps, L.counters, st);
  // the spill bound's table (only where a sample says it pays: FP8's sweep costs about half
  // BF16's per row, so there it must decide more rows)
  const BoundLayout BL = bound_layout(L.bound, K, bound ? topk : 1);
  // the table forks off to the side stream once the codebook norms are ready and joins back
  // before the decisions (it reads X, C and the norms, and writes only its own workspace part);
  // without a side stream it runs in place
  hipStream_t side = bound && !(flags & kLowpNoSideStream) ? side_stream() : nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // on every return: the caller's stream waits for the side stream's part (a no-op when the
  // join was never recorded), then the events go (their release waits for their completion)
  struct Joined {
    hipStream_t st;
    hipStream_t& side;
    hipEvent_t& fork;
    hipEvent_t& join;
    ~Joined() {
      if (side && join) (void)hipStreamWaitEvent(st, join, 0);
      if (fork) (void)hipEventDestroy(fork);
      if (join) (void)hipEventDestroy(join);
    }
  } joined{st, side, fork, join};
  if (side && (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
               hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess))
    side = nullptr;
  if (e == hipSuccess && bound) {
    const int payoff = always ? 0 : fmt == LOWP_BF16 ? 32 : 48;
    if (side) {
      e = hipEventRecord(fork, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
      if (e == hipSuccess) e = launch_bound_table(X, n, C, K, d, L.cnorm, topk, lam, BL, payoff, side);
      if (e == hipSuccess) e = hipEventRecord(join, side);
    } else {
      e = launch_bound_table(X, n, C, K, d, L.cnorm, topk, lam, BL, payoff, st);
    }
  }
  if (e == hipSuccess)
    e = launch_lowp_quantize(fmt, X, n, d, P.dp, false, L.Xq, L.xs, L.counters, st);
  if (e == hipSuccess) e = mark(1);
  if (e == hipSuccess) e = launch_lowp_sweep(fmt, P, false, st);
  if (e == hipSuccess) e = mark(2);
  if (bound) P.radius = L.radius;
  if (e == hipSuccess) e = launch_lowp_rescore(fmt, P, false, st);
  P.radius = nullptr;
  if (e == hipSuccess) e = mark(3);
  P.cand = L.cand;
  if (grouped) {
    // rows the spill bound decides
    if (e == hipSuccess && side) e = hipStreamWaitEvent(st, join, 0);
    if (e == hipSuccess && bound)
      e = launch_bound_decide(topk, n, K, primary, L.radius, BL, L.cand, L.gkey, st);
    if (e == hipSuccess)
      e = launch_group_by_primary(bound ? L.gkey : primary, n, nullptr, K, GL, st);
    if (e == hipSuccess && bound) e = launch_bound_count(GL.off, K, n, L.counters, st);
    if (e == hipSuccess) e = mark(4);
    if (e == hipSuccess) e = launch_lowp_sweep_grouped(fmt, P, st);
  } else {
    if (e == hipSuccess) e = mark(4);
    if (e == hipSuccess) e = launch_lowp_sweep(fmt, P, true, st);
  }
  if (e == hipSuccess) e = mark(5);
  if (e == hipSuccess) e = launch_lowp_rescore(fmt, P, true, st);
  if (e == hipSuccess) e = mark(6);
  if (e != hipSuccess) return SOAR_E_DEVICE;
  if (counters_out_host &&
      hipMemcpyAsync(counters_out_host, L.counters, CNT_WORDS * sizeof(unsigned),
                     hipMemcpyDeviceToHost, st) != hipSuccess)
    return SOAR_E_DEVICE;
  return SOAR_OK;
}

}  // namespace soar

namespace {

// One assignment on a validated, large enough workspace.  A blocking call reads the counters
// (and the status record an enqueue-only call left in the same workspace) and clears the record.
soar_status assign_impl(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                        const OptsView& o, int32_t* primary, int32_t* spill, float* primary_dist,
                        float* spill_loss, void* workspace, hipStream_t st, soar_stats* stats,
                        bool side_ok) {
  const bool async = (o.flags & SOAR_ASYNC) != 0;
  const bool lowp = o.precision != SOAR_FP32;
  // the counters lead both workspace layouts
  unsigned* counters = static_cast<unsigned*>(workspace);
  hipEvent_t ev[soar::kPhaseEvents] = {};
  auto destroy = [&]() {
    for (hipEvent_t& e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  if (!async && stats) {
    for (hipEvent_t& e : ev)
      if (hipEventCreate(&e) != hipSuccess) { destroy(); return SOAR_E_DEVICE; }
  }
  unsigned cnt[soar::CNT_WORDS] = {0};
  const uint32_t form = o.flags & (SOAR_SPILL_GROUPED | SOAR_SPILL_DIRECT);
  const uint32_t lowp_flags = form | (o.flags & (SOAR_NO_BOUND | SOAR_BOUND_ALWAYS)) |
                              (side_ok ? 0u : soar::kLowpNoSideStream);
  soar_status s;
  if (!lowp)
    s = soar::run_assign_fp32(X, n, d, C, K, o.lambda, o.near_tie_rel, true, primary, spill,
                              primary_dist, spill_loss, workspace, st, async ? nullptr : cnt,
                              ev[0] ? ev : nullptr, form);
  else
    s = soar::run_assign_lowp(X, n, d, C, K, o.lambda, o.near_tie_rel, lowp_fmt(o),
                              lowp_topk(o, d), primary, spill, primary_dist, spill_loss, workspace,
                              st, async ? nullptr : cnt, ev[0] ? ev : nullptr, lowp_flags);
  if (s != SOAR_OK) { destroy(); return s; }
  if (async) {
    destroy();
    return dev_err(soar::launch_async_note(counters, st));
  }
  unsigned rec[3] = {0u, 0u, 0u};
  hipError_t e = hipMemcpyAsync(rec, counters + soar::CNT_ASYNC_M0, sizeof(rec),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = soar::launch_async_clear(counters, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  s = dev_err(e);
  if (s == SOAR_OK && stats) {
    float ph[soar::kPhaseEvents - 1] = {};
    for (int k = 0; k + 1 < soar::kPhaseEvents; ++k)
      (void)hipEventElapsedTime(&ph[k], ev[k], ev[k + 1]);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[soar::kPhaseEvents - 1]);
    stats->device_ms = ms;
    // the sweeps and the grouping by primary
    stats->assign_kernel_ms = ph[1] + ph[3] + ph[4];
    stats->rows_full_scan = cnt[soar::CNT_FULLSCAN];
    stats->rows_fp64 = cnt[soar::CNT_FP64];
    stats->mfma_flops = 4.0 * (double)n * (double)K * (double)d;
    for (int k = 0; k < 6; ++k) stats->phase_ms[k] = ph[k];
    if (stats->struct_size >= offsetof(soar_stats, rows_bounded) + sizeof(int64_t))
      stats->rows_bounded = cnt[soar::CNT_BOUNDED];
  }
  destroy();
  const bool async_bad = rec[0] == soar::kAsyncMagic0 && rec[1] == soar::kAsyncMagic1 && rec[2];
  if (s == SOAR_OK && (cnt[soar::CNT_NONFINITE] || async_bad)) s = SOAR_E_NONFINITE;
  return s;
}

}  // namespace

namespace soar {

soar_status assign_validate(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                            const soar_assign_opts* opts, const int32_t* primary,
                            const int32_t* spill, size_t* need) {
  OptsView o;
  if (!read_opts(opts, &o)) return SOAR_E_INVAL;
  soar_status s = validate_assign(n, d, K, o);
  if (s != SOAR_OK) return s;
  if (!X || !C || !primary || !spill) return SOAR_E_INVAL;
  if (!aligned(X, 4) || !aligned(C, 4)) return SOAR_E_INVAL;
  *need = o.precision == SOAR_FP32 ? assign_workspace_bytes(n, d, K)
                                   : layout_lowp(nullptr, n, d, K, lowp_fmt(o), lowp_topk(o, d)).bytes;
  return SOAR_OK;
}

soar_status assign_run(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                       const soar_assign_opts* opts, int32_t* primary, int32_t* spill,
                       float* primary_dist, float* spill_loss, void* workspace, hipStream_t st,
                       soar_stats* stats, bool side_stream) {
  OptsView o;
  if (!read_opts(opts, &o)) return SOAR_E_INVAL;
  return assign_impl(X, n, d, C, K, o, primary, spill, primary_dist, spill_loss, workspace, st,
                     stats, side_stream);
}

}  // namespace soar

extern "C" {

const char* soar_status_string(soar_status s) {
  switch (s) {
    case SOAR_OK: return "ok";
    case SOAR_E_INVAL: return "invalid argument";
    case SOAR_E_NOMEM: return "out of memory (arena or request too large)";
    case SOAR_E_DEVICE: return "device error";
    case SOAR_E_UNSUPPORTED: return "unsupported shape or precision";
    case SOAR_E_NONFINITE: return "non-finite value in X or C";
    case SOAR_E_TIMEOUT: return "timed out";
    case SOAR_E_SHUTDOWN: return "index is shutting down";
  }
  return "unknown status";
}

soar_status soar_assign_workspace_size(int64_t n, int32_t d, int32_t K,
                                       const soar_assign_opts* opts, size_t* bytes) {
  OptsView o;
  if (!bytes || !read_opts(opts, &o)) return SOAR_E_INVAL;
  const soar_status s = validate_assign(n, d, K, o);
  if (s != SOAR_OK) return s;
  *bytes = o.precision == SOAR_FP32
               ? soar::assign_workspace_bytes(n, d, K)
               : layout_lowp(nullptr, n, d, K, lowp_fmt(o), lowp_topk(o, d)).bytes;
  return SOAR_OK;
}

soar_status soar_assign_candidates(int64_t n, int32_t d, int32_t K, const soar_assign_opts* opts,
                                   size_t* primary_off, size_t* spill_off, int32_t* topk,
                                   size_t* bound_key_off) {
  OptsView o;
  if (!primary_off || !spill_off || !topk || !read_opts(opts, &o)) return SOAR_E_INVAL;
  const soar_status s = validate_assign(n, d, K, o);
  if (s != SOAR_OK) return s;
  if (o.precision == SOAR_FP32) return SOAR_E_UNSUPPORTED;
  // the layout of a workspace placed at a stand-in address: only the offsets are used
  char* base = reinterpret_cast<char*>(kAlign);
  const LowpLayout L = layout_lowp(base, n, d, K, lowp_fmt(o), lowp_topk(o, d));
  *primary_off = reinterpret_cast<char*>(L.cand_p) - base;
  *spill_off = reinterpret_cast<char*>(L.cand) - base;
  if (bound_key_off) *bound_key_off = reinterpret_cast<char*>(L.gkey) - base;
  *topk = lowp_topk(o, d);
  return SOAR_OK;
}

soar_status soar_spill_further_workspace_size(int64_t n, int32_t d, int32_t K, int32_t m,
                                             size_t* bytes) {
  if (!bytes) return SOAR_E_INVAL;
  const soar_status s = validate_further(n, d, K, m, 0.f, 0.f);
  if (s != SOAR_OK) return s;
  *bytes = layout_further(nullptr, n, d, K).bytes;
  return SOAR_OK;
}

soar_status soar_spill_further(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                               const int32_t* prior, int32_t m, float lambda, float near_tie_rel,
                               int32_t* next, float* next_loss, void* workspace, size_t ws_bytes,
                               void* stream, soar_stats* stats) {
  soar_status s = validate_further(n, d, K, m, lambda, near_tie_rel);
  if (s != SOAR_OK) return s;
  if (!X || !C || !prior || !next || !aligned(X, 4) || !aligned(C, 4) || !aligned(prior, 4))
    return SOAR_E_INVAL;
  const FurtherLayout L = layout_further(workspace, n, d, K);
  if (!workspace || !aligned(workspace, kAlign) || ws_bytes < L.bytes) return SOAR_E_INVAL;
  if (stats && stats->struct_size < offsetof(soar_stats, rows_bounded)) return SOAR_E_INVAL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t ev[2] = {};
  auto destroy = [&]() {
    for (hipEvent_t& e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  if (stats)
    for (hipEvent_t& e : ev)
      if (hipEventCreate(&e) != hipSuccess) { destroy(); return SOAR_E_DEVICE; }
  // the penalty has m terms, each bounded like the spill's: the bands of lambda m
  const float lam_m = lambda * (float)m;
  AssignParams P;
  P.X = X; P.n = n; P.d = d; P.C = C; P.K = K; P.Crec = L.crec;
  P.cnorm = L.cnorm; P.counters = L.counters;
  P.lam = lambda;
  P.tie_rel = soar::tie_threshold(d, lam_m, near_tie_rel);
  P.band_p = soar::band_coef_primary(d);
  P.band_s = soar::band_coef_spill(d, lam_m);
  P.primary = nullptr; P.spill = next; P.pdist = nullptr; P.sloss = next_loss;
  P.full_rows = L.full_rows;
  P.prior = prior;
  unsigned cnt[soar::CNT_WORDS] = {0};
  // the earlier assignments are checked before any kernel follows them
  hipError_t e = ev[0] ? hipEventRecord(ev[0], st) : hipSuccess;
  if (e == hipSuccess) e = soar::launch_prep_codebook(C, K, d, L.cnorm, L.counters, st);
  if (e == hipSuccess) e = soar::launch_check_priors(prior, n, m, K, L.counters, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cnt, L.counters, sizeof(cnt), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { destroy(); return SOAR_E_DEVICE; }
  if (cnt[soar::CNT_BADINPUT]) { destroy(); return SOAR_E_INVAL; }
  e = soar::launch_pack_fp32_further(C, K, d, L.cnorm, L.crec, st);
  if (e == hipSuccess) e = soar::launch_further_fp32(P, m, st);
  if (e == hipSuccess && ev[1]) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cnt, L.counters, sizeof(cnt), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  s = dev_err(e);
  if (s == SOAR_OK && stats) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    stats->device_ms = ms;
    stats->assign_kernel_ms = ms;
    stats->rows_full_scan = cnt[soar::CNT_FULLSCAN];
    stats->rows_fp64 = cnt[soar::CNT_FP64];
    stats->mfma_flops = 2.0 * (double)n * (double)K * (double)d * (double)(1 + m);
    for (int k = 0; k < 6; ++k) stats->phase_ms[k] = 0.f;
    stats->phase_ms[4] = ms;
  }
  destroy();
  if (s == SOAR_OK && cnt[soar::CNT_NONFINITE]) s = SOAR_E_NONFINITE;
  return s;
}

soar_status soar_assign(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                        const soar_assign_opts* opts, int32_t* primary, int32_t* spill,
                        float* primary_dist, float* spill_loss, void* workspace, size_t ws_bytes,
                        void* stream, soar_stats* stats) {
  size_t need = 0;
  const soar_status s = soar::assign_validate(X, n, d, C, K, opts, primary, spill, &need);
  if (s != SOAR_OK) return s;
  if (!workspace || !aligned(workspace, kAlign) || ws_bytes < need) return SOAR_E_INVAL;
  if (stats && stats->struct_size < offsetof(soar_stats, rows_bounded)) return SOAR_E_INVAL;
  return soar::assign_run(X, n, d, C, K, opts, primary, spill, primary_dist, spill_loss,
                          workspace, static_cast<hipStream_t>(stream), stats);
}

}  // extern "C"
