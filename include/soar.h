/*
 * soar.h -- C ABI of the MI355X (gfx950) SOAR assignment library.
 *
 * SOAR ("Spilling with Orthogonality-Amplified Residuals", Sun et al.) gives every datapoint x a
 * primary VQ partition and one spilled partition:
 *
 *   primary   pi(x)  = argmin_j ||x - C_j||^2                              (Section 2.2)
 *   residual  r      = x - C_pi(x)                                         (Section 3.1)
 *   spill     pi'(x) = argmin_{j != pi(x)} ||x - C_j||^2
 *                                + lambda * <r, x - C_j>^2 / ||r||^2        (Section 3.4, Eq. 2
 *                                                                            via Theorem 3.1)
 *
 * and the codebook C is trained by Lloyd k-means seeded by k-means++ (the paper trains VQ "as
 * usual" before spilling, Section 3.5).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers unless the comment says "host".  Matrices are row-major
 *    and contiguous: X is n x d, C is K x d, both float32.  Indices are 0-based int32 (the paper
 *    numbers partitions from 1).
 *  - The caller owns every buffer.  The library never frees caller memory and keeps no pointer
 *    after a call returns, except that a soar_index borrows its arena until soar_index_destroy.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are stream-ordered and, unless
 *    SOAR_ASYNC is set in a flags field, block until the device work has finished so that the
 *    returned status covers device-side errors.
 *  - Validation runs before any launch; on SOAR_E_INVAL / SOAR_E_UNSUPPORTED nothing is written,
 *    except for checks of array contents made on the device (indices in range), whose
 *    SOAR_E_INVAL comes after the call: each such call's comment says what it wrote.
 *    On SOAR_E_NONFINITE (a NaN or Inf in X or C) the outputs have been written but hold no
 *    meaning.  Nothing aborts and nothing throws across this interface.
 *  - Ties: an arg-min tie goes to the lowest index.  ||r|| = 0 makes the projection term 0.
 *    The primary is excluded from the spill by index only.
 */
#ifndef SOAR_H
#define SOAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum soar_status {
  SOAR_OK = 0,
  SOAR_E_INVAL = -1,        /* bad argument: sizes, null pointers, lambda, workspace, alignment */
  SOAR_E_NOMEM = -2,        /* a request does not fit the arena / internal allocation failed     */
  SOAR_E_DEVICE = -3,       /* a HIP call failed; the device context may be unusable             */
  SOAR_E_UNSUPPORTED = -4,  /* valid but not implemented for this shape or precision             */
  SOAR_E_NONFINITE = -5,    /* NaN or Inf found in X or C                                        */
  SOAR_E_TIMEOUT = -6,      /* soar_wait ran out of time; the ticket stays valid                 */
  SOAR_E_SHUTDOWN = -7      /* the index is shutting down                                        */
} soar_status;

typedef enum soar_precision {
  SOAR_FP32 = 0,            /* both contractions in FP32 on MFMA                                 */
  SOAR_BF16 = 1,            /* X, C, R as BF16 on MFMA, FP32 accumulate, FP32 re-score of top-k  */
  SOAR_FP8_E4M3 = 2         /* OCP e4m3 with per-row power-of-two scales, FP32 re-score of top-k */
} soar_precision;

/* flags bit: enqueue only.  Nothing is read back; a non-finite input found by such a call is
   kept in its workspace, and the next blocking soar_assign on the same workspace returns
   SOAR_E_NONFINITE (and clears it).  Stats are not filled. */
#define SOAR_ASYNC 1u
/* Form of the spill sweep (results are the same up to the low-precision candidate ranking; only
   the work differs).  The grouped form sorts the rows by primary and takes <c_pi, c_j> from the
   same MFMA stream as the rows (x, or with lambda >= 1/64 the residual r); the direct
   form runs a second stream over R = X - C[pi].  Without either bit the grouped form is taken when
   n >= 8 K and, for BF16, lambda >= 1/64; for FP8, d > 384 (FP32: at every d).
   Both bits: SOAR_E_INVAL. */
#define SOAR_SPILL_GROUPED 2u
#define SOAR_SPILL_DIRECT 4u
/* BF16/FP8, grouped form, topk <= 8: the spill bound is on by default.  A row with primary p
   whose nearest other re-scored candidate j2 gives U = (1 + lambda) ||x - C_j2||^2 has its spill
   within ||r|| + sqrt(U) of C_p (the penalty lies between 0 and lambda ||x - C_j||^2, then the
   triangle inequality; Section 3.4's loss).  When the topk centroids nearest to C_p include all
   centroids that close (FP32 distances lowered by their rounding bound), those topk are the row's
   spill candidates, re-scored exactly, and the row skips the spill sweep.  The bound needs a
   table of every centroid's topk nearest centroids (2 K^2 d FP32 flop); for calls of at least
   2^40 n K d a sample of 256 rows decides on the device whether it pays (it must decide 32 rows
   per centroid for BF16, 48 for FP8), smaller calls go without it.  SOAR_NO_BOUND turns the bound
   off (every row goes through the sweep); SOAR_BOUND_ALWAYS builds the table at any size.  Both
   bits: SOAR_E_INVAL. */
#define SOAR_NO_BOUND 8u
#define SOAR_BOUND_ALWAYS 16u

/* Options of soar_assign.  Set struct_size = sizeof(soar_assign_opts). */
typedef struct soar_assign_opts {
  uint32_t struct_size;
  float lambda;             /* >= 0 and finite; the weight of the parallelism penalty           */
  int32_t precision;        /* a soar_precision                                                  */
  int32_t topk;             /* BF16/FP8: candidates re-scored in FP32 per row (0 = 8, max 16)    */
  float near_tie_rel;       /* relative gap under which FP32 re-scores are decided in FP64
                               (0 = 1e-5)                                                        */
  uint32_t flags;           /* SOAR_ASYNC | SOAR_SPILL_GROUPED or SOAR_SPILL_DIRECT             */
} soar_assign_opts;

/* Optional statistics of one blocking call (host struct).  Set struct_size. */
typedef struct soar_stats {
  uint32_t struct_size;
  float device_ms;          /* device time of the whole call (HIP events on the stream)          */
  float assign_kernel_ms;   /* the sweeps and the grouping by primary: phase_ms[1] + [3] + [4]   */
  int64_t rows_full_scan;   /* rows whose candidate set could not be proven complete and were
                               re-done by an exact scan over all K                               */
  int64_t rows_fp64;        /* rows whose decision was taken in FP64 (near-ties)                 */
  double mfma_flops;        /* algorithmic work 4 n K d: X C^T and R C^T, each once              */
  float phase_ms[6];        /* [0] codebook and row preparation (norms, packing, quantization;
                               BF16/FP8 with the spill bound: its table of nearest centroids),
                               [1] primary sweep, [2] primary re-score (BF16/FP8), [3] grouping
                               of the rows by primary, [4] spill sweep, [5] spill re-score
                               (BF16/FP8) or exact full scan (FP32).  An FP32 direct-form call
                               runs both sweeps in one pass, reported under [1].                */
  int64_t rows_bounded;     /* BF16/FP8: rows whose spill the spill bound confined to the topk
                               centroids nearest their primary (no spill sweep; see
                               SOAR_NO_BOUND); filled when struct_size covers it (a struct that
                               ends at phase_ms is accepted)                                     */
} soar_stats;

/* Bytes of device workspace soar_assign needs for these sizes and options. */
soar_status soar_assign_workspace_size(int64_t n, int32_t d, int32_t K,
                                       const soar_assign_opts* opts, size_t* bytes);

/*
 * SOAR assignment of n points (Section 3.5's indexing step: primary, residual, spill).
 *   X [n x d], C [K x d]          inputs (device, float32, 16-byte aligned)
 *   primary [n], spill [n]        outputs (device int32): pi and pi'
 *   primary_dist [n]              nullable output: ||x - C_pi||^2
 *   spill_loss [n]                nullable output: the SOAR loss at pi'
 *   workspace / ws_bytes          device scratch of at least soar_assign_workspace_size bytes
 *   stats                         nullable host struct, filled by blocking calls
 * Requires n >= 1, d >= 1, K >= 2.  FP32: d <= 1024 (rows above 256 are processed in chunks of
 * 128 dimensions); BF16: d <= 1024; FP8: d <= 1024.  Larger d: SOAR_E_UNSUPPORTED.
 * Accuracy (FP32): indices are exact arg-mins up to near-ties of 1e-6 relative; reported values
 * are within 1e-5 relative of the exact value at the reported index.
 */
soar_status soar_assign(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                        const soar_assign_opts* opts, int32_t* primary, int32_t* spill,
                        float* primary_dist, float* spill_loss, void* workspace, size_t ws_bytes,
                        void* stream, soar_stats* stats);

/*
 * soar_assign without a workspace, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments, options,
 * results and errors as soar_assign, minus workspace and stats; it allocates nothing.  Its
 * workspace is a fixed device array of soar_assign_noalloc_limit() bytes (64 MiB) that each GPU
 * holds from the library's load until the process ends.
 *  - A call whose soar_assign_workspace_size exceeds that limit returns SOAR_E_NOMEM before any
 *    launch (for BF16 at d=96 and K=40,000 that is about 100,000 rows).
 *  - Every call on one GPU shares that GPU's array and leaves its contents behind (each call
 *    initializes what it reads).  Calls that overlap on one GPU (two streams, two host threads,
 *    an enqueue-only call still running) race on it: the caller must order them.
 *  - SOAR_ASYNC works as for soar_assign; the status record then lives in the shared array.
 */
soar_status soar_assign_noalloc(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                                const soar_assign_opts* opts, int32_t* primary, int32_t* spill,
                                float* primary_dist, float* spill_loss, void* stream);

/* Bytes of the fixed device workspace of soar_assign_noalloc. */
size_t soar_assign_noalloc_limit(void);

/*
 * Where a BF16/FP8 soar_assign leaves its re-scored candidates in its workspace (diagnostics):
 * byte offsets from the workspace start of two row-major int32 [n x topk] arrays, the candidates
 * of the primary and of the spill (-1: an empty place), for the same n, d, K and opts.  They hold
 * the last such call's candidates until the workspace is reused.  bound_key_off (nullable): an
 * int32 [n] array that a call which used the spill bound (SOAR_NO_BOUND) leaves there: -1 for
 * the rows the bound decided (and rows without a primary), else the row's primary.  FP32:
 * SOAR_E_UNSUPPORTED (its candidate sets are proven complete instead, and rows that are not go
 * to an exact full scan).
 */
soar_status soar_assign_candidates(int64_t n, int32_t d, int32_t K, const soar_assign_opts* opts,
                                   size_t* primary_off, size_t* spill_off, int32_t* topk,
                                   size_t* bound_key_off);

/* ---- Further spilled assignments (Section 3.5.1) ---- */

/* Bytes of device workspace soar_spill_further needs for these sizes. */
soar_status soar_spill_further_workspace_size(int64_t n, int32_t d, int32_t K, int32_t m,
                                              size_t* bytes);

/*
 * One more spilled assignment per row given its m earlier ones (Section 3.5.1 generalises the
 * spill to further assignments without giving the loss; this library takes one Theorem 3.1
 * penalty per earlier residual):
 *   next_i = argmin over j not in prior_i of
 *            ||x_i - c_j||^2 + lambda * sum_k <r_k, x_i - c_j>^2 / ||r_k||^2,
 *   r_k = x_i - C[prior_i,k]  (a term with r_k = 0 is dropped; ties go to the lowest index).
 * With m = 1 and the primary as prior this is soar_assign's FP32 spill; soar_assign followed by
 * calls with m = 2, 3 gives up to four assignments per point.
 *   X [n x d], C [K x d]    device float32 (4-byte aligned)
 *   prior [n x m]           device int32, row-major; each row's entries distinct and in [0, K)
 *                           (otherwise SOAR_E_INVAL, returned before any result is written)
 *   m                       1..3; K > m
 *   next [n]                device int32 output; next_loss [n] nullable device float32 output
 *   workspace / ws_bytes    at least soar_spill_further_workspace_size bytes, 256-byte aligned
 *   stats                   nullable; device_ms, rows_full_scan, rows_fp64 and mfma_flops
 *                           (the algorithmic 2 n K d (1 + m)) are filled
 * FP32 throughout, d <= 1024 (rows above 128 dimensions are processed in chunks of 64).  Accuracy
 * as soar_assign's FP32 form: indices exact up to near-ties, reported losses within 1e-5
 * relative.  Blocking: the call synchronises the stream (twice: after checking prior, at the end).
 */
soar_status soar_spill_further(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                               const int32_t* prior, int32_t m, float lambda, float near_tie_rel,
                               int32_t* next, float* next_loss, void* workspace, size_t ws_bytes,
                               void* stream, soar_stats* stats);

/* ---- PQ codes of the residuals (Section 3.5, implementation considerations) ---- */

/*
 * For every point i and each of its m assignments a = assign[i m + j], the residual x_i - C[a]
 * is cut into M = d / s subspaces of s dimensions and each piece is coded by the index of the
 * nearest of the 16 codewords P[sub][0..15] of its subspace (squared Euclidean distance formed in
 * FP64 from the FP32 inputs; ties to the lowest index).  A spilled copy of a point thus carries
 * the code of its own residual; these codes (d / (2 s) bytes) plus a 4-byte id per copy are what
 * spilling adds to a VQ-PQ index.
 *   X [n x d], C [K x d]      device float32
 *   assign [n x m]            device int32, row-major, values in [0, K)
 *   P [M x 16 x s]            device float32 PQ codebook
 *   codes [n x m x M/2]       device uint8 output: subspace 2 j in the low nibble of byte j,
 *                             2 j + 1 in the high nibble
 *   workspace                 >= 256 bytes of device memory
 * Requires 1 <= s <= 16, d % (2 s) == 0, d <= 1024 (larger: SOAR_E_UNSUPPORTED).  An assignment
 * outside [0, K): SOAR_E_INVAL after the call (its code is written as zeros).  Blocking.
 */
soar_status soar_pq_encode(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                           const int32_t* assign, int32_t m, const float* P, int32_t s,
                           uint8_t* codes, void* workspace, size_t ws_bytes, void* stream);

/* Bytes of workspace for soar_kmeanspp / soar_lloyd_update / soar_train_codebook. */
soar_status soar_train_workspace_size(int64_t n, int32_t d, int32_t K, size_t* bytes);

/*
 * k-means++ seeding.  Round 0 takes row floor(w * n / 2^32); round m >= 1 takes the smallest row i
 * whose prefix sum of D^2 exceeds u_m * sum(D^2), where D is the distance to the nearest centre
 * chosen so far and u_m = (w >> 8) * 2^-24.  w is the first word of Philox4x32-10 with counter
 * (m, 0, 0, 0) and key (seed mod 2^32, seed >> 32).  If sum(D^2) = 0 the lowest-index row not yet
 * chosen is taken.
 *   C_out [K x d] (device), rows_out [K] (device, nullable): the chosen rows.
 * Requires 1 <= K <= n and d <= 1024 (larger d: SOAR_E_UNSUPPORTED).
 */
soar_status soar_kmeanspp(const float* X, int64_t n, int32_t d, int32_t K, uint64_t seed,
                          float* C_out, int32_t* rows_out, void* workspace, size_t ws_bytes,
                          void* stream);

/*
 * One Lloyd update: C_out[j] = mean of the rows with labels == j; a cluster with no rows keeps
 * C_prev[j].  The per-cluster sums are exact (64-bit fixed point), so the result does not depend
 * on the order rows are visited in.  counts [K] (device, nullable) receives the cluster sizes.
 * C_out may equal C_prev.  labels must lie in [0, K).
 */
soar_status soar_lloyd_update(const float* X, int64_t n, int32_t d, const int32_t* labels,
                              int32_t K, const float* C_prev, float* C_out, int32_t* counts,
                              void* workspace, size_t ws_bytes, void* stream);

/*
 * Codebook training: k-means++ (skipped when C_init is given), then exactly `iters` Lloyd
 * iterations, each an exact nearest-centroid assignment followed by soar_lloyd_update.
 *   C_init [K x d]        nullable device input (resume from a saved codebook)
 *   C_out [K x d]         device output: the codebook after the last update
 *   labels [n]            nullable device output: nearest centroid of every row in C_out
 *   inertia [iters + 1]   nullable HOST output: sum of squared distances before each update and,
 *                         last, against C_out
 * Requires 1 <= K <= n (K >= 2 when the codebook is meant for soar_assign), iters >= 0, d <= 1024.
 */
soar_status soar_train_codebook(const float* X, int64_t n, int32_t d, int32_t K, int32_t iters,
                                uint64_t seed, const float* C_init, float* C_out, int32_t* labels,
                                double* inertia, void* workspace, size_t ws_bytes, void* stream);

/* ---- Query-side probing over the inverted lists (Section 2.2 search; spilled copies, Section
   3.5, count once) ---- */

/* Bytes of workspace for soar_lists_build. */
soar_status soar_lists_workspace_size(int64_t n, int32_t K, size_t* bytes);

/*
 * Inverted lists in CSR form from assignment arrays: partition j lists ids[offsets[j] ..
 * offsets[j+1]) (device int64 offsets [K + 1], device int32 ids [n] or [2 n] with spill), every
 * point under primary[i] and, if spill is non-null, also under spill[i].  The order of ids
 * inside a list is not specified.  Indices outside [0, K): SOAR_E_INVAL (after the lists were
 * written).  Blocking.
 */
soar_status soar_lists_build(const int32_t* primary, const int32_t* spill, int64_t n, int32_t K,
                             int64_t* offsets, int32_t* ids, void* workspace, size_t ws_bytes,
                             void* stream);

/* Bytes of workspace for soar_search. */
soar_status soar_search_workspace_size(int64_t nq, int32_t d, int32_t K, size_t* bytes);

/*
 * VQ search of nq queries Q [nq x d] (device FP32): per query the t partitions with the largest
 * <q, c_j> (MIPS over the codebook C [K x d]; equal scores to the lower index) are probed, every
 * point in their lists (offsets, ids from soar_lists_build over the dataset X [n x d]) is scored
 * exactly by <q, x> and the k best distinct points (higher score, then lower id) are returned:
 *   out_ids [nq x k] (device int32; -1 where fewer than k points were reached)
 *   out_scores [nq x k] (device FP64: FP32 inputs, FP64 accumulation; -inf where empty)
 *   searched [nq] (device int64, nullable): points scored, i.e. the summed sizes of the probed
 *   lists, a spilled point counted once per list it was reached through.
 * Requires 1 <= k <= 16, t >= 1 (t > K probes every partition), finite inputs.  Blocking.
 */
soar_status soar_search(const float* Q, int64_t nq, int32_t d, const float* C, int32_t K,
                        const float* X, int64_t n, const int64_t* offsets, const int32_t* ids,
                        int32_t t, int32_t k, int32_t* out_ids, double* out_scores,
                        int64_t* searched, void* workspace, size_t ws_bytes, void* stream);

/* ---- Two-level VQ probing (App. A.4.1: the partition centres vector-quantized again) ---- */

/* Bytes of workspace for soar_search_two_level. */
soar_status soar_search_two_level_workspace_size(int64_t nq, int32_t d, int32_t K, int32_t K2,
                                                 size_t* bytes);

/*
 * soar_search with a two-level probe.  The K partition centres C are themselves quantized by an
 * upper codebook U [K2 x d] (device FP32); upper_offsets [K2 + 1] / upper_ids list the partitions
 * under each upper centroid (soar_lists_build over the partitions' upper assignment, n = K).
 * Per query the t2 upper centroids with the largest <q, u> are probed, every partition listed
 * under them is scored by <q, c_p>, and the t best of those (equal scores to the lower index)
 * are searched as soar_search does: their lists' points scored exactly, the k best distinct
 * points returned.  All inner products are FP64 sums of the FP32 products in dimension order, so
 * with t2 = K2 the probed partitions, and the result, are soar_search's.  A query whose probed
 * upper lists hold fewer than t partitions searches those.  out_ids / out_scores / searched as
 * for soar_search.  Requires 1 <= k <= 16, t >= 1, t2 >= 1, d <= 1024 (larger:
 * SOAR_E_UNSUPPORTED), finite inputs.  Blocking.
 */
soar_status soar_search_two_level(const float* Q, int64_t nq, int32_t d, const float* U,
                                  int32_t K2, const int64_t* upper_offsets,
                                  const int32_t* upper_ids, int32_t t2, const float* C, int32_t K,
                                  const float* X, int64_t n, const int64_t* offsets,
                                  const int32_t* ids, int32_t t, int32_t k, int32_t* out_ids,
                                  double* out_scores, int64_t* searched, void* workspace,
                                  size_t ws_bytes, void* stream);

/* ---- Lists with PQ-coded copies and their search (Section 2.2 search, Section 3.5 layout) ---- */

/*
 * The PQ codes of the list entries, in list order: entry pos of list p (offsets, ids from
 * soar_lists_build) is a copy of point i = ids[pos] in partition p, made by the first
 * assignment j with assign[i m + j] == p, and takes that copy's code codes[(i m + j) code_bytes
 * ..] (from soar_pq_encode with the same assign [n x m]).  list_codes [offsets[K] x code_bytes]
 * device uint8 output.  *max_list (host, nullable) receives the longest list's length.  An
 * entry whose point has no assignment to its list, or an id outside [0, n): SOAR_E_INVAL after
 * the call (its code is written as zeros).  workspace >= 256 bytes of device memory.  Blocking.
 */
soar_status soar_lists_codes(const int64_t* offsets, const int32_t* ids, int32_t K, int64_t n,
                             const int32_t* assign, int32_t m, const uint8_t* codes,
                             int32_t code_bytes, uint8_t* list_codes, int64_t* max_list,
                             void* workspace, size_t ws_bytes, void* stream);

/* The most list entries any t of the lists hold: the sum of the t longest lists' lengths
 * (offsets [K + 1] on the device, read back).  *bound on the host.  Blocking. */
soar_status soar_lists_probe_bound(const int64_t* offsets, int32_t K, int32_t t, int64_t* bound,
                                   void* stream);

/* Bytes of workspace for soar_search_pq when a query's t probed lists hold at most max_probed
 * entries (soar_lists_probe_bound; SOAR_E_UNSUPPORTED from 2^31). */
soar_status soar_search_pq_workspace_size(int64_t nq, int32_t d, int32_t K, int32_t t,
                                          int64_t max_probed, size_t* bytes);

/*
 * VQ-PQ search of nq queries Q [nq x d] over lists whose copies carry PQ codes of their own
 * residuals.  Per query:
 *   1. the t partitions with the largest <q, c_p> (FP64 products of the FP32 inputs summed in
 *      dimension order; equal scores to the lower index) are probed;
 *   2. every copy listed there is estimated from its code: <q, c_p> + sum over subspaces m, in
 *      order, of LUT[m][code_m] with LUT[m][c] = <q_m, P[m][c]> (FP64, the s dimensions in
 *      order), P [M x 16 x s] the PQ codebook, M = d / s;
 *   3. a point reached through several copies keeps its largest estimate, and the R points with
 *      the largest estimates (equal estimates: lower id first) are scored exactly by <q, x>
 *      (FP64, dimension order) over X [n x d];
 *   4. the k best of them (higher score, then lower id) are returned.
 *   offsets, ids           lists from soar_lists_build; list_codes [offsets[K] x M/2] from
 *                          soar_lists_codes (4-byte aligned)
 *   out_ids [nq x k]       device int32 (-1 where fewer than k points were reached)
 *   out_scores [nq x k]    device FP64 exact scores (-inf there)
 *   scored [nq]            device int64, nullable: copies estimated (the probed lists' sizes)
 * Every step is the same arithmetic in the same order as its definition above, so the result is
 * reproducible bit for bit.  The lists hold each point at most twice (as soar_lists_build makes
 * them): only the 2 R best copies of a query can then matter, and the call keeps a superset of
 * them before selecting.  Requires 1 <= k <= 16, k <= R <= 4096, t >= 1, d % (2 s) == 0,
 * M <= 512 (larger: SOAR_E_UNSUPPORTED), finite inputs, and t lists holding at most max_probed
 * entries, which the call checks (else SOAR_E_INVAL; the workspace is sized for max_probed).
 * Blocking.
 */
soar_status soar_search_pq(const float* Q, int64_t nq, int32_t d, const float* C, int32_t K,
                           const float* X, int64_t n, const int64_t* offsets, const int32_t* ids,
                           const uint8_t* list_codes, const float* P, int32_t s, int32_t t,
                           int32_t R, int32_t k, int64_t max_probed, int32_t* out_ids,
                           double* out_scores, int64_t* scored, void* workspace, size_t ws_bytes,
                           void* stream);

/* ---- Serving: a resident codebook plus inverted lists (Section 2.2) fed by insert requests ---- */

typedef struct soar_index soar_index;

/*
 * Bytes of arena an index needs for these sizes and a list capacity of list_capacity_ids ids in
 * total (two per inserted point); the rest of a larger arena also holds list chunks.
 */
soar_status soar_index_arena_size(int32_t K, int32_t d, int32_t precision, int32_t max_step_rows,
                                  int64_t list_capacity_ids, size_t* bytes);

/*
 * Create an index over codebook C [K x d] (device, copied into the arena) with spill weight
 * lambda.  The index places the codebook, its per-step buffers and the partition lists inside
 * the caller's device arena (arena_bytes) and never allocates device memory of its own.
 * max_step_rows bounds the rows assigned in one device step.  With K >= 8192 every step's sweeps
 * run in S = min(8, K / 4096) codebook splits (workgroups over 1/S of the centroids each), whose
 * candidates (BF16/FP8) or exact answers (FP32, d <= 256) are joined; S is fixed per index, so a
 * point's assignment does not depend on the step it lands in, and FP32 answers equal
 * soar_assign's.
 */
soar_status soar_index_create(const float* C, int32_t K, int32_t d, float lambda,
                              int32_t precision, void* arena, size_t arena_bytes,
                              int32_t max_step_rows, soar_index** out);

/*
 * Queue n vectors (HOST pointer X_host [n x d], copied before the call returns) with ids
 * first_id .. first_id + n - 1.  Non-blocking: returns a ticket for soar_wait.  Continuous
 * batching: queued rows go into the next free step slot as soon as there is one, shared out
 * max-min fairly between the queued requests (a small request behind a large one joins the next
 * step), and steps in different slots overlap on the GPU.  A step is admitted when the list
 * arena can take its worst-case growth; a request that can never fit gets SOAR_E_NOMEM.
 */
soar_status soar_insert(soar_index* index, const float* X_host, int64_t n, int64_t first_id,
                        uint64_t* ticket);

/* Wait for a ticket; writes its primary and spill indices to HOST arrays of n entries each.
   It returns as soon as the last of the request's rows has been assigned; the ids then enter the
   lists in step order (soar_index_list waits for every append in flight).  timeout_s < 0 waits
   without limit; on SOAR_E_TIMEOUT the ticket stays valid.  A ticket is consumed by the call that
   returns its result. */
soar_status soar_wait(soar_index* index, uint64_t ticket, int32_t* primary_host,
                      int32_t* spill_host, double timeout_s);

/* Copy partition `part`'s member ids to a HOST array (at most cap); *len gets the full length.
   The ids of a list are in no particular order.  Steps in flight finish first. */
soar_status soar_index_list(soar_index* index, int32_t part, int64_t* ids_host, int64_t cap,
                            int64_t* len);

/* Counters of an index (host struct; set struct_size). */
typedef struct soar_index_stats {
  uint32_t struct_size;
  int64_t requests;             /* insert requests accepted                                     */
  int64_t steps;                /* device steps launched                                        */
  int64_t rows;                 /* rows assigned by those steps                                 */
  int64_t max_steps_in_flight;  /* most steps on the device at once                             */
  int64_t chunks_used;          /* list chunks in use (after the last finished append)          */
  int64_t chunks_total;         /* list chunks the arena holds                                  */
} soar_index_stats;
soar_status soar_index_get_stats(soar_index* index, soar_index_stats* stats);

/* Arena bytes one list chunk (64 ids and a link) takes. */
size_t soar_index_chunk_bytes(void);

/* Drain queued and in-flight work, then release the index's host objects (never the arena). */
void soar_index_destroy(soar_index* index);

const char* soar_status_string(soar_status status);

#ifdef __cplusplus
}
#endif

#endif /* SOAR_H */
