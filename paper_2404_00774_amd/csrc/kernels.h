// Internal interface between the C-ABI layer and the HIP kernels (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace soar {

struct GroupLayout;

struct AssignParams {
  const float* X;
  int64_t n;
  int d;
  const float* C;
  int K;
  const char* Crec;     // packed tile records of C (launch_pack_fp32)
  const float* cnorm;   // [K] ||c_j||^2
  unsigned* counters;   // CNT_* words
  float lam;
  float tie_rel;        // relative gap under which FP32 re-scores are re-decided in FP64
  // Screens: twice the rounding-error bound of centroid j's expanded value is
  //   primary band_p * (||x|| + ||c_j||)^2,   spill band_s * (||x|| + ||c_j||)^2
  float band_p;
  float band_s;
  // Gram form of the spill screen (G non-null): <r, c_j> = <x, c_j> - G[pi][j]; the spill band
  // gains (band_g1 P / ||r|| + band_g2 P^2 / ||r||^2) (||x|| + ||c_j||)^2, P = ||x|| + ||c_pi||
  const float* G = nullptr;   // [K x K] C C^T, or null
  float band_g1 = 0.f, band_g2 = 0.f;
  // grouped form of the spill sweep (launch_assign_fp32 with a GroupLayout): rows by primary
  const int32_t* perm = nullptr;
  const int4* stripes = nullptr;
  const int32_t* nstripes = nullptr;
  int32_t* primary;
  int32_t* spill;
  float* pdist;
  float* sloss;
  int32_t* full_rows;   // [n] rows handed to the exact full scan
  const int64_t* live_n = nullptr;   // device row count <= n (serving steps), or null
  // further spilled assignments: [n x np] earlier assignments per row (row-major)
  const int32_t* prior = nullptr;
  // codebook splits (launch_assign_fp32_split): split s of gridDim.y writes its split-relative
  // arg-min and value to split_idx / split_val[s * n + row] and lists its unproven rows in
  // split_rows[s * n + k], counted by split_cnt[s]; Crec_all is the whole codebook's records
  const char* Crec_all = nullptr;
  int32_t* split_idx = nullptr;
  float* split_val = nullptr;
  int32_t* split_rows = nullptr;
  unsigned* split_cnt = nullptr;
};

// Padded row length of the FP32 path (-1: unsupported); rows above 256 are processed in chunks.
int fp32_padded_dim(int d);
// Bytes of the packed codebook records read by the FP32 sweeps, and the kernel that writes them
// (after launch_prep_codebook, whose norms it copies).
size_t fp32_codebook_bytes(int d, int K);
hipError_t launch_pack_fp32(const float* C, int K, int d, const float* cnorm, void* rec,
                            hipStream_t st);
// Screening bands and near-tie threshold of the FP32 path (defined with the C ABI).
float band_coef_primary(int d);
float band_coef_spill(int d, float lam);
float tie_threshold(int d, float lam, float near_tie_rel);
// Largest K for which the spill sweep uses the Gram form (G = C C^T in the workspace).
constexpr int kGramMaxK = 4096;
bool fp32_uses_gram(int d, int K);
float band_coef_gram1(int d, float lam);
float band_coef_gram2(int d, float lam);
// G = C C^T (K x K, FP32, any summation order).
hipError_t launch_gram(const float* C, int K, int d, float* G, hipStream_t st);
// Clears all counters, then ||c_j||^2, max ||c||^2 and the finiteness flag of the codebook.
hipError_t launch_prep_codebook(const float* C, int K, int d, float* cnorm, unsigned* counters,
                                hipStream_t st);
// Clears the per-assignment counters only (the codebook's maximum norm is kept).
hipError_t launch_reset_step_counters(unsigned* counters, hipStream_t st);
// Enqueue-only calls keep their non-finite flag in the counters' status record; a blocking call
// reads and clears it.
hipError_t launch_async_note(unsigned* counters, hipStream_t st);
hipError_t launch_async_clear(unsigned* counters, hipStream_t st);
// ev (nullable, 4 events) is recorded after the primary pass [0], after the primary phase's
// tail [1] (same point here), after the grouping [2] and after the spill pass [3], before the
// exact full scan; a single fused pass records all four after itself.  With `grouped` (rows of
// up to 256 dimensions only) the spill runs in its grouped form: primary pass, grouping of the
// rows by primary into G, grouped spill pass.
hipError_t launch_assign_fp32(const AssignParams& P, bool spill, bool vec, hipStream_t st,
                              hipEvent_t* ev = nullptr, const GroupLayout* grouped = nullptr);

// FP32 SOAR assignment with the codebook split S ways (serving steps of few rows: S workgroups per
// row block, each over 1/S of the tiles), rows of up to 256 dimensions: primary pass, exact full
// scan of the splits' unproven rows, join of the splits (FP64 on near-ties across splits), then
// the same for the spill given the joined primary.  P.split_* must hold S * n entries (split_cnt
// S words).  Same results as launch_assign_fp32.
hipError_t launch_assign_fp32_split(const AssignParams& P, int S, bool vec, hipStream_t st);
bool fp32_split_supported(int d);

// ---- further spilled assignments (the next assignment given np = 1..3 earlier ones) ----
constexpr int kFurtherMaxPrior = 3;
// Counter word set when an earlier assignment is out of range or repeated within its row (one of
// the words every call clears, unused by the other kernels).
constexpr int CNT_BADINPUT = 4;
static_assert(CNT_BADINPUT > CNT_CMAX2 && CNT_BADINPUT < CNT_WORDS, "a per-call counter word");
// Padded row length of the further-assignment sweep (-1: unsupported); rows above 128 go in
// chunks of 64 (the residual rows of every earlier assignment are held beside X).
int fp32_further_padded_dim(int d);
size_t fp32_further_codebook_bytes(int d, int K);
hipError_t launch_pack_fp32_further(const float* C, int K, int d, const float* cnorm, void* rec,
                                    hipStream_t st);
// Sets CNT_BADINPUT when a row's earlier assignments leave [0, K) or repeat.
hipError_t launch_check_priors(const int32_t* prior, int64_t n, int np, int K, unsigned* counters,
                               hipStream_t st);
// Sweep, candidate decision and exact full scan of the rows whose candidates were not proven
// complete; writes P.spill (the next assignment) and P.sloss.
hipError_t launch_further_fp32(const AssignParams& P, int np, hipStream_t st);

// ---- grouping rows by primary (grouped form of the spill sweep) ----
constexpr int GROUP_ROWS = 15;   // data rows per 16-row MFMA stripe; the 16th row is the centroid
struct GroupLayout {
  int32_t* cnt;      // [K]
  int32_t* cursor;   // [K]
  int32_t* off;      // [K + 1]
  int32_t* sbeg;     // [K + 1]
  int32_t* meta;     // [0]: number of stripes
  int32_t* perm;     // [n] row ids grouped by primary
  int4* stripes;     // [group_max_stripes]: {partition, first position in perm, rows, 0}
  size_t bytes;
};
int64_t group_max_stripes(int64_t n, int K);
GroupLayout group_layout(void* ws, int64_t n, int K);   // ws may be null (sizes only)
// Groups the live rows (prim[i] outside [0, K) are left out).  Stream-ordered; no host sync.
hipError_t launch_group_by_primary(const int32_t* prim, int64_t cap, const int64_t* live_n, int K,
                                   const GroupLayout& L, hipStream_t st);
// The grouped form pays when partitions hold several rows on average.
inline bool grouped_spill_pays(int64_t n, int K) { return n >= 8 * (int64_t)K; }

// ---- low-precision (BF16 / FP8-e4m3) path ----
enum LowpFormat : int { LOWP_BF16 = 0, LOWP_FP8 = 1 };

struct LowpParams {
  int64_t n;
  int d;
  int dp;                 // padded row length of the quantized operands (elements)
  int K;
  int topk;               // candidates re-scored per row (<= 16)
  float lam;
  float tie_rel;
  const float* X;         // FP32 originals
  const float* C;
  const void* Xq;         // quantized rows, row stride dp elements
  const void* Cq;         // packed codebook records (launch_lowp_pack_codebook)
  const void* Rq;
  const float* xs;        // FP8: inverse power-of-two row scales of Xq, Cq
  const float* cs;
  const float* cnorm;     // [K] ||c_j||^2 (FP32)
  const float4* rowc;     // [n] residual rows: {inverse scale, <r, x>, lambda / ||r||^2, sigma}
  int32_t* cand;          // [n * topk]
  int32_t* primary;
  int32_t* spill;
  float* pdist;
  float* sloss;
  unsigned* counters;
  float4* rowc_out;       // written by the primary re-score
  void* Rq_out;           // null: the residual rows are not needed (grouped form over X)
  // grouped spill form: rows grouped by primary, the centroid as the 16th row of every stripe
  const int32_t* perm = nullptr;
  const int4* stripes = nullptr;
  const int32_t* nstripes = nullptr;
  const void* Cp = nullptr;      // [K x dp] codebook rows quantized like X (not -2 c)
  const float* cps = nullptr;    // FP8: their inverse row scales
  const int64_t* live_n = nullptr;   // device row count <= n (serving steps), or null
  // codebook split of the direct sweeps (1: none).  With S > 1 each sweep writes, per row and
  // split, topk candidates and their ranking values to cand_split / cand_val ([n][S][topk]), and
  // launch_lowp_merge reduces them to cand before the re-score.  S <= K / 64.
  int ksplit = 1;
  int32_t* cand_split = nullptr;
  float* cand_val = nullptr;
  // spill bound: with radius set, the primary re-score writes every row's bound radius
  // ||r|| + sqrt((1 + lambda) ||x - c_j2||^2) (j2: the nearest other candidate; +inf without a
  // primary) for launch_bound_decide
  float* radius = nullptr;          // [n]
};

int lowp_padded_dim(int fmt, int d);
// codebook = true stores BF16 rows as -2 c (the sweep's accumulators start at ||c||^2).
hipError_t launch_lowp_quantize(int fmt, const float* A, int64_t rows, int d, int dp,
                                bool codebook, void* out, float* inv_scale, unsigned* counters,
                                hipStream_t st, const int64_t* live_n = nullptr);
hipError_t launch_lowp_sweep(int fmt, const LowpParams& P, bool spill, hipStream_t st);
// Spill sweep in grouped form (P.perm, P.stripes, P.nstripes, P.Cp set; rowc from the re-score).
// Where grouped_residual_rows() holds it also reads the residual rows P.Rq, so the primary
// re-score must have written them (P.Rq_out set).
hipError_t launch_lowp_sweep_grouped(int fmt, const LowpParams& P, hipStream_t st);
// The grouped form runs over residual rows when lambda is at least this: the ranking value then
// carries the row constant ||r||^2 / lambda, which must stay within a few powers of two of the
// loss to keep the FP32 epilogue's resolution.
constexpr float kGroupedResidualMinLam = 1.f / 64;
inline bool grouped_residual_rows(int /*fmt*/, float lam) { return lam >= kGroupedResidualMinLam; }
// The sweep reads the codebook from packed per-tile records (see assign_lowp.hip).
size_t lowp_codebook_bytes(int fmt, int d, int K);
hipError_t launch_lowp_pack_codebook(int fmt, const float* C, int K, int d, const float* cnorm,
                                     void* rec, unsigned* counters, hipStream_t st);
hipError_t launch_lowp_rescore(int fmt, const LowpParams& P, bool spill, hipStream_t st);
// Merges the split candidates of a sweep (no-op for P.ksplit <= 1).
hipError_t launch_lowp_merge(const LowpParams& P, hipStream_t st);
// Spill bound (bound.hip).  launch_bound_table, before the sweeps: from the two nearest
// centroids of a sample of rows it estimates on the device how many rows the bound would decide;
// when that pays for the table (2 K^2 d FP32 flop), it builds for every centroid p its M
// (<= kBoundMaxM) nearest other centroids and a lower bound on the distance to the others.
// launch_bound_decide, after the primary re-score (radius): a row whose radius lies below its
// primary's bound takes those M as spill candidates (cand) and -1 as group key (gkey); every
// other row takes its primary (-1 without one).  counters[CNT_BOUNDED] then counts the decided
// rows once the grouping has run (launch_bound_count).  cnorm holds ||c_j||^2.
constexpr int kBoundMaxM = 8;
constexpr int kBoundSample = 256;
struct BoundLayout {
  int32_t* nbr;        // [K x M]
  float* nbr_lb;       // [K]
  int32_t* xrows;      // [kBoundSample] the sample rows
  float* xnorm;        // [kBoundSample] their squared norms
  int32_t* xnear;      // [kBoundSample] their nearest centroids
  float* xd1;          // [kBoundSample] distances to them
  float* xd2;          // [kBoundSample] distances to the second nearest
  int32_t* snbr;       // [kBoundSample x M] table entries of xnear
  float* slb;          // [kBoundSample]
  float* scratch_v;    // per-part lists before their merge
  int32_t* scratch_j;
  int32_t* enable;     // [1] the device's decision to build the table
  size_t bytes;
};
BoundLayout bound_layout(void* ws, int K, int M);
// payoff: rows per centroid the bound must decide to pay for the table; 0 builds it regardless.
hipError_t launch_bound_table(const float* X, int64_t n, const float* C, int K, int d,
                              const float* cnorm, int M, float lam, const BoundLayout& B,
                              int payoff, hipStream_t st);
hipError_t launch_bound_decide(int M, int64_t n, int K, const int32_t* primary,
                               const float* radius, const BoundLayout& B, int32_t* cand,
                               int32_t* gkey, hipStream_t st);
// counters[CNT_BOUNDED] = n - group_off[K]: the rows the grouping left out.
hipError_t launch_bound_count(const int32_t* group_off, int K, int64_t n, unsigned* counters,
                              hipStream_t st);

}  // namespace soar
