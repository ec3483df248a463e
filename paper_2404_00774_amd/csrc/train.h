// Internal interface of the codebook-training kernels (k-means++ and Lloyd updates).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/soar.h"

namespace soar {

soar_status run_assign_fp32(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                            float lam, float near_tie_rel, bool spill, int32_t* primary,
                            int32_t* spill_out, float* pdist, float* sloss, void* ws,
                            hipStream_t st, unsigned* counters_out_host,
                            hipEvent_t* ev = nullptr, uint32_t spill_form = 0);
size_t assign_workspace_bytes(int64_t n, int32_t d, int32_t K);
soar_status run_assign_lowp(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                            float lam, float near_tie_rel, int fmt, int topk, int32_t* primary,
                            int32_t* spill_out, float* pdist, float* sloss, void* ws,
                            hipStream_t st, unsigned* counters_out_host,
                            hipEvent_t* ev = nullptr, uint32_t flags = 0);
// Phase boundaries recorded by run_assign_fp32 / run_assign_lowp when given 7 events:
// [0] start, [1] after the codebook and row preparation, [2] after the primary sweep, [3] after
// the primary re-score, [4] after the grouping by primary, [5] after the spill sweep, [6] end
// (after the spill re-score or exact full scan).  Phases a form does not have are empty.
constexpr int kPhaseEvents = 7;

// Argument checks of soar_assign without the workspace (need: the workspace bytes), and the
// assignment itself on a workspace of at least that size.
soar_status assign_validate(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                            const soar_assign_opts* opts, const int32_t* primary,
                            const int32_t* spill, size_t* need);
// side_stream: the spill bound may run its table on a second stream of the library's (the
// allocation-free entry point asks for none: creating one allocates).
soar_status assign_run(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                       const soar_assign_opts* opts, int32_t* primary, int32_t* spill,
                       float* primary_dist, float* spill_loss, void* workspace, hipStream_t st,
                       soar_stats* stats, bool side_stream = true);
// run_assign_lowp flags bit (beside the public ones): no second stream.
constexpr uint32_t kLowpNoSideStream = 1u << 30;

}  // namespace soar
