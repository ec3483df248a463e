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
                            hipEvent_t ev_kernel_begin = nullptr,
                            hipEvent_t ev_kernel_end = nullptr, uint32_t spill_form = 0);
size_t assign_workspace_bytes(int64_t n, int32_t d, int32_t K);
soar_status run_assign_lowp(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                            float lam, float near_tie_rel, int fmt, int topk, int32_t* primary,
                            int32_t* spill_out, float* pdist, float* sloss, void* ws,
                            hipStream_t st, unsigned* counters_out_host, hipEvent_t* ev,
                            uint32_t spill_form = 0);

}  // namespace soar
