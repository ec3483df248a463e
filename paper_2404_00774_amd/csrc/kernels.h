// Internal interface between the C-ABI layer and the HIP kernels (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace soar {

struct AssignParams {
  const float* X;
  int64_t n;
  int d;
  const float* C;
  int K;
  const float* cnorm;   // [K] ||c_j||^2
  unsigned* counters;   // CNT_* words
  float lam;
  float tie_rel;        // relative gap under which FP32 re-scores are re-decided in FP64
  float band_p;         // primary screen: band = band_p * (||x|| + max||c||)^2
  float band_s;         // spill screen:   band = band_s * (||x|| + max||c||)^2
  int32_t* primary;
  int32_t* spill;
  float* pdist;
  float* sloss;
  int32_t* full_rows;   // [n] rows handed to the exact full scan
};

int fp32_padded_dim(int d);
hipError_t launch_prep_codebook(const float* C, int K, int d, float* cnorm, unsigned* counters,
                                hipStream_t st);
// ev_begin / ev_end (nullable) are recorded around the main assignment kernel alone.
hipError_t launch_assign_fp32(const AssignParams& P, bool spill, bool vec, hipStream_t st,
                              hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);

}  // namespace soar
