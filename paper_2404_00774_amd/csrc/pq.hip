// Product-quantized residual codes (Section 3.5, implementation considerations): for every point
// and each of its assignments a, the residual x - c_a is cut into M = d / s subspaces of s
// dimensions, and each piece takes the index of the nearest of 16 codewords of its subspace.  With
// SOAR a point's spilled copy carries the code of its own residual; these codes, with a 4-byte id
// per copy, are what spilling duplicates.  Codes are packed two per byte: subspace 2 j in the low
// nibble of byte j, 2 j + 1 in the high nibble.
//
// One thread per (point, assignment, subspace), in a grid-stride loop over a grid sized to the
// chip (each workgroup copies the PQ codebook into LDS once): a thread forms its s residual
// entries from x and the row of c_a (consecutive threads read consecutive pieces, so the loads
// coalesce), takes the squared distance to each of the 16 codewords in FP64, and the even and odd
// subspace of a byte meet through one lane swap.  The codebook sits in LDS as [16][s][M], so the
// threads of a wave read consecutive words.  The distances are formed in FP64 from the FP32
// inputs (the differences x - c are exact there for inputs within 2^29 of each other in
// magnitude), so the codes are the definition's up to FP64 rounding; ties go to the lowest
// codeword index.  The work per thread is 16 s FP64 fma and as many subtractions: for s = 2 and
// d = 96 about 3,000 FP64 operations per (point, assignment) against 2 d = 192 bytes of x and c,
// so the kernel is bound by FP64 issue, not by memory.
#include <algorithm>

#include "../../include/soar.h"
#include "common.h"

namespace soar {
namespace {

constexpr int kPQCentres = 16;
constexpr int kPQMaxS = 16;
constexpr int kPQMaxD = 1024;         // 16 d floats of codebook in 64 KB of LDS

// S: the subspace width at compile time (1, 2, 4, 8, 16), or 0 for any width up to 16.
// T: the codebook's type in LDS: double where 16 d of them fit 64 KB (d <= 512; no conversion
// per use), else float.
template <int S, typename T>
__global__ __launch_bounds__(256) void pq_encode_kernel(
    const float* __restrict__ X, int64_t n, int d, const float* __restrict__ C, int K,
    const int32_t* __restrict__ assign, int m, const float* __restrict__ P, int s_rt,
    uint8_t* __restrict__ codes, unsigned* bad) {
  extern __shared__ __attribute__((aligned(16))) char sP_raw[];
  T* sP = reinterpret_cast<T*>(sP_raw);  // [16][s][M]
  const int s = S ? S : s_rt;
  const int M = d / s;
  for (int i = threadIdx.x; i < kPQCentres * d; i += blockDim.x) {
    const int sub = i / (kPQCentres * s), rem = i % (kPQCentres * s);   // P is [M][16][s]
    sP[rem * M + sub] = (T)P[i];
  }
  __syncthreads();
  const int64_t items = n * m * M;       // M is even, so each byte's two subspaces are lanes
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;   // g and g ^ 1 of one wave
  // every lane of a wave runs the same number of rounds (the swap needs its partner)
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wave0 = first & ~(int64_t)63;
  for (int64_t g0 = wave0; g0 < items; g0 += stride) {
    const int64_t g = g0 + (first - wave0);
    const bool live = g < items;
    const int64_t pair = live ? g / M : 0;
    const int sub = live ? (int)(g - pair * M) : 0;
    const int a = live ? assign[pair] : 0;
    const bool ok = live && a >= 0 && a < K;
    int bk = 0;
    if (ok) {
      const float* x = X + (pair / m) * (int64_t)d + sub * s;
      const float* c = C + (int64_t)a * d + sub * s;
      double best = __builtin_inf();
      if constexpr (S > 0) {
        double r[S];
#pragma unroll
        for (int t = 0; t < S; ++t) r[t] = (double)x[t] - (double)c[t];
#pragma unroll 4
        for (int k = 0; k < kPQCentres; ++k) {
          double dd = 0.0;
#pragma unroll
          for (int t = 0; t < S; ++t) {
            const double e = r[t] - (double)sP[(k * S + t) * M + sub];
            dd = fma(e, e, dd);
          }
          if (dd < best) { best = dd; bk = k; }
        }
      } else {
        for (int k = 0; k < kPQCentres; ++k) {
          double dd = 0.0;
          for (int t = 0; t < s; ++t) {
            const double e = ((double)x[t] - (double)c[t]) - (double)sP[(k * s + t) * M + sub];
            dd = fma(e, e, dd);
          }
          if (dd < best) { best = dd; bk = k; }
        }
      }
    } else if (live && (sub & 1) == 0) {
      atomicOr(bad, 1u);
    }
    const int hi = __shfl_xor(bk, 1);
    if (live && (sub & 1) == 0) codes[pair * (M / 2) + sub / 2] = (uint8_t)(bk | (hi << 4));
  }
}

__global__ void zero_word_kernel(unsigned* p) { *p = 0u; }

template <int S>
void launch_pq(const float* X, int64_t n, int d, const float* C, int K, const int32_t* assign,
               int m, const float* P, int s, uint8_t* codes, unsigned* bad, hipStream_t st) {
  const int64_t items = n * m * (d / s);
  const int64_t blocks = std::min<int64_t>((items + 255) / 256, 8 * 256);
  if ((size_t)kPQCentres * d * sizeof(double) <= 65536)
    hipLaunchKernelGGL((pq_encode_kernel<S, double>), dim3((unsigned)blocks), dim3(256),
                       (size_t)kPQCentres * d * sizeof(double), st, X, n, d, C, K, assign, m, P,
                       s, codes, bad);
  else
    hipLaunchKernelGGL((pq_encode_kernel<S, float>), dim3((unsigned)blocks), dim3(256),
                       (size_t)kPQCentres * d * sizeof(float), st, X, n, d, C, K, assign, m, P,
                       s, codes, bad);
}

}  // namespace
}  // namespace soar

extern "C" {

soar_status soar_pq_encode(const float* X, int64_t n, int32_t d, const float* C, int32_t K,
                           const int32_t* assign, int32_t m, const float* P, int32_t s,
                           uint8_t* codes, void* workspace, size_t ws_bytes, void* stream) {
  if (!X || !C || !assign || !P || !codes || !workspace || ws_bytes < 256 || n < 1 || d < 1 ||
      K < 1 || m < 1 || s < 1 || s > soar::kPQMaxS || d % (2 * s) != 0 ||
      n * m > (int64_t)INT32_MAX * 16)
    return SOAR_E_INVAL;
  if (d > soar::kPQMaxD) return SOAR_E_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned* bad = static_cast<unsigned*>(workspace);
  hipLaunchKernelGGL(soar::zero_word_kernel, dim3(1), dim3(1), 0, st, bad);
  switch (s) {
    case 1: soar::launch_pq<1>(X, n, d, C, K, assign, m, P, s, codes, bad, st); break;
    case 2: soar::launch_pq<2>(X, n, d, C, K, assign, m, P, s, codes, bad, st); break;
    case 4: soar::launch_pq<4>(X, n, d, C, K, assign, m, P, s, codes, bad, st); break;
    case 8: soar::launch_pq<8>(X, n, d, C, K, assign, m, P, s, codes, bad, st); break;
    case 16: soar::launch_pq<16>(X, n, d, C, K, assign, m, P, s, codes, bad, st); break;
    default: soar::launch_pq<0>(X, n, d, C, K, assign, m, P, s, codes, bad, st); break;
  }
  unsigned hbad = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SOAR_E_DEVICE;
  return hbad ? SOAR_E_INVAL : SOAR_OK;
}

}  // extern "C"
