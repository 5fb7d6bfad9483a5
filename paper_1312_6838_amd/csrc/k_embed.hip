// Outputs built on the embedding W = Q^T A (Section 3, Eq. CSS_LowDim) that
// the streaming passes write row by row.
#include "gcss_device.h"

namespace gcss {

// Q-less R factor (Section 6): R[s][j] = W[s][idx[j]] on and above the
// diagonal, 0 below it; a pick outside [0, n) gives a NaN column.  One
// thread per entry of R, rows of R over blockIdx.y.
__global__ __launch_bounds__(256) void k_qless_r(const float *__restrict__ w, int64_t n,
                                                 int64_t ldw, const int64_t *__restrict__ idx,
                                                 int k, float *__restrict__ r, int64_t ldr) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= k) return;
  const int64_t p = idx[j];
  float v;
  if (p < 0 || p >= n)
    v = __builtin_nanf("");
  else
    v = s <= j ? w[(int64_t)s * ldw + p] : 0.f;
  r[(int64_t)s * ldr + j] = v;
}

hipError_t launch_qless_r(const float *w, int64_t n, int64_t ldw, const int64_t *idx, int k,
                          float *r, int64_t ldr, hipStream_t s) {
  if (k < 1) return hipSuccess;
  hipLaunchKernelGGL(k_qless_r, dim3((unsigned)((k + 255) / 256), (unsigned)k), dim3(256), 0, s,
                     w, n, ldw, idx, k, r, ldr);
  return hipGetLastError();
}

}  // namespace gcss
