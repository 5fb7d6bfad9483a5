// Reduced-precision storage of A: bfloat16 (round to nearest even) and OCP
// FP8 E4M3 (e4m3fn) with one binary32 scale per column.  One wavefront per
// column.  The encoders are written from the formats' definitions with
// exact scaling by powers of two and round-half-even (v_rndne_f32).
#include "gcss_device.h"

namespace gcss {

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)(((u >> 16) & 0x8000u) | 0x7FC0u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// E4M3: bias 7, subnormal step 2^-9, largest finite 448 (S.1111.110).
__device__ __forceinline__ uint8_t fp8_rne_sat(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
  const float ax = fabsf(x);
  if (ax != ax) return (uint8_t)(sign | 0x7Fu);
  if (ax >= 448.f) return (uint8_t)(sign | 0x7Eu);
  if (ax < 0.015625f) {  // below 2^-6: multiples of 2^-9 (code 8 is 2^-6 itself)
    const int c = (int)rintf(ax * 512.f);
    return (uint8_t)(sign | c);
  }
  int e = (int)((__float_as_uint(ax) >> 23) & 0xFFu) - 127;  // 2^e <= ax < 2^(e+1)
  float sc = ldexpf(ax, 3 - e);                                // in [8, 16)
  int q = (int)rintf(sc);
  if (q == 16) {
    q = 8;
    e += 1;
  }
  return (uint8_t)(sign | ((e + 7) << 3) | (q - 8));
}

__global__ __launch_bounds__(256) void k_quantize(const float *__restrict__ a, int64_t m,
                                                  int64_t n, int64_t lda, int dtype,
                                                  void *__restrict__ out, int64_t ldo,
                                                  float *__restrict__ scales) {
  const int lane = threadIdx.x & 63;
  const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= n) return;
  const float *src = a + col * lda;
  if (dtype == DT_BF16) {
    uint16_t *dst = (uint16_t *)out + col * ldo;
    for (int64_t j = lane; j < ldo; j += 64) dst[j] = j < m ? bf16_rne(src[j]) : (uint16_t)0;
    return;
  }
  float amax = 0.f;
  for (int64_t j = lane; j < m; j += 64) amax = fmaxf(amax, fabsf(src[j]));
  amax = wave_max(amax);
  const float s = amax > 0.f ? amax / 448.f : 1.f;
  if (lane == 0) scales[col] = s;
  uint8_t *dst = (uint8_t *)out + col * ldo;
  for (int64_t j = lane; j < ldo; j += 64) dst[j] = j < m ? fp8_rne_sat(src[j] / s) : (uint8_t)0;
}

// out[j + c*ldo] = the bfloat16 value in[j + c*ldi] as binary32 (exact),
// rows m..ldo-1 set to zero.  One wavefront per column.
__global__ __launch_bounds__(256) void k_bf16_to_f32(const uint16_t *__restrict__ in, int64_t m,
                                                     int64_t n, int64_t ldi,
                                                     float *__restrict__ out, int64_t ldo) {
  const int lane = threadIdx.x & 63;
  const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= n) return;
  const uint16_t *src = in + col * ldi;
  float *dst = out + col * ldo;
  for (int64_t j = lane; j < ldo; j += 64)
    dst[j] = j < m ? __uint_as_float((uint32_t)src[j] << 16) : 0.f;
}

hipError_t launch_bf16_to_f32(const void *in, int64_t m, int64_t n, int64_t ldi, float *out,
                              int64_t ldo, hipStream_t s) {
  hipLaunchKernelGGL(k_bf16_to_f32, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s,
                     (const uint16_t *)in, m, n, ldi, out, ldo);
  return hipGetLastError();
}

hipError_t launch_quantize(const float *a, int64_t m, int64_t n, int64_t lda, int dtype,
                           void *out, int64_t ldo, float *scales, hipStream_t s) {
  hipLaunchKernelGGL(k_quantize, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, a, m, n, lda,
                     dtype, out, ldo, scales);
  return hipGetLastError();
}

}  // namespace gcss
