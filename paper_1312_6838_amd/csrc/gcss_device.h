// Device-side helpers shared by the kernels: wavefront reductions, the
// candidate order used by every argmax, and element decoding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "gcss_internal.h"

namespace gcss {

constexpr int kWave = 64;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

// Candidate order of the argmax: larger score first, then the lower index.
// Non-candidates carry score -inf and index INT64_MAX, so they lose to any
// real candidate and the order is total (the reduction order cannot change
// the result).
constexpr int64_t kNoIdx = INT64_MAX;

__device__ __forceinline__ bool better(double a, int64_t ia, double b, int64_t ib) {
  return a > b || (a == b && ia < ib);
}

__device__ __forceinline__ void wave_argmax(double &s, int64_t &i) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double os = __shfl_xor(s, o, kWave);
    int64_t oi = __shfl_xor((long long)i, o, kWave);
    if (better(os, oi, s, i)) {
      s = os;
      i = oi;
    }
  }
}

// Reads of values another workgroup published before its release fence.
__device__ __forceinline__ double load_acquire_f64(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t load_acquire_i64(const int64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last-block-done protocol: every workgroup publishes its partial results,
// then one thread releases them at device scope (a single fence per
// workgroup: on CDNA a device-scope fence writes back the L2, so one per
// thread would cost far more than the work) and bumps a counter; the
// workgroup that sees the final count acquires (one fence) and does the
// cross-workgroup step, then re-arms the counter.  Must be called by all
// threads of the block.  Returns true in the last one.
__device__ __forceinline__ bool last_block_arrive(uint32_t *counter) {
  __shared__ int am_last;
  __syncthreads();  // this block's stores are complete at workgroup scope
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = atomicAdd(counter, 1u);
    am_last = (prev == gridDim.x - 1);
    if (am_last) __threadfence();
  }
  __syncthreads();
  return am_last != 0;
}

// ---- element decoding ----
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// Decode one 32-bit word holding four E4M3 codes (byte 0 first).
__device__ __forceinline__ void fp8x4_decode(uint32_t w, float *o) {
  f32x2 a = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
  f32x2 b = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
  o[0] = a[0];
  o[1] = a[1];
  o[2] = b[0];
  o[3] = b[1];
}

// Element j of column i of A as float, without the FP8 column scale.
__device__ __forceinline__ float load_elem(const AView &A, int64_t i, int64_t j) {
  if (A.dtype == DT_F32) return ((const float *)A.a)[i * A.lda + j];
  if (A.dtype == DT_BF16) {
    uint16_t h = ((const uint16_t *)A.a)[i * A.lda + j];
    return __uint_as_float((uint32_t)h << 16);
  }
  uint8_t c = ((const uint8_t *)A.a)[i * A.lda + j];
  f32x2 v = __builtin_amdgcn_cvt_pk_f32_fp8((uint32_t)c, false);
  return v[0];
}

__device__ __forceinline__ double col_scale(const AView &A, int64_t i) {
  return A.dtype == DT_FP8 ? (double)A.scale[i] : 1.0;
}

}  // namespace gcss
