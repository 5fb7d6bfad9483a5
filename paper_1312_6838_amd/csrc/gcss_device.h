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

// Sum over the 64 lanes of a wave, returned wave-uniform: four DPP steps sum
// each row of 16 lanes into all of its lanes (quad swaps, then the half-row
// and row mirrors), two row broadcasts carry rows 0-2 into row 3, and lane 63
// holds the total.  All VALU: no LDS crossbar round trips per column.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_step(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
__device__ __forceinline__ float wave_total(float v) {
  v += dpp_step<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_step<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_step<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_step<0x140, 0xF>(v);  // row_mirror
  v += dpp_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
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

// Element size and elements per 16-byte chunk of each storage type.
template <int DT>
struct Elem;
template <>
struct Elem<DT_F32> {
  static constexpr int esize = 4, epc = 4;
};
template <>
struct Elem<DT_BF16> {
  static constexpr int esize = 2, epc = 8;
};
template <>
struct Elem<DT_FP8> {
  static constexpr int esize = 1, epc = 16;
};

// Decode one 16-byte chunk into EPC floats.
template <int DT>
__device__ __forceinline__ void decode_chunk(const uint4 &r, float *v) {
  if constexpr (DT == DT_F32) {
    v[0] = __uint_as_float(r.x);
    v[1] = __uint_as_float(r.y);
    v[2] = __uint_as_float(r.z);
    v[3] = __uint_as_float(r.w);
  } else if constexpr (DT == DT_BF16) {
    v[0] = bf16_lo(r.x);
    v[1] = bf16_hi(r.x);
    v[2] = bf16_lo(r.y);
    v[3] = bf16_hi(r.y);
    v[4] = bf16_lo(r.z);
    v[5] = bf16_hi(r.z);
    v[6] = bf16_lo(r.w);
    v[7] = bf16_hi(r.w);
  } else {
    fp8x4_decode(r.x, v + 0);
    fp8x4_decode(r.y, v + 4);
    fp8x4_decode(r.z, v + 8);
    fp8x4_decode(r.w, v + 12);
  }
}

__device__ __forceinline__ double col_scale(const AView &A, int64_t i) {
  return A.dtype == DT_FP8 ? (double)A.scale[i] : 1.0;
}

// ---- counter-based random signs (concise target, Section 5.1) ----
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of
// (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)), the key bumped by the Weyl constants before every round but
// the first.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = c.x * 0xD2511F53u, hi0 = __umulhi(c.x, 0xD2511F53u);
    const uint32_t lo1 = c.z * 0xCD9E8D57u, hi1 = __umulhi(c.z, 0xCD9E8D57u);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// Entries i (row of Omega = column of A), 4*jb .. 4*jb+3 of the sign matrix
// for key (k0, k1): word w of Philox(counter (i lo, i hi, jb, 0)) gives
// 0 if (w >> 1) >= thr, else -1 (w odd) or +1 (w even).
__device__ __forceinline__ uint4 sign_words(int64_t i, uint32_t jb, uint32_t k0, uint32_t k1) {
  return philox4x32_10(make_uint4((uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), jb, 0u),
                       k0, k1);
}
__device__ __forceinline__ float sign_entry(uint32_t w, uint32_t thr) {
  return (w >> 1) < thr ? ((w & 1u) ? -1.f : 1.f) : 0.f;
}

}  // namespace gcss
