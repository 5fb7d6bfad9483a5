// Dense contractions of the selection, on the CDNA matrix cores
// (v_mfma_f32_16x16x4_f32, FP32 in / FP32 accumulate):
//
//   init scores (Algorithm 3, first line):   f_i = || X A_i ||^2,
//       X = B^T (r x m), the epilogue sums the squares so the r x n product is
//       never stored; g_i = || A_i ||^2 is accumulated from the same A tiles.
//   init scores, Gram target (B = A enters only through C = A A^T):
//       f_i = A_i^T C A_i = A_i^T T A_i with T = diag(C) + 2 strictly-upper(C),
//       so only the tiles of C on or right of the diagonal are multiplied
//       (half the flops); T is formed from C while its tiles are loaded.
//   Gram matrix C = A A^T (symmetric rank-n update, upper tiles, split-K).
//   Projection B = A Omega (Section 5.1), split-K with a fixed-order reduce.
//
// Two LDS layouts feed the 16x16x4 instruction (lane l supplies row l%16 and
// k index l/16 of each operand; lane l, register v of the result holds
// D[4*(l/16) + v][l%16]):
//  * k-major (operands whose k index is contiguous in memory: rows of X,
//    columns of A as the right operand): each tile row holds BKT consecutive
//    k values (pitch BKT + 4).  A lane reads one 16-byte quad of k values per
//    operand and feeds four instructions with its components, the four lane
//    groups covering 16 consecutive k.
//  * MN-major (operands whose row index is contiguous: A as the left operand
//    of A A^T and A Omega, Omega itself): each LDS row holds one k value and
//    128 tile rows (pitch 132), written with 16-byte stores.  Tile row
//    4*rho + b is row rho of the b-th 16-row instruction block, so one 16-byte
//    read gives a lane its operand for four blocks at one k.
#include <cstdlib>
#include <type_traits>

#include "gcss_device.h"

namespace gcss {

namespace {
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kX3BK = 32;          // k per stage
constexpr int kX3RP = 40;          // LDS row pitch in bfloat16 (32 + pad)
constexpr int kX3Plane = 256 * kX3RP;  // one plane of a 256-row operand

__device__ __forceinline__ void split3(float a, __bf16 &h, __bf16 &m, __bf16 &l) {
  h = (__bf16)a;
  const float r1 = a - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}

// Load tasks of a 256-row x 32-k operand stage, for operands whose rows are
// contiguous in memory: task t (0..255) moves rows x3_task_row(t) .. +3 for
// k = x3_task_k(t) .. +7 into the k-contiguous planes (pitch kX3RP).  The 16
// tasks of a 16-lane group cover four row quads and the four k groups, so
// their 16-byte plane stores fall in distinct bank quads (row quads alone,
// 320 bytes apart, would share four of them).  A wave's loads still read
// 256 contiguous bytes per k group.
__device__ __forceinline__ int x3_task_row(int t) {
  return 64 * (t >> 6) + 4 * ((t & 3) + 4 * ((t >> 4) & 3));
}
__device__ __forceinline__ int x3_task_k(int t) { return 8 * ((t >> 2) & 3); }

// binary32 products on the bfloat16 matrix cores (three-part split) for the
// Gram matrix and the initial scores; GCSS_MFMA_X3=0 keeps the binary32 MFMA
// kernels
bool mfma_x3() {
  const char *e = std::getenv("GCSS_MFMA_X3");
  return !(e && e[0] == '0');
}
}  // namespace


// MFMA/LDS interleaving strategy of the compiler for the stage loops
#ifndef GCSS_IGLP
#define GCSS_IGLP 1
#endif

constexpr int BK = 16;   // k values per stage of the FP64 kernel
constexpr int MP = 132;  // MN-major LDS pitch in floats (128 rows + pad)

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// k-major: acc[rb][nb] += X_rows(rb) * Y_cols(nb) over one stage of BKT k values.
template <int RB, int NB, int BKT>
__device__ __forceinline__ void mma_stage_k(const float *Xs, int xrow0, const float *Ys,
                                            int ycol0, int lane, f32x4 (&acc)[RB][NB]) {
  constexpr int KP = BKT + 4;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < BKT / 16; ++kk) {
    const int kq = 16 * kk + 4 * g;
    float4 xa[RB], yb[NB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) xa[rb] = *(const float4 *)(Xs + (xrow0 + 16 * rb + r) * KP + kq);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) yb[nb] = *(const float4 *)(Ys + (ycol0 + 16 * nb + r) * KP + kq);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        acc[rb][nb] = mfma4(xa[rb].x, yb[nb].x, acc[rb][nb]);
        acc[rb][nb] = mfma4(xa[rb].y, yb[nb].y, acc[rb][nb]);
        acc[rb][nb] = mfma4(xa[rb].z, yb[nb].z, acc[rb][nb]);
        acc[rb][nb] = mfma4(xa[rb].w, yb[nb].w, acc[rb][nb]);
      }
  }
  __builtin_amdgcn_iglp_opt(GCSS_IGLP);
}

// MN-major: a wave's 64 x 64 block at tile rows xr0.., columns yc0..;
// acc[rb][nb] row rho <-> tile row xr0 + 4*rho + rb, column c <-> yc0 + 4*c + nb.
// The operands of step s + 1 are read from LDS before the 16 instructions of
// step s are issued (the compiler's MFMA/LDS interleaving strategy keeps that
// order), so the LDS latency overlaps matrix work instead of stalling the
// pipe between steps.
template <int BKT>
__device__ __forceinline__ void mma_stage_mn(const float *Xs, int xr0, const float *Ys, int yc0,
                                             int lane, f32x4 (&acc)[4][4]) {
  const int r = lane & 15, g = lane >> 4;
  constexpr int NS = BKT / 4;
  float4 xb = *(const float4 *)(Xs + g * MP + xr0 + 4 * r);
  float4 yb = *(const float4 *)(Ys + g * MP + yc0 + 4 * r);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const float4 x = xb, y = yb;
    if (s + 1 < NS) {
      const int k = 4 * (s + 1) + g;
      xb = *(const float4 *)(Xs + k * MP + xr0 + 4 * r);
      yb = *(const float4 *)(Ys + k * MP + yc0 + 4 * r);
    }
    const float xv[4] = {x.x, x.y, x.z, x.w};
    const float yv[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[rb][nb] = mfma4(xv[rb], yv[nb], acc[rb][nb]);
  }
  __builtin_amdgcn_iglp_opt(GCSS_IGLP);
}

template <int DT>
struct EInfo;
template <>
struct EInfo<DT_F32> {
  static constexpr int esize = 4, epc = 4;
};
template <>
struct EInfo<DT_BF16> {
  static constexpr int esize = 2, epc = 8;
};
template <>
struct EInfo<DT_FP8> {
  static constexpr int esize = 1, epc = 16;
};

template <int DT>
__device__ __forceinline__ void decode16(const uint4 &r, float *v) {
  if constexpr (DT == DT_F32) {
    v[0] = __uint_as_float(r.x);
    v[1] = __uint_as_float(r.y);
    v[2] = __uint_as_float(r.z);
    v[3] = __uint_as_float(r.w);
  } else if constexpr (DT == DT_BF16) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      v[2 * x] = bf16_lo(w[x]);
      v[2 * x + 1] = bf16_hi(w[x]);
    }
  } else {
    fp8x4_decode(r.x, v + 0);
    fp8x4_decode(r.y, v + 4);
    fp8x4_decode(r.z, v + 8);
    fp8x4_decode(r.w, v + 12);
  }
}

// Four consecutive elements of a column starting at a multiple of 4, as floats.
template <int DT>
__device__ __forceinline__ float4 load4(const void *base, int64_t off) {
  if constexpr (DT == DT_F32) {
    return *(const float4 *)((const float *)base + off);
  } else if constexpr (DT == DT_BF16) {
    const uint2 w = *(const uint2 *)((const uint16_t *)base + off);
    return make_float4(bf16_lo(w.x), bf16_hi(w.x), bf16_lo(w.y), bf16_hi(w.y));
  } else {
    const uint32_t w = *(const uint32_t *)((const uint8_t *)base + off);
    float v[4];
    fp8x4_decode(w, v);
    return make_float4(v[0], v[1], v[2], v[3]);
  }
}

// ---------------------------------------------------------------------------
// Initial scores.  Workgroup: 4 waves stacked along the rows of X (R), one
// tile of NT = 16*NB columns of A.  Rows are processed in chunks of
// RT = 64*RB; the column results are accumulated across chunks.  With TRI,
// X = C is weighted as T/2 (zero left of the diagonal, so the k loop starts
// at r0; one half on it) and the sum is doubled.
template <int DT, int RB, int NB, int BKT, bool TRI, bool DB>
__global__ __launch_bounds__(256) void k_init(const float *__restrict__ X, int64_t ldx,
                                              int64_t R, AView A, double *__restrict__ f0,
                                              double *__restrict__ g0,
                                              uint8_t *__restrict__ mask0) {
  constexpr int RT = 64 * RB, NT = 16 * NB, KP = BKT + 4;
  constexpr int ES = EInfo<DT>::esize, EPC = EInfo<DT>::epc;
  constexpr int XQ = BKT / 4;              // float4 per X row per stage
  constexpr int XPT = RT * XQ / 256;       // X float4 per thread per stage
  constexpr int YCC = BKT * ES / 16;       // 16-byte chunks per A column per stage
  constexpr int YCH = NT * YCC;            // A chunks per stage
  constexpr int YPT = (YCH + 255) / 256;   // A chunks per thread per stage
  static_assert(RT % BKT == 0 && YCC >= 1 && YCC <= 16, "tile shape");
  constexpr int NBUF = DB ? 2 : 1;
  __shared__ __align__(16) float Xsb[NBUF][RT * KP];
  __shared__ __align__(16) float Ysb[NBUF][NT * KP];
  __shared__ double red[4][NT];
  __shared__ double gs[NT];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m = A.m, n = A.n;
  const int64_t j0 = (int64_t)blockIdx.x * NT;
  const char *abase = (const char *)A.a;
  const int64_t colb = A.lda * ES;

  double gacc[YPT];
#pragma unroll
  for (int u = 0; u < YPT; ++u) gacc[u] = 0.0;
  double colacc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) colacc[nb] = 0.0;

  const int64_t nchunks = (R + RT - 1) / RT;
  const int64_t ksteps = (m + BKT - 1) / BKT;
  for (int64_t rc = 0; rc < nchunks; ++rc) {
    const int64_t r0 = rc * RT;
    f32x4 acc[RB][NB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    float4 xr[XPT];
    uint4 yr[YPT];
    // X loads are unconditional 16-byte loads from clamped (valid) addresses;
    // only the uniform tail and diagonal stages apply masks
    const bool rtail = r0 + RT > R;
    auto gload = [&](int64_t k0) {
      const bool ktail = k0 + BKT > m;
      const bool diag = TRI && k0 < r0 + RT;
#pragma unroll
      for (int u = 0; u < XPT; ++u) {
        const int q = tid + 256 * u;
        const int row = q / XQ, kq = (q % XQ) * 4;
        const int64_t gr = r0 + row, gk = k0 + kq;
        const int64_t grc = gr < R ? gr : R - 1, gkc = gk < m ? gk : 0;
        float4 v = *(const float4 *)(X + grc * ldx + gkc);
        if (rtail || ktail) {
          const bool rok = gr < R;
          v.x = (rok && gk < m) ? v.x : 0.f;
          v.y = (rok && gk + 1 < m) ? v.y : 0.f;
          v.z = (rok && gk + 2 < m) ? v.z : 0.f;
          v.w = (rok && gk + 3 < m) ? v.w : 0.f;
        }
        if (diag) {
          // rows of T/2: weight 1 right of the diagonal, 1/2 on it, 0 left of it
          const int d = (int)(gk - gr);
          v.x *= d > 0 ? 1.f : (d == 0 ? 0.5f : 0.f);
          v.y *= d + 1 > 0 ? 1.f : (d + 1 == 0 ? 0.5f : 0.f);
          v.z *= d + 2 > 0 ? 1.f : (d + 2 == 0 ? 0.5f : 0.f);
          v.w *= d + 3 > 0 ? 1.f : (d + 3 == 0 ? 0.5f : 0.f);
        }
        xr[u] = v;
      }
#pragma unroll
      for (int u = 0; u < YPT; ++u) {
        const int q = tid + 256 * u;
        const int col = q / YCC, ch = q % YCC;
        const int64_t gk = k0 + ch * EPC;
        if (q < YCH && j0 + col < n && gk < m)
          yr[u] = *(const uint4 *)(abase + (j0 + col) * colb + gk * ES);
        else
          yr[u] = make_uint4(0u, 0u, 0u, 0u);
      }
    };
    auto sstore = [&](int64_t k0, int bsel) {
      float *Xs = Xsb[bsel];
      float *Ys = Ysb[bsel];
#pragma unroll
      for (int u = 0; u < XPT; ++u) {
        const int q = tid + 256 * u;
        const int row = q / XQ, kq = (q % XQ) * 4;
        *(float4 *)(Xs + row * KP + kq) = xr[u];
      }
#pragma unroll
      for (int u = 0; u < YPT; ++u) {
        const int q = tid + 256 * u;
        if (q >= YCH) continue;
        const int col = q / YCC, ch = q % YCC;
        float v[EPC];
        decode16<DT>(yr[u], v);
        const int64_t gk = k0 + ch * EPC;
#pragma unroll
        for (int e = 0; e < EPC; ++e)
          if (gk + e >= m) v[e] = 0.f;
        if (rc == 0) {
#pragma unroll
          for (int e = 0; e < EPC; ++e) gacc[u] = fma((double)v[e], (double)v[e], gacc[u]);
        }
#pragma unroll
        for (int e = 0; e < EPC; e += 4)
          *(float4 *)(Ys + col * KP + ch * EPC + e) = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
      }
    };

    const int64_t ks0 = TRI ? r0 / BKT : 0;
    gload(ks0 * BKT);
    if constexpr (DB) {
      __syncthreads();  // the previous row chunk's last stage is done with both buffers
      sstore(ks0 * BKT, 0);
      __syncthreads();
      int cur = 0;
      for (int64_t ks = ks0; ks < ksteps; ++ks) {
        const bool more = ks + 1 < ksteps;
        if (more) gload((ks + 1) * BKT);
        mma_stage_k<RB, NB, BKT>(Xsb[cur], wave * 16 * RB, Ysb[cur], 0, lane, acc);
        if (more) sstore((ks + 1) * BKT, cur ^ 1);
        __syncthreads();
        cur ^= 1;
      }
    } else {
      for (int64_t ks = ks0; ks < ksteps; ++ks) {
        __syncthreads();
        sstore(ks * BKT, 0);
        __syncthreads();
        if (ks + 1 < ksteps) gload((ks + 1) * BKT);
        mma_stage_k<RB, NB, BKT>(Xsb[0], wave * 16 * RB, Ysb[0], 0, lane, acc);
      }
    }

    // epilogue of this row chunk, one 16-row block at a time (bounded registers)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int64_t i = r0 + wave * 16 * RB + 16 * rb + 4 * (lane >> 4);
      if constexpr (TRI) {
        // branch-free: clamped (always valid) addresses, masked values
        const int64_t ic = i < m ? i : 0;
        const float w0 = i < m ? 1.f : 0.f, w1 = i + 1 < m ? 1.f : 0.f;
        const float w2 = i + 2 < m ? 1.f : 0.f, w3 = i + 3 < m ? 1.f : 0.f;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int64_t j = j0 + 16 * nb + (lane & 15);
          const float wj = j < n ? 1.f : 0.f;
          const float4 a = load4<DT>(A.a, (j < n ? j : 0) * A.lda + ic);
          const float p = acc[rb][nb][0] * (a.x * w0) + acc[rb][nb][1] * (a.y * w1) +
                          acc[rb][nb][2] * (a.z * w2) + acc[rb][nb][3] * (a.w * w3);
          colacc[nb] += (double)(p * wj);
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          double s = 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v) s += (double)acc[rb][nb][v] * (double)acc[rb][nb][v];
          colacc[nb] += s;
        }
      }
    }
  }

  // columns: sum over the 4 lane groups, then over the 4 waves (fixed order)
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    double s = colacc[nb];
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    if (lane < 16) red[wave][16 * nb + lane] = s;
  }
  // g: sum over the YCC threads of a column
#pragma unroll
  for (int u = 0; u < YPT; ++u) {
    const int q = tid + 256 * u;
    double gsum = gacc[u];
    if constexpr (YCC >= 2) gsum += __shfl_xor(gsum, 1, 64);
    if constexpr (YCC >= 4) gsum += __shfl_xor(gsum, 2, 64);
    if constexpr (YCC >= 8) gsum += __shfl_xor(gsum, 4, 64);
    if constexpr (YCC >= 16) gsum += __shfl_xor(gsum, 8, 64);
    if (q < YCH && q % YCC == 0) gs[q / YCC] = gsum;
  }
  __syncthreads();
  if (tid < NT) {
    const int64_t j = j0 + tid;
    if (j < n) {
      const double fv = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      const double sc = col_scale(A, j);
      const double f = (TRI ? 2.0 : 1.0) * sc * sc * fv, g = sc * sc * gs[tid];
      f0[j] = f;
      g0[j] = g;
      mask0[j] = (g > 0.0 && isfinite(g) && isfinite(f)) ? 0 : 2;
    }
  }
}

// ---------------------------------------------------------------------------
// Initial scores with 256 x 256 workgroup tiles (rows of X x columns of A),
// 8 waves of 128 x 64 (8 x 4 instruction blocks, two waves per SIMD),
// k-major LDS stages of 16 k values, two buffers.  Same arithmetic as k_init:
// per row chunk of 256 rows the product is reduced into per-column sums
// (sum of squares, or the dot with A for TRI), and g_i comes from the A
// tiles of the first chunk.
constexpr int kI2Threads = 512;

template <int DT, bool TRI>
__global__ __launch_bounds__(kI2Threads, 1) void k_init256(const float *__restrict__ X,
                                                          int64_t ldx, int64_t R, AView A,
                                                          double *__restrict__ f0,
                                                          double *__restrict__ g0,
                                                          uint8_t *__restrict__ mask0) {
  constexpr int BKT = 16, KP = BKT + 4, RT = 256, NT = 256;
  constexpr int ES = EInfo<DT>::esize, EPC = EInfo<DT>::epc;
  constexpr int XQ = BKT / 4;                                  // float4 per X row per stage
  constexpr int XPT = RT * XQ / kI2Threads;                    // 2
  constexpr int YCC = BKT * ES / 16;                           // 16-byte chunks per column
  constexpr int YCH = NT * YCC;                                // chunks per stage
  constexpr int YPT = (YCH + kI2Threads - 1) / kI2Threads;     // chunks per thread
  __shared__ __align__(16) float Xsb[2][RT * KP];
  __shared__ __align__(16) float Ysb[2][NT * KP];
  __shared__ double red[2][NT];
  __shared__ double gs[NT];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 2) * 128, wc = (wave & 3) * 64;
  const int64_t m = A.m, n = A.n;
  const int64_t j0 = (int64_t)blockIdx.x * NT;
  const char *abase = (const char *)A.a;
  const int64_t colb = A.lda * ES;

  double gacc[YPT];
#pragma unroll
  for (int u = 0; u < YPT; ++u) gacc[u] = 0.0;
  double colacc[4] = {0.0, 0.0, 0.0, 0.0};

  const int64_t nchunks = (R + RT - 1) / RT;
  const int64_t ksteps = (m + BKT - 1) / BKT;
  for (int64_t rc = 0; rc < nchunks; ++rc) {
    const int64_t r0 = rc * RT;
    f32x4 acc[8][4];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    float4 xr[XPT];
    uint4 yr[YPT];
    const bool rtail = r0 + RT > R;
    auto gload = [&](int64_t k0) {
      const bool ktail = k0 + BKT > m;
      const bool diag = TRI && k0 < r0 + RT;
#pragma unroll
      for (int u = 0; u < XPT; ++u) {
        const int q = tid + kI2Threads * u;
        const int row = q / XQ, kq = (q % XQ) * 4;
        const int64_t gr = r0 + row, gk = k0 + kq;
        const int64_t grc = gr < R ? gr : R - 1, gkc = gk < m ? gk : 0;
        float4 v = *(const float4 *)(X + grc * ldx + gkc);
        if (rtail || ktail) {
          const bool rok = gr < R;
          v.x = (rok && gk < m) ? v.x : 0.f;
          v.y = (rok && gk + 1 < m) ? v.y : 0.f;
          v.z = (rok && gk + 2 < m) ? v.z : 0.f;
          v.w = (rok && gk + 3 < m) ? v.w : 0.f;
        }
        if (diag) {
          const int d = (int)(gk - gr);
          v.x *= d > 0 ? 1.f : (d == 0 ? 0.5f : 0.f);
          v.y *= d + 1 > 0 ? 1.f : (d + 1 == 0 ? 0.5f : 0.f);
          v.z *= d + 2 > 0 ? 1.f : (d + 2 == 0 ? 0.5f : 0.f);
          v.w *= d + 3 > 0 ? 1.f : (d + 3 == 0 ? 0.5f : 0.f);
        }
        xr[u] = v;
      }
#pragma unroll
      for (int u = 0; u < YPT; ++u) {
        const int q = tid + kI2Threads * u;
        const int col = q / YCC, ch = q % YCC;
        const int64_t gk = k0 + ch * EPC;
        if (q < YCH && j0 + col < n && gk < m)
          yr[u] = *(const uint4 *)(abase + (j0 + col) * colb + gk * ES);
        else
          yr[u] = make_uint4(0u, 0u, 0u, 0u);
      }
    };
    auto sstore = [&](int64_t k0, int bsel) {
      float *Xs = Xsb[bsel];
      float *Ys = Ysb[bsel];
#pragma unroll
      for (int u = 0; u < XPT; ++u) {
        const int q = tid + kI2Threads * u;
        const int row = q / XQ, kq = (q % XQ) * 4;
        *(float4 *)(Xs + row * KP + kq) = xr[u];
      }
#pragma unroll
      for (int u = 0; u < YPT; ++u) {
        const int q = tid + kI2Threads * u;
        if (q >= YCH) continue;
        const int col = q / YCC, ch = q % YCC;
        float v[EPC];
        decode16<DT>(yr[u], v);
        const int64_t gk = k0 + ch * EPC;
#pragma unroll
        for (int e = 0; e < EPC; ++e)
          if (gk + e >= m) v[e] = 0.f;
        if (rc == 0) {
#pragma unroll
          for (int e = 0; e < EPC; ++e) gacc[u] = fma((double)v[e], (double)v[e], gacc[u]);
        }
#pragma unroll
        for (int e = 0; e < EPC; e += 4)
          *(float4 *)(Ys + col * KP + ch * EPC + e) = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
      }
    };

    const int64_t ks0 = TRI ? r0 / BKT : 0;
    gload(ks0 * BKT);
    __syncthreads();  // the previous chunk's last stage is done with both buffers
    sstore(ks0 * BKT, 0);
    __syncthreads();
    int cur = 0;
    for (int64_t ks = ks0; ks < ksteps; ++ks) {
      const bool more = ks + 1 < ksteps;
      if (more) gload((ks + 1) * BKT);
      {
        const float *Xs = Xsb[cur];
        const float *Ys = Ysb[cur];
        const int r = lane & 15, g = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < BKT / 16; ++kk) {
          const int kq = 16 * kk + 4 * g;
          float4 yb[4];
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) yb[nb] = *(const float4 *)(Ys + (wc + 16 * nb + r) * KP + kq);
          // row fragments in two halves of four (fewer operand registers live)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            float4 xa[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) xa[b] = *(const float4 *)(Xs + (wr + 16 * (4 * h + b) + r) * KP + kq);
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
              for (int nb = 0; nb < 4; ++nb) {
                f32x4 &c = acc[4 * h + b][nb];
                c = mfma4(xa[b].x, yb[nb].x, c);
                c = mfma4(xa[b].y, yb[nb].y, c);
                c = mfma4(xa[b].z, yb[nb].z, c);
                c = mfma4(xa[b].w, yb[nb].w, c);
              }
          }
        }
      }
      if (more) sstore((ks + 1) * BKT, cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }

    // epilogue of this row chunk, one 16-row block at a time (bounded registers)
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) {
      const int64_t i = r0 + wr + 16 * rb + 4 * (lane >> 4);
      if constexpr (TRI) {
        const int64_t ic = i < m ? i : 0;
        const float w0 = i < m ? 1.f : 0.f, w1 = i + 1 < m ? 1.f : 0.f;
        const float w2 = i + 2 < m ? 1.f : 0.f, w3 = i + 3 < m ? 1.f : 0.f;
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const int64_t j = j0 + wc + 16 * nb + (lane & 15);
          const float wj = j < n ? 1.f : 0.f;
          const float4 a = load4<DT>(A.a, (j < n ? j : 0) * A.lda + ic);
          const float p = acc[rb][nb][0] * (a.x * w0) + acc[rb][nb][1] * (a.y * w1) +
                          acc[rb][nb][2] * (a.z * w2) + acc[rb][nb][3] * (a.w * w3);
          colacc[nb] += (double)(p * wj);
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          double sq = 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v) sq += (double)acc[rb][nb][v] * (double)acc[rb][nb][v];
          colacc[nb] += sq;
        }
      }
    }
  }

  // columns: sum over the 4 lane groups, then over the 2 row-waves (fixed order)
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    double s = colacc[nb];
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    if (lane < 16) red[wave >> 2][wc + 16 * nb + lane] = s;
  }
  // g: sum over the YCC threads of a column
#pragma unroll
  for (int u = 0; u < YPT; ++u) {
    const int q = tid + kI2Threads * u;
    double gsum = gacc[u];
    if constexpr (YCC >= 2) gsum += __shfl_xor(gsum, 1, 64);
    if constexpr (YCC >= 4) gsum += __shfl_xor(gsum, 2, 64);
    if constexpr (YCC >= 8) gsum += __shfl_xor(gsum, 4, 64);
    if (q < YCH && q % YCC == 0) gs[q / YCC] = gsum;
  }
  __syncthreads();
  if (tid < NT) {
    const int64_t j = j0 + tid;
    if (j < n) {
      const double fv = red[0][tid] + red[1][tid];
      const double sc = col_scale(A, j);
      const double f = (TRI ? 2.0 : 1.0) * sc * sc * fv, g = sc * sc * gs[tid];
      f0[j] = f;
      g0[j] = g;
      mask0[j] = (g > 0.0 && isfinite(g) && isfinite(f)) ? 0 : 2;
    }
  }
}

// ---------------------------------------------------------------------------
// Initial scores on the bfloat16 matrix cores: k_init256's computation
// (f_j = ||X A_j||^2, or with TRI f_j = A_j^T (X + X^T) A_j / 2 for the
// symmetric X = C by its upper triangle).  X (binary32) is split into three
// bfloat16 parts as in k_gram_x3; so is binary32 A (six part products per
// product), while BF16 and FP8 codes are exact in one bfloat16 part (three
// part products; the FP8 column scale enters f and g at the end).  X rows
// and A columns both hold k contiguously, so a thread loads eight
// consecutive k of one row or column and writes each plane with one 16-byte
// LDS store.  One workgroup per 256 columns of A, all row chunks of RT rows
// of X: 256 (eight waves of 128 x 64), or 128 for narrow targets (R <= 128:
// eight waves of 64 x 64, one X load task per thread).
template <bool TRI, int DT, int RT>
__global__ __launch_bounds__(kI2Threads, 1) void k_init_x3(const float *__restrict__ X,
                                                           int64_t ldx, int64_t R, AView A,
                                                           double *__restrict__ f0,
                                                           double *__restrict__ g0,
                                                           uint8_t *__restrict__ mask0) {
  constexpr int NT = 256;
  static_assert(kI2Threads == 512, "two load tasks per operand and thread");
  static_assert(RT == 256 || (RT == 128 && !TRI), "row chunk of 256, or 128 without the triangle");
  constexpr int XT = RT * 4 / kI2Threads;  // X load tasks per thread (2 or 1)
  constexpr int RBW = RT / 32;             // 16-row blocks per wave
  __shared__ __align__(16) __bf16 Ls[2][3][kX3Plane];  // [X rows / A columns][plane][.][k]
  __shared__ double red[2][NT];     // f partial sums per row-wave, over the row chunks
  __shared__ double gpart[4][NT];   // g partial sums per k group

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 2) * (RT / 2), wc = (wave & 3) * 64;
  const int lr = lane & 15, kq = (lane >> 4) * 8;
  const int64_t m = A.m, n = A.n;
  const int64_t j0 = (int64_t)blockIdx.x * NT;
  const float *a = (const float *)A.a;
  constexpr int ES = EInfo<DT>::esize;
  constexpr int YP = DT == DT_F32 ? 3 : 1;  // bfloat16 parts of an A element

  // load tasks: task t of X = row t % RT, k group t / RT; task t (0..1023) of
  // A = column t & 255, k group t >> 8
  // (partial sums live in LDS, keeping registers for the operands)
  for (int t = tid; t < 2 * NT; t += kI2Threads) red[t >> 8][t & 255] = 0.0;
  for (int t = tid; t < 4 * NT; t += kI2Threads) gpart[t >> 8][t & 255] = 0.0;
  float4 xr[2][2], yr[2][2];
  uint4 yq[2];  // raw BF16 / FP8 codes: eight k of one column

  const int64_t nchunks = (R + RT - 1) / RT;
  for (int64_t rc = 0; rc < nchunks; ++rc) {
    const int64_t r0 = rc * RT;
    f32x4 acc[RBW][4];
#pragma unroll
    for (int x = 0; x < RBW; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};

    auto gload = [&](int64_t k0) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = tid + kI2Threads * u;
        const int row = t & 255, kg = (t >> 8) * 8;
        const int64_t gk = k0 + kg;
        float v[8];
        if (u < XT) {
          // X row r0 + xrow, k xgk .. xgk + 7 (weighted for TRI)
          const int xrow = t % RT;
          const int64_t xgk = k0 + (t / RT) * 8;
          const int64_t gr = r0 + xrow;
          if (gr < R && xgk < m) {
            const float *src = X + gr * ldx + xgk;
            if (xgk + 7 < m) {
              const float4 p0 = *(const float4 *)src, p1 = *(const float4 *)(src + 4);
              v[0] = p0.x; v[1] = p0.y; v[2] = p0.z; v[3] = p0.w;
              v[4] = p1.x; v[5] = p1.y; v[6] = p1.z; v[7] = p1.w;
            } else {
#pragma unroll
              for (int e = 0; e < 8; ++e) v[e] = xgk + e < m ? src[e] : 0.f;
            }
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = 0.f;
          }
          xr[u][0] = make_float4(v[0], v[1], v[2], v[3]);
          xr[u][1] = make_float4(v[4], v[5], v[6], v[7]);
        }
        // A column j0 + row, k gk .. gk + 7
        const int64_t gj = j0 + row;
        if constexpr (DT == DT_F32) {
          if (gj < n && gk < m) {
            const float *src = a + gj * A.lda + gk;
            if (gk + 7 < m) {
              const float4 p0 = *(const float4 *)src, p1 = *(const float4 *)(src + 4);
              v[0] = p0.x; v[1] = p0.y; v[2] = p0.z; v[3] = p0.w;
              v[4] = p1.x; v[5] = p1.y; v[6] = p1.z; v[7] = p1.w;
            } else {
#pragma unroll
              for (int e = 0; e < 8; ++e) v[e] = gk + e < m ? src[e] : 0.f;
            }
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = 0.f;
          }
          yr[u][0] = make_float4(v[0], v[1], v[2], v[3]);
          yr[u][1] = make_float4(v[4], v[5], v[6], v[7]);
        } else {
          // eight codes (16 or 8 bytes, inside the column's lda); elements
          // past m are zeroed after decoding
          const char *src = (const char *)A.a + (gj * A.lda + gk) * ES;
          uint4 q = make_uint4(0u, 0u, 0u, 0u);
          if (gj < n && gk < m) {
            if constexpr (DT == DT_BF16) {
              q = *(const uint4 *)src;
            } else {
              const uint2 w = *(const uint2 *)src;
              q.x = w.x;
              q.y = w.y;
            }
          }
          yq[u] = q;
        }
      }
    };
    auto lstore = [&](int64_t k0) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = tid + kI2Threads * u;
        const int row = t & 255, kg = (t >> 8) * 8;
        const int xrow = t % RT, xkg = (t / RT) * 8;
#pragma unroll
        for (int op = 0; op < 2; ++op) {
          if (op == 0 && u >= XT) continue;
          const int off = op == 0 ? xrow * kX3RP + xkg : row * kX3RP + kg;
          float v[8];
          if (op == 0 || DT == DT_F32) {
            const float4 q0 = op == 0 ? xr[u][0] : yr[u][0], q1 = op == 0 ? xr[u][1] : yr[u][1];
            v[0] = q0.x; v[1] = q0.y; v[2] = q0.z; v[3] = q0.w;
            v[4] = q1.x; v[5] = q1.y; v[6] = q1.z; v[7] = q1.w;
          } else if constexpr (DT == DT_BF16) {
            const uint4 q = yq[u];
            v[0] = bf16_lo(q.x); v[1] = bf16_hi(q.x); v[2] = bf16_lo(q.y); v[3] = bf16_hi(q.y);
            v[4] = bf16_lo(q.z); v[5] = bf16_hi(q.z); v[6] = bf16_lo(q.w); v[7] = bf16_hi(q.w);
          } else {
            fp8x4_decode(yq[u].x, v);
            fp8x4_decode(yq[u].y, v + 4);
          }
          if (op == 1 && DT != DT_F32) {
            const int64_t gk = k0 + kg;
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (gk + e >= m) v[e] = 0.f;
          }
          if (TRI && op == 0 && k0 < r0 + RT) {
            // weights of the triangle: 1 above the diagonal, 1/2 on it, 0 below
            // (stages from k = r0 + 256 on lie wholly above it: weight 1)
            const int d0 = (int)(k0 + xkg - (r0 + xrow));
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] *= d0 + e > 0 ? 1.f : (d0 + e == 0 ? 0.5f : 0.f);
          }
          if (op == 0 || DT == DT_F32) {
            bf16x8 h, md, lo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              __bf16 xh, xm, xl;
              split3(v[e], xh, xm, xl);
              h[e] = xh;
              md[e] = xm;
              lo[e] = xl;
            }
            *(bf16x8 *)(&Ls[op][0][off]) = h;
            *(bf16x8 *)(&Ls[op][1][off]) = md;
            *(bf16x8 *)(&Ls[op][2][off]) = lo;
          } else {
            bf16x8 h;  // exact: BF16 and E4M3 values are bfloat16 numbers
#pragma unroll
            for (int e = 0; e < 8; ++e) h[e] = (__bf16)v[e];
            *(bf16x8 *)(&Ls[op][0][off]) = h;
          }
          if (op == 1 && rc == 0) {
            double g = gpart[t >> 8][t & 255];
#pragma unroll
            for (int e = 0; e < 8; ++e) g = fma((double)v[e], (double)v[e], g);
            gpart[t >> 8][t & 255] = g;  // this thread's own entry
          }
        }
      }
    };

    const int64_t kstart = TRI ? r0 : 0;
    if (kstart < m) gload(kstart);
    for (int64_t k0 = kstart; k0 < m; k0 += kX3BK) {
      __syncthreads();  // the previous stage's operands are consumed
      lstore(k0);
      __syncthreads();
      if (k0 + kX3BK < m) gload(k0 + kX3BK);
      bf16x8 b[4][YP];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int p = 0; p < YP; ++p)
          b[nb][p] = *(const bf16x8 *)(&Ls[1][p][(wc + 16 * nb + lr) * kX3RP + kq]);
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb) {
        bf16x8 av[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) av[p] = *(const bf16x8 *)(&Ls[0][p][(wr + 16 * rb + lr) * kX3RP + kq]);
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          f32x4 c = acc[rb][nb];
          if constexpr (YP == 3) {
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], b[nb][1], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[2], b[nb][0], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][2], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], b[nb][0], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][1], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][0], c, 0, 0, 0);
          } else {
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[2], b[nb][0], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], b[nb][0], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][0], c, 0, 0, 0);
          }
          acc[rb][nb] = c;
        }
      }
    }

    // epilogue of this row chunk (as in k_init256), summed into red
    double colacc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
      const int64_t i = r0 + wr + 16 * rb + 4 * (lane >> 4);
      if constexpr (TRI) {
        const int64_t ic = i < m ? i : 0;
        const float w0 = i < m ? 1.f : 0.f, w1 = i + 1 < m ? 1.f : 0.f;
        const float w2 = i + 2 < m ? 1.f : 0.f, w3 = i + 3 < m ? 1.f : 0.f;
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const int64_t j = j0 + wc + 16 * nb + lr;
          const float wj = j < n ? 1.f : 0.f;
          // one load in flight at a time: hoisting all 32 would spill the tile
          __builtin_amdgcn_sched_barrier(0);
          const float4 av4 = load4<DT>(A.a, (j < n ? j : 0) * A.lda + ic);
          const float p = acc[rb][nb][0] * (av4.x * w0) + acc[rb][nb][1] * (av4.y * w1) +
                          acc[rb][nb][2] * (av4.z * w2) + acc[rb][nb][3] * (av4.w * w3);
          colacc[nb] += (double)(p * wj);
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          double sq = 0.0;
#pragma unroll
          for (int v = 0; v < 4; ++v) sq += (double)acc[rb][nb][v] * (double)acc[rb][nb][v];
          colacc[nb] += sq;
        }
      }
    }
    // sum over the 4 lane groups; one writer per (row-wave, column): fixed order
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      double sv = colacc[nb];
      sv += __shfl_xor(sv, 16, 64);
      sv += __shfl_xor(sv, 32, 64);
      if (lane < 16) red[wave >> 2][wc + 16 * nb + lane] += sv;
    }
  }

  __syncthreads();
  if (tid < NT) {
    const int64_t j = j0 + tid;
    if (j < n) {
      const double fv = red[0][tid] + red[1][tid];
      const double g = ((gpart[0][tid] + gpart[1][tid]) + gpart[2][tid]) + gpart[3][tid];
      const double sc = col_scale(A, j);
      const double f = (TRI ? 2.0 : 1.0) * sc * sc * fv;
      const double gsc = sc * sc * g;
      f0[j] = f;
      g0[j] = gsc;
      mask0[j] = (gsc > 0.0 && isfinite(gsc) && isfinite(f)) ? 0 : 2;
    }
  }
}

// ---------------------------------------------------------------------------
// MN-major operand from A: rows i0..i0+127 of columns k0..k0+BKT-1 (decoded,
// FP8 columns scaled), staged through registers into Ts[k * MP + i].
template <int DT, int BKT>
struct MnTileA {
  static constexpr int EPC = EInfo<DT>::epc, ES = EInfo<DT>::esize;
  static constexpr int CPK = 128 / EPC;        // 16-byte chunks per k
  static constexpr int CH = BKT * CPK;         // chunks per stage
  static constexpr int PT = (CH + 255) / 256;  // chunks per thread
  uint4 raw[PT];
  float sc[PT];

  __device__ __forceinline__ void load(const AView &A, int64_t i0, int64_t k0, int64_t kend,
                                       int tid) {
    const char *abase = (const char *)A.a;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int q = tid + 256 * u;
      const int kk = q / CPK, ii = (q % CPK) * EPC;
      const bool ok = q < CH && (k0 + kk) < kend && (i0 + ii) < A.m;
      raw[u] = ok ? *(const uint4 *)(abase + ((k0 + kk) * A.lda + i0 + ii) * ES)
                  : make_uint4(0u, 0u, 0u, 0u);
      if constexpr (DT == DT_FP8) sc[u] = ok ? A.scale[k0 + kk] : 0.f;
    }
  }
  __device__ __forceinline__ void store(float *Ts, const AView &A, int64_t i0, int tid) const {
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int q = tid + 256 * u;
      if (q >= CH) continue;
      const int kk = q / CPK, ii = (q % CPK) * EPC;
      float v[EPC];
      decode16<DT>(raw[u], v);
#pragma unroll
      for (int e = 0; e < EPC; ++e) {
        if constexpr (DT == DT_FP8) v[e] *= sc[u];
        if (i0 + ii + e >= A.m) v[e] = 0.f;
      }
#pragma unroll
      for (int e = 0; e < EPC; e += 4)
        *(float4 *)(Ts + kk * MP + ii + e) = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
    }
  }
};

// Store a wave's 64 x 64 MN-major accumulator block: rows i0.. (contiguous in
// P), columns j0.. (stride ldp), rows < mrow and columns < ncol.
__device__ __forceinline__ void store_block_mn(float *P, int64_t ldp, int64_t i0, int64_t j0,
                                               int64_t mrow, int64_t ncol, int lane,
                                               const f32x4 (&acc)[4][4]) {
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int64_t j = j0 + 4 * (lane & 15) + nb;
    if (j >= ncol) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + 16 * (lane >> 4) + 4 * v;
      const float4 val = make_float4(acc[0][nb][v], acc[1][nb][v], acc[2][nb][v], acc[3][nb][v]);
      float *dst = P + j * ldp + i;
      if (i + 3 < mrow) {
        *(float4 *)dst = val;
      } else {
        if (i < mrow) dst[0] = val.x;
        if (i + 1 < mrow) dst[1] = val.y;
        if (i + 2 < mrow) dst[2] = val.z;
      }
    }
  }
}

// 128 x 128 upper tiles of C = A A^T, 4 waves in a 2 x 2 arrangement of 64 x 64.
// DB: two LDS buffers, one barrier per stage (the next stage's global loads
// are in flight while this stage multiplies, then land in the other buffer).
template <int DT, int BKT, bool DB>
__global__ __launch_bounds__(256) void k_gram(AView A, float *__restrict__ P, int64_t ldp,
                                              int ntile, int64_t kchunk) {
  constexpr int NBUF = DB ? 2 : 1;
  __shared__ __align__(16) float Xs[NBUF][BKT * MP];
  __shared__ __align__(16) float Ys[NBUF][BKT * MP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m = A.m, n = A.n;
  // tile id -> (bi, bj), bi <= bj
  const int64_t tile = blockIdx.x % ntile, split = blockIdx.x / ntile;
  int64_t bj = 0;
  while ((bj + 1) * (bj + 2) / 2 <= tile) ++bj;
  const int64_t bi = tile - bj * (bj + 1) / 2;
  const int64_t i0 = bi * 128, j0 = bj * 128;
  const int64_t kb = split * kchunk;
  const int64_t ke = (kb + kchunk) < n ? (kb + kchunk) : n;
  float *Pout = P + split * ldp * m;

  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  MnTileA<DT, BKT> xt, yt;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  if (kb < ke) {
    xt.load(A, i0, kb, ke, tid);
    yt.load(A, j0, kb, ke, tid);
  }
  if constexpr (DB) {
    if (kb < ke) {
      xt.store(Xs[0], A, i0, tid);
      yt.store(Ys[0], A, j0, tid);
    }
    __syncthreads();
    int cur = 0;
    for (int64_t k0 = kb; k0 < ke; k0 += BKT) {
      const bool more = k0 + BKT < ke;
      if (more) {
        xt.load(A, i0, k0 + BKT, ke, tid);
        yt.load(A, j0, k0 + BKT, ke, tid);
      }
      mma_stage_mn<BKT>(Xs[cur], wr, Ys[cur], wc, lane, acc);
      if (more) {
        xt.store(Xs[cur ^ 1], A, i0, tid);
        yt.store(Ys[cur ^ 1], A, j0, tid);
      }
      __syncthreads();
      cur ^= 1;
    }
  } else {
    for (int64_t k0 = kb; k0 < ke; k0 += BKT) {
      __syncthreads();
      xt.store(Xs[0], A, i0, tid);
      yt.store(Ys[0], A, j0, tid);
      __syncthreads();
      if (k0 + BKT < ke) {
        xt.load(A, i0, k0 + BKT, ke, tid);
        yt.load(A, j0, k0 + BKT, ke, tid);
      }
      mma_stage_mn<BKT>(Xs[0], wr, Ys[0], wc, lane, acc);
    }
  }
  store_block_mn(Pout, ldp, i0 + wr, j0 + wc, m, m, lane, acc);
}

// ---------------------------------------------------------------------------
// Large-tile MN-major product P = X Y^T over a k range, 256 x 256 per
// workgroup: 8 waves (2 along the rows x 4 along the columns) of 128 x 64,
// 8 x 4 instruction blocks each, two waves per SIMD.  X is always A (rows
// i0.., columns of A as k); Y is A (Gram) or Omega (projection, row-major
// n x r).  Per 4-k step a lane reads 3 x 16 B of operands and issues 32
// MFMAs.  Tile row of block rb, instruction row rho: 4*rho + rb (rb < 4) or
// 64 + 4*rho + (rb - 4) within the wave's 128 rows; column of block nb,
// instruction column c: 4*c + nb within the wave's 64 columns.
constexpr int MP2 = 260;  // LDS pitch (256 rows + pad) of the large tiles
constexpr int kG2Threads = 512;

template <int DT, int BKT>
struct MnTile256 {
  static constexpr int EPC = EInfo<DT>::epc, ES = EInfo<DT>::esize;
  static constexpr int CPK = 256 / EPC;  // 16-byte chunks per k
  static constexpr int CH = BKT * CPK;   // chunks per stage
  static constexpr int PT = (CH + kG2Threads - 1) / kG2Threads;
  uint4 raw[PT];
  float sc[PT];

  __device__ __forceinline__ void load(const AView &A, int64_t i0, int64_t k0, int64_t kend,
                                       int tid) {
    const char *abase = (const char *)A.a;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int q = tid + kG2Threads * u;
      const int kk = q / CPK, ii = (q % CPK) * EPC;
      const bool ok = q < CH && (k0 + kk) < kend && (i0 + ii) < A.m;
      raw[u] = ok ? *(const uint4 *)(abase + ((k0 + kk) * A.lda + i0 + ii) * ES)
                  : make_uint4(0u, 0u, 0u, 0u);
      if constexpr (DT == DT_FP8) sc[u] = ok ? A.scale[k0 + kk] : 0.f;
    }
  }
  __device__ __forceinline__ void store(float *Ts, const AView &A, int64_t i0, int tid) const {
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int q = tid + kG2Threads * u;
      if (q >= CH) continue;
      const int kk = q / CPK, ii = (q % CPK) * EPC;
      float v[EPC];
      decode16<DT>(raw[u], v);
#pragma unroll
      for (int e = 0; e < EPC; ++e) {
        if constexpr (DT == DT_FP8) v[e] *= sc[u];
        if (i0 + ii + e >= A.m) v[e] = 0.f;
      }
#pragma unroll
      for (int e = 0; e < EPC; e += 4)
        *(float4 *)(Ts + kk * MP2 + ii + e) = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
    }
  }
};

// Omega rows k0.. (row-major n x r), columns j0..j0+255, into Ts[k * MP2 + j].
template <int BKT>
struct OmTile256 {
  static constexpr int PT = (BKT * 64 + kG2Threads - 1) / kG2Threads;  // float4 per thread
  float4 v[PT];
  __device__ __forceinline__ void load(const float *Om, int64_t r, int64_t j0, int64_t k0,
                                       int64_t kend, int tid) {
    const bool vec4 = (r % 4) == 0;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int q = tid + kG2Threads * u;
      const int kk = q >> 6, jj = (q & 63) * 4;
      const int64_t gk = k0 + kk, gj = j0 + jj;
      float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
      if (kk < BKT && gk < kend && gj < r) {
        const float *src = Om + gk * r + gj;
        if (vec4) {
          x = *(const float4 *)src;
        } else {
          x.x = src[0];
          if (gj + 1 < r) x.y = src[1];
          if (gj + 2 < r) x.z = src[2];
          if (gj + 3 < r) x.w = src[3];
        }
      }
      v[u] = x;
    }
  }
  __device__ __forceinline__ void store(float *Ts, int tid) const {
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int q = tid + kG2Threads * u;
      const int kk = q >> 6, jj = (q & 63) * 4;
      if (kk < BKT) *(float4 *)(Ts + kk * MP2 + jj) = v[u];
    }
  }
};

// Random sign Omega generated in place of the loaded one: the same tile,
// entries from sign_words (one Philox call per four entries).
template <int BKT>
struct OmGen256 {
  static constexpr int PT = (BKT * 64 + kG2Threads - 1) / kG2Threads;
  float4 v[PT];
  __device__ __forceinline__ void load(uint32_t k0s, uint32_t k1s, uint32_t thr, int64_t r,
                                       int64_t j0, int64_t k0, int64_t kend, int tid) {
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int q = tid + kG2Threads * u;
      const int kk = q >> 6, jj = (q & 63) * 4;
      const int64_t gk = k0 + kk, gj = j0 + jj;
      float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
      if (kk < BKT && gk < kend && gj < r) {
        const uint4 w = sign_words(gk, (uint32_t)(gj >> 2), k0s, k1s);
        x.x = sign_entry(w.x, thr);
        x.y = gj + 1 < r ? sign_entry(w.y, thr) : 0.f;
        x.z = gj + 2 < r ? sign_entry(w.z, thr) : 0.f;
        x.w = gj + 3 < r ? sign_entry(w.w, thr) : 0.f;
      }
      v[u] = x;
    }
  }
  __device__ __forceinline__ void store(float *Ts, int tid) const {
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int q = tid + kG2Threads * u;
      const int kk = q >> 6, jj = (q & 63) * 4;
      if (kk < BKT) *(float4 *)(Ts + kk * MP2 + jj) = v[u];
    }
  }
};

template <int BKT>
__device__ __forceinline__ void mma_stage_mn256(const float *Xs, int xr0, const float *Ys, int yc0,
                                                int lane, f32x4 (&acc)[8][4]) {
  const int r = lane & 15, g = lane >> 4;
  constexpr int NS = BKT / 4;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int k = 4 * s + g;
    const float4 x0 = *(const float4 *)(Xs + k * MP2 + xr0 + 4 * r);
    const float4 x1 = *(const float4 *)(Xs + k * MP2 + xr0 + 64 + 4 * r);
    const float4 y0 = *(const float4 *)(Ys + k * MP2 + yc0 + 4 * r);
    const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    const float yv[4] = {y0.x, y0.y, y0.z, y0.w};
#pragma unroll
    for (int rb = 0; rb < 8; ++rb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[rb][nb] = mfma4(xv[rb], yv[nb], acc[rb][nb]);
  }
  __builtin_amdgcn_iglp_opt(GCSS_IGLP);
}

// Store a wave's 128 x 64 block (rows i0.. contiguous in P, columns j0..
// with stride ldp), rows < mrow and columns < ncol; one column block at a
// time so few accumulators are copied out at once.
__device__ __forceinline__ void store_block_mn256(float *P, int64_t ldp, int64_t i0, int64_t j0,
                                                  int64_t mrow, int64_t ncol, int lane,
                                                  const f32x4 (&acc)[8][4]) {
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int64_t j = j0 + 4 * (lane & 15) + nb;
    if (j < ncol) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t i = i0 + 64 * h + 16 * (lane >> 4) + 4 * v;
          const float4 val = make_float4(acc[4 * h + 0][nb][v], acc[4 * h + 1][nb][v],
                                         acc[4 * h + 2][nb][v], acc[4 * h + 3][nb][v]);
          float *dst = P + j * ldp + i;
          if (i + 3 < mrow) {
            *(float4 *)dst = val;
          } else {
            if (i < mrow) dst[0] = val.x;
            if (i + 1 < mrow) dst[1] = val.y;
            if (i + 2 < mrow) dst[2] = val.z;
          }
        }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// MODE 0: upper 256-tiles of C = A A^T; 1: tiles of B = A Omega (Omega
// loaded); 2: tiles of B = A Omega with the random sign Omega generated from
// the key (gk0, gk1) and threshold gthr.
template <int DT, int BKT, int MODE>
__global__ __launch_bounds__(kG2Threads, 1) void k_gemm256(AView A, const float *__restrict__ Om,
                                                           int64_t r, float *__restrict__ P,
                                                           int64_t ldp, int ntm, int ntile,
                                                           int64_t kchunk, uint32_t gk0,
                                                           uint32_t gk1, uint32_t gthr) {
  constexpr bool PROJ = MODE != 0;
  __shared__ __align__(16) float Xs[2][BKT * MP2];
  __shared__ __align__(16) float Ys[2][BKT * MP2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m = A.m, n = A.n;
  const int64_t tile = blockIdx.x % ntile, split = blockIdx.x / ntile;
  int64_t i0, j0;
  if constexpr (PROJ) {
    i0 = (tile % ntm) * 256;
    j0 = (tile / ntm) * 256;
  } else {
    int64_t bj = 0;
    while ((bj + 1) * (bj + 2) / 2 <= tile) ++bj;
    i0 = (tile - bj * (bj + 1) / 2) * 256;
    j0 = bj * 256;
  }
  const int64_t ncol = PROJ ? r : m;
  const int64_t kb = split * kchunk;
  const int64_t ke = (kb + kchunk) < n ? (kb + kchunk) : n;
  float *Pout = P + split * ldp * ncol;

  f32x4 acc[8][4];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  MnTile256<DT, BKT> xt;
  typename std::conditional<
      MODE == 2, OmGen256<BKT>,
      typename std::conditional<PROJ, OmTile256<BKT>, MnTile256<DT, BKT>>::type>::type yt;
  auto yload = [&](int64_t k0) {
    if constexpr (MODE == 2)
      yt.load(gk0, gk1, gthr, r, j0, k0, ke, tid);
    else if constexpr (PROJ)
      yt.load(Om, r, j0, k0, ke, tid);
    else
      yt.load(A, j0, k0, ke, tid);
  };
  auto ystore = [&](float *Ts) {
    if constexpr (PROJ)
      yt.store(Ts, tid);
    else
      yt.store(Ts, A, j0, tid);
  };
  const int wr = (wave >> 2) * 128, wc = (wave & 3) * 64;
  if (kb < ke) {
    xt.load(A, i0, kb, ke, tid);
    yload(kb);
    xt.store(Xs[0], A, i0, tid);
    ystore(Ys[0]);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += BKT) {
    const bool more = k0 + BKT < ke;
    if (more) {
      xt.load(A, i0, k0 + BKT, ke, tid);
      yload(k0 + BKT);
    }
    mma_stage_mn256<BKT>(Xs[cur], wr, Ys[cur], wc, lane, acc);
    if (more) {
      xt.store(Xs[cur ^ 1], A, i0, tid);
      ystore(Ys[cur ^ 1]);
    }
    __syncthreads();
    cur ^= 1;
  }
  store_block_mn256(Pout, ldp, i0 + wr, j0 + wc, m, ncol, lane, acc);
}

// ---------------------------------------------------------------------------
// Gram matrix of binary32 A on the bfloat16 matrix cores.  Each element is
// split exactly into three bfloat16 parts, a = a_h + a_m + a_l (a_h the
// nearest bfloat16 to a, a_m the nearest to a - a_h, a_l the rest), and a
// product a b is formed from the six part products whose order is at most
// 2^-16 a b (h h, h m, m h, h l, l h, m m); the three dropped ones are below
// 2^-24 |a b|, under binary32 rounding.  The bfloat16 MFMA (16 x 16 x 32)
// runs 16 times the binary32 one, so six of them still take 3/8 of the time.
// Tiles as in k_gemm256 (256 x 256 per workgroup, eight waves of 128 x 64);
// each k-stage of 32 columns is split into planes once, on its way into LDS,
// with rows of 32 consecutive k per plane (one 16-byte read per lane and
// plane feeds an MFMA operand).

__global__ __launch_bounds__(kG2Threads, 1) void k_gram_x3(AView A, float *__restrict__ P,
                                                           int64_t ldp, int ntile,
                                                           int64_t kchunk) {
  // [operand 0 / 1][plane h, m, l][row][k]
  __shared__ __align__(16) __bf16 Ls[2][3][kX3Plane];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m = A.m, n = A.n;
  const int64_t tile = blockIdx.x % ntile, split = blockIdx.x / ntile;
  int64_t bj = 0;
  while ((bj + 1) * (bj + 2) / 2 <= tile) ++bj;
  const int64_t i0 = (tile - bj * (bj + 1) / 2) * 256, j0 = bj * 256;
  const int64_t kb = split * kchunk;
  const int64_t ke = (kb + kchunk) < n ? (kb + kchunk) : n;
  float *Pout = P + split * ldp * m;
  const float *a = (const float *)A.a;

  // load task of this thread: operand op, rows r0..r0+3, k k8..k8+7 of the stage
  const int op = tid >> 8, task = tid & 255;
  const int r0 = x3_task_row(task), k8 = x3_task_k(task);
  const int64_t row0 = (op == 0 ? i0 : j0) + r0;
  float4 reg[8];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t k = k0 + k8 + e;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (k < ke) {
        const float *src = a + k * A.lda + row0;
        if (row0 + 3 < m) {
          v = *(const float4 *)src;
        } else {
          if (row0 < m) v.x = src[0];
          if (row0 + 1 < m) v.y = src[1];
          if (row0 + 2 < m) v.z = src[2];
        }
      }
      reg[e] = v;
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      bf16x8 h, md, lo;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = rr == 0 ? reg[e].x : rr == 1 ? reg[e].y : rr == 2 ? reg[e].z : reg[e].w;
        __bf16 xh, xm, xl;
        split3(x, xh, xm, xl);
        h[e] = xh;
        md[e] = xm;
        lo[e] = xl;
      }
      const int off = (r0 + rr) * kX3RP + k8;
      *(bf16x8 *)(&Ls[op][0][off]) = h;
      *(bf16x8 *)(&Ls[op][1][off]) = md;
      *(bf16x8 *)(&Ls[op][2][off]) = lo;
    }
  };

  f32x4 acc[8][4];
#pragma unroll
  for (int x = 0; x < 8; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int wr = (wave >> 2) * 128, wc = (wave & 3) * 64;
  const int lr = lane & 15, kq = (lane >> 4) * 8;

  if (kb < ke) gload(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kX3BK) {
    __syncthreads();  // the previous stage's operands are consumed
    lstore();
    __syncthreads();
    if (k0 + kX3BK < ke) gload(k0 + kX3BK);
    // B operands of this wave's four column blocks (rows of operand 1)
    bf16x8 b[4][3];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int p = 0; p < 3; ++p)
        b[nb][p] = *(const bf16x8 *)(&Ls[1][p][(wc + 16 * nb + lr) * kX3RP + kq]);
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) {
      bf16x8 av[3];
#pragma unroll
      for (int p = 0; p < 3; ++p) av[p] = *(const bf16x8 *)(&Ls[0][p][(wr + 16 * rb + lr) * kX3RP + kq]);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        f32x4 c = acc[rb][nb];
        // smallest terms first
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], b[nb][1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[2], b[nb][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], b[nb][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][0], c, 0, 0, 0);
        acc[rb][nb] = c;
      }
    }
  }
  // D of block (rb, nb): lane holds column wc + 16 nb + (lane & 15), rows
  // wr + 16 rb + 4 (lane >> 4) + v
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int64_t j = j0 + wc + 16 * nb + lr;
    if (j >= m) continue;
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) {
      const int64_t i = i0 + wr + 16 * rb + 4 * (lane >> 4);
      float *dst = Pout + j * ldp + i;
      const f32x4 v = acc[rb][nb];
      if (i + 3 < m) {
        *(float4 *)dst = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        if (i < m) dst[0] = v[0];
        if (i + 1 < m) dst[1] = v[1];
        if (i + 2 < m) dst[2] = v[2];
      }
    }
  }
}

// B = A Omega on the bfloat16 matrix cores: the tiles of k_gemm256's
// projection (MODE 1), with Omega (binary32; an FP8 column scale of A is
// folded into Omega's row) split into three bfloat16 parts and A into three
// (binary32) or one (BF16 and FP8 codes are exact): six or three part
// products per product, as in k_gram_x3.  Both operands are transposed on
// their way into LDS (a thread loads four rows of A or four columns of
// Omega for eight consecutive k) so that each plane row holds 32
// consecutive k.  Needs m and r to be multiples of 4.
//
// TN is the tile's width in columns of Omega: 256 (eight waves of 128 rows x
// 64 columns), or 128 for narrow targets (eight waves of 64 x 64, so every
// wave multiplies; the Omega loads of waves 6-7 are then empty).
template <int DT, int TN>
__global__ __launch_bounds__(kG2Threads, 1) void k_proj_x3(AView A, const float *__restrict__ Om,
                                                           int64_t r, float *__restrict__ P,
                                                           int64_t ldp, int ntm, int ntile,
                                                           int64_t kchunk) {
  constexpr int AP = DT == DT_F32 ? 3 : 1;
  constexpr int ES = EInfo<DT>::esize;
  __shared__ __align__(16) __bf16 La[AP][kX3Plane];
  __shared__ __align__(16) __bf16 Lo[3][kX3Plane];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m = A.m, n = A.n;
  const int64_t tile = blockIdx.x % ntile, split = blockIdx.x / ntile;
  const int64_t i0 = (tile % ntm) * 256, j0 = (tile / ntm) * TN;
  const int64_t kb = split * kchunk;
  const int64_t ke = (kb + kchunk) < n ? (kb + kchunk) : n;
  float *Pout = P + split * ldp * r;
  const char *abase = (const char *)A.a;

  // load task: op 0 -> rows i0 + q0 .. +3 of A, op 1 -> columns j0 + q0 .. +3
  // of Omega, for k = k0 + k8 .. k0 + k8 + 7 (op is the same in a wave:
  // waves 0-3 load A, waves 4-7 Omega)
  const int op = __builtin_amdgcn_readfirstlane(tid >> 8), task = tid & 255;
  const int q0 = x3_task_row(task), k8 = x3_task_k(task);

  // a wave's block of the tile: RBW blocks of 16 rows x 4 blocks of 16 columns
  constexpr int CW = TN / 64;          // waves across the tile's columns
  constexpr int RBW = 8 * CW / 4;      // 16-row blocks per wave (8 or 4)
  f32x4 acc[RBW][4];
#pragma unroll
  for (int x = 0; x < RBW; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int wr = (wave / CW) * (16 * RBW), wc = (wave % CW) * 64;
  const int lr = lane & 15, kq = (lane >> 4) * 8;

  // the matrix products of one stage from the LDS planes
  auto mma = [&]() {
    bf16x8 b[4][3];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int p = 0; p < 3; ++p) b[nb][p] = *(const bf16x8 *)(&Lo[p][(wc + 16 * nb + lr) * kX3RP + kq]);
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
      bf16x8 av[AP];
#pragma unroll
      for (int p = 0; p < AP; ++p) av[p] = *(const bf16x8 *)(&La[p][(wr + 16 * rb + lr) * kX3RP + kq]);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        f32x4 c = acc[rb][nb];
        if constexpr (AP == 3) {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], b[nb][1], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[2], b[nb][0], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][2], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], b[nb][0], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][1], c, 0, 0, 0);
        } else {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][2], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][1], c, 0, 0, 0);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], b[nb][0], c, 0, 0, 0);
        acc[rb][nb] = c;
      }
    }
  };

  // The k loop, one instance per load role (a wave runs its role's): the
  // registers a stage is loaded into then belong to one role only, so the
  // compiler neither merges nor copies them, and a stage's loads stay in
  // flight until the LDS store that consumes them.  Both instances pass the
  // same barriers.
  auto run = [&](auto role) {
    constexpr int OP = decltype(role)::value;
    // 32-bit words per loaded element: four binary32 values, or four BF16 /
    // E4M3 codes of A
    constexpr int LW = (OP == 1 || DT == DT_F32) ? 4 : (DT == DT_BF16 ? 2 : 1);
    // the loads of a stage are kept raw (codes of A as bits, Omega and the
    // FP8 column scales unmultiplied) and decoded only when the stage goes to
    // LDS, so the next stage's loads stay in flight through this stage's
    // matrix products instead of being waited for where they are issued
    uint32_t reg[8][LW];
    float scl[8];
    uint32_t okm = 0;  // bit e: element e of the stage is inside the chunk and the matrix
    // Addresses: a base shared by the wave (the stage's first k) plus a 32-bit
    // lane offset formed just before each load (the host keeps 32 columns of
    // A and 32 rows of Omega within 2^31 bytes), so no 64-bit address per
    // element stays live across the matrix products.  Rows or columns past
    // the edge and k past the chunk load a clamped in-range element, zeroed
    // when the stage goes to LDS (m and r are multiples of 4: four rows or
    // columns are in or out together).
    const int64_t qn = OP == 0 ? m : r;
    const int64_t qg = (OP == 0 ? i0 : j0) + q0;
    const bool inq = qg < qn;
    const uint32_t qoff = (uint32_t)(inq ? qg : qn - 4);
    // (TN = 128: the Omega tasks of columns 128 .. 255, waves 6-7, have no work)
    const bool idle = OP == 1 && q0 >= TN;
    const uint32_t colb = OP == 0 ? (uint32_t)(A.lda * ES) : (uint32_t)(r * 4);  // bytes per k
    const uint32_t qb = qoff * (OP == 0 ? (uint32_t)ES : 4u);
    const char *src0 = OP == 0 ? abase : (const char *)Om;
    auto gload = [&](int64_t k0) {
      const int64_t kleft = ke - k0;  // > 0
      const char *base = src0 + k0 * (int64_t)colb;
      okm = 0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int kk = k8 + e;
        const int kc = kk < kleft ? kk : (int)kleft - 1;
        const char *src = base + ((uint32_t)kc * colb + qb);
        if constexpr (LW == 4) {
          const uint4 v = *(const uint4 *)src;
          reg[e][0] = v.x;
          reg[e][1] = v.y;
          reg[e][2] = v.z;
          reg[e][3] = v.w;
        } else if constexpr (LW == 2) {
          const uint2 v = *(const uint2 *)src;
          reg[e][0] = v.x;
          reg[e][1] = v.y;
        } else {
          reg[e][0] = *(const uint32_t *)src;
        }
        if constexpr (OP == 1 && DT == DT_FP8) scl[e] = A.scale[k0 + kc];
        okm |= (uint32_t)(inq && kk < kleft) << e;
      }
    };
    // element (row / column q0 + rr, k k8 + e) of the stage as a binary32 value
    auto elem = [&](int e, int rr) -> float {
      if constexpr (OP == 0 && DT == DT_BF16) {
        const uint32_t w = reg[e][rr >> 1];
        return (rr & 1) ? bf16_hi(w) : bf16_lo(w);
      } else if constexpr (OP == 0 && DT == DT_FP8) {
        float d[4];
        fp8x4_decode(reg[e][0], d);
        return d[rr];
      } else {
        const float x = __uint_as_float(reg[e][rr]);
        if constexpr (OP == 1 && DT == DT_FP8) return x * scl[e];
        return x;
      }
    };
    auto lstore = [&]() {
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = (okm >> e) & 1 ? elem(e, rr) : 0.f;
        const int off = (q0 + rr) * kX3RP + k8;
        if constexpr (OP == 1 || AP == 3) {
          bf16x8 h, md, lo;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 xh, xm, xl;
            split3(x[e], xh, xm, xl);
            h[e] = xh;
            md[e] = xm;
            lo[e] = xl;
          }
          __bf16 *base = OP == 0 ? &La[0][0] : &Lo[0][0];
          *(bf16x8 *)(base + off) = h;
          *(bf16x8 *)(base + kX3Plane + off) = md;
          *(bf16x8 *)(base + 2 * kX3Plane + off) = lo;
        } else {
          bf16x8 h;  // BF16 and E4M3 values are bfloat16 numbers
#pragma unroll
          for (int e = 0; e < 8; ++e) h[e] = (__bf16)x[e];
          *(bf16x8 *)(&La[0][off]) = h;
        }
      }
    };

    if (kb < ke && !idle) gload(kb);
    for (int64_t k0 = kb; k0 < ke; k0 += kX3BK) {
      __syncthreads();  // the previous stage's operands are consumed
      if (!idle) lstore();
      __syncthreads();
      if (k0 + kX3BK < ke && !idle) gload(k0 + kX3BK);
      mma();
    }
  };
  if (op == 0)
    run(std::integral_constant<int, 0>{});
  else
    run(std::integral_constant<int, 1>{});
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int64_t j = j0 + wc + 16 * nb + lr;
    if (j >= r) continue;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
      const int64_t i = i0 + wr + 16 * rb + 4 * (lane >> 4);
      float *dst = Pout + j * ldp + i;
      const f32x4 v = acc[rb][nb];
      if (i + 3 < m) {
        *(float4 *)dst = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        if (i < m) dst[0] = v[0];
        if (i + 1 < m) dst[1] = v[1];
        if (i + 2 < m) dst[2] = v[2];
      }
    }
  }
}

// C = sum_s P_s over the upper triangle, mirrored (exact symmetry).  One
// workgroup per 64 x 64 tile (bi <= bj) of the upper part: partial sums are
// read along the contiguous rows, the tile is written in place and, through
// LDS, transposed into the lower part, so every access is coalesced.
__global__ __launch_bounds__(256) void k_gram_reduce(const float *__restrict__ P, int64_t ldp,
                                                     int64_t m, int nsplit,
                                                     float *__restrict__ C, int64_t ldc) {
  __shared__ float T[64][65];
  int64_t bj = 0;
  const int64_t tile = blockIdx.x;
  while ((bj + 1) * (bj + 2) / 2 <= tile) ++bj;
  const int64_t bi = tile - bj * (bj + 1) / 2;
  const int rr = threadIdx.x & 63, c0 = threadIdx.x >> 6;
  const int64_t i = bi * 64 + rr;
  for (int x = c0; x < 64; x += 4) {
    const int64_t j = bj * 64 + x;
    float v = 0.f;
    if (i < m && j < m && (bi < bj || i <= j)) {
      for (int sp = 0; sp < nsplit; ++sp) v += P[(int64_t)sp * ldp * m + j * ldp + i];
      C[j * ldc + i] = v;
    }
    T[rr][x] = v;
  }
  __syncthreads();
  // lower part: C[j][i] = C[i][j] for the tile's (i, j), i < j
  for (int x = c0; x < 64; x += 4) {
    const int64_t ic = bi * 64 + x;   // column of the lower element
    const int64_t jr = bj * 64 + rr;  // its row
    if (ic < m && jr < m && ic < jr) C[ic * ldc + jr] = T[x][rr];
  }
}

// B = A Omega: left operand A (MN-major), right operand Omega[k][j]
// (row-major n x r, MN-major as stored).
template <int DT, int BKT, bool DB>
__global__ __launch_bounds__(256) void k_project(AView A, const float *__restrict__ Om,
                                                 int64_t r, float *__restrict__ P, int64_t ldp,
                                                 int ntm, int ntn, int64_t kchunk) {
  constexpr int YPT = BKT * 32 / 256;  // Omega float4 per thread per stage
  constexpr int NBUF = DB ? 2 : 1;
  __shared__ __align__(16) float Xs[NBUF][BKT * MP];
  __shared__ __align__(16) float Ys[NBUF][BKT * MP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = A.n;
  const int ntile = ntm * ntn;
  const int64_t tile = blockIdx.x % ntile, split = blockIdx.x / ntile;
  const int64_t i0 = (tile % ntm) * 128, j0 = (tile / ntm) * 128;
  const int64_t kb = split * kchunk;
  const int64_t ke = (kb + kchunk) < n ? (kb + kchunk) : n;
  float *Pout = P + split * ldp * r;
  const bool vec4 = (r % 4) == 0;

  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  MnTileA<DT, BKT> xt;
  float4 yv[YPT];
  auto yload = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < YPT; ++u) {
      const int q = tid + 256 * u;
      const int kk = q >> 5, jj = (q & 31) * 4;
      const int64_t gk = k0 + kk, gj = j0 + jj;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gk < ke && gj < r) {
        const float *src = Om + gk * r + gj;
        if (vec4) {
          v = *(const float4 *)src;
        } else {
          v.x = src[0];
          if (gj + 1 < r) v.y = src[1];
          if (gj + 2 < r) v.z = src[2];
          if (gj + 3 < r) v.w = src[3];
        }
      }
      yv[u] = v;
    }
  };
  auto ystore = [&](float *Yb) {
#pragma unroll
    for (int u = 0; u < YPT; ++u) {
      const int q = tid + 256 * u;
      const int kk = q >> 5, jj = (q & 31) * 4;
      *(float4 *)(Yb + kk * MP + jj) = yv[u];
    }
  };
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  if (kb < ke) {
    xt.load(A, i0, kb, ke, tid);
    yload(kb);
  }
  if constexpr (DB) {
    if (kb < ke) {
      xt.store(Xs[0], A, i0, tid);
      ystore(Ys[0]);
    }
    __syncthreads();
    int cur = 0;
    for (int64_t k0 = kb; k0 < ke; k0 += BKT) {
      const bool more = k0 + BKT < ke;
      if (more) {
        xt.load(A, i0, k0 + BKT, ke, tid);
        yload(k0 + BKT);
      }
      mma_stage_mn<BKT>(Xs[cur], wr, Ys[cur], wc, lane, acc);
      if (more) {
        xt.store(Xs[cur ^ 1], A, i0, tid);
        ystore(Ys[cur ^ 1]);
      }
      __syncthreads();
      cur ^= 1;
    }
  } else {
    for (int64_t k0 = kb; k0 < ke; k0 += BKT) {
      __syncthreads();
      xt.store(Xs[0], A, i0, tid);
      ystore(Ys[0]);
      __syncthreads();
      if (k0 + BKT < ke) {
        xt.load(A, i0, k0 + BKT, ke, tid);
        yload(k0 + BKT);
      }
      mma_stage_mn<BKT>(Xs[0], wr, Ys[0], wc, lane, acc);
    }
  }
  store_block_mn(Pout, ldp, i0 + wr, j0 + wc, A.m, r, lane, acc);
}

__global__ void k_proj_reduce(const float *__restrict__ P, int64_t ldp, int64_t m, int64_t r,
                              int nsplit, float *__restrict__ B, int64_t ldb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * r) return;
  const int64_t j = e / m, i = e % m;
  float s = 0.f;
  for (int x = 0; x < nsplit; ++x) s += P[x * ldp * r + j * ldp + i];
  B[j * ldb + i] = s;
}

// ---------------------------------------------------------------------------
// Exact decrements for the Gram target: quad_s = || A^T q_s ||^2 for the
// basis vectors q_s (FP64), as row sums of squares of W = Q^T A.  FP64
// matrix cores (v_mfma_f64_16x16x4_f64: operands laid out as in the FP32
// form, but lane l, register v of the result holds row (l/16) + 4v);
// A is decoded to FP64 on the way into LDS, so every product is exact and
// only FP64 accumulation rounds.  Each workgroup owns 64 columns of A and
// writes one partial per basis vector; a fixed-order reduce follows.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int PIT64 = 18;  // LDS row pitch in doubles (16 k values + pad)

__device__ __forceinline__ f64x4 mfma4d(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int DT, int RB>
__global__ __launch_bounds__(256) void k_qta_rowsq(const double *__restrict__ Q, int64_t ldq,
                                                   int kmax, const DevState *st, AView A,
                                                   double *__restrict__ part, int kpad) {
  constexpr int NB = 4, NT = 64, RT = 64 * RB;
  constexpr int ES = EInfo<DT>::esize, EPC = EInfo<DT>::epc, CPC = ES;
  __shared__ __align__(16) double Xs[RT * PIT64];
  __shared__ __align__(16) double Ys[NT * PIT64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m = A.m, n = A.n;
  int nrow = st ? st->t : kmax;
  if (nrow > kmax) nrow = kmax;
  const int64_t j0 = (int64_t)blockIdx.x * NT;
  const char *abase = (const char *)A.a;
  const int64_t colb = A.lda * ES;
  const int ycol = tid / CPC, ych = tid % CPC;
  const bool yact = tid < NT * CPC;
  const bool ycolv = yact && (j0 + ycol) < n;
  const int64_t ksteps = (m + BK - 1) / BK;
  double jscale[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t j = j0 + 16 * nb + (lane & 15);
    jscale[nb] = j < n ? col_scale(A, j) : 0.0;
  }

  for (int r0 = 0; r0 < nrow; r0 += RT) {
    f64x4 acc[RB][NB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = f64x4{0.0, 0.0, 0.0, 0.0};
    double2 xr[2 * RB];
    uint4 yr;
    auto gload = [&](int64_t k0) {
#pragma unroll
      for (int u = 0; u < 2 * RB; ++u) {
        const int q = tid + 256 * u;
        const int row = q >> 3, c = (q & 7) * 2;
        const int64_t gr = r0 + row, gk = k0 + c;
        double2 v = make_double2(0.0, 0.0);
        if (gr < nrow && gk < m) {
          v = *(const double2 *)(Q + gr * ldq + gk);
          if (gk + 1 >= m) v.y = 0.0;
        }
        xr[u] = v;
      }
      const int64_t gk = k0 + ych * EPC;
      if (ycolv && gk < m)
        yr = *(const uint4 *)(abase + (j0 + ycol) * colb + gk * ES);
      else
        yr = make_uint4(0u, 0u, 0u, 0u);
    };
    auto sstore = [&](int64_t k0) {
#pragma unroll
      for (int u = 0; u < 2 * RB; ++u) {
        const int q = tid + 256 * u;
        const int row = q >> 3, c = (q & 7) * 2;
        *(double2 *)(Xs + row * PIT64 + c) = xr[u];
      }
      if (yact) {
        float v[EPC];
        decode16<DT>(yr, v);
        const int64_t gk = k0 + ych * EPC;
#pragma unroll
        for (int e = 0; e < EPC; e += 2)
          *(double2 *)(Ys + ycol * PIT64 + ych * EPC + e) =
              make_double2(gk + e < m ? (double)v[e] : 0.0, gk + e + 1 < m ? (double)v[e + 1] : 0.0);
      }
    };
    gload(0);
    for (int64_t ks = 0; ks < ksteps; ++ks) {
      __syncthreads();
      sstore(ks * BK);
      __syncthreads();
      if (ks + 1 < ksteps) gload((ks + 1) * BK);
      const int r = lane & 15, kq = (lane >> 4) * 4;
      double xa[RB][4], yb[NB][4];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const double *px = Xs + (wave * 16 * RB + 16 * rb + r) * PIT64 + kq;
        const double2 a0 = *(const double2 *)px, a1 = *(const double2 *)(px + 2);
        xa[rb][0] = a0.x; xa[rb][1] = a0.y; xa[rb][2] = a1.x; xa[rb][3] = a1.y;
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const double *py = Ys + (16 * nb + r) * PIT64 + kq;
        const double2 b0 = *(const double2 *)py, b1 = *(const double2 *)(py + 2);
        yb[nb][0] = b0.x; yb[nb][1] = b0.y; yb[nb][2] = b1.x; yb[nb][3] = b1.y;
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[rb][nb] = mfma4d(xa[rb][s], yb[nb][s], acc[rb][nb]);
    }
    // row sums of squares over this workgroup's 64 columns
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double sq = 0.0;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const double d = acc[rb][nb][v] * jscale[nb];
          sq = fma(d, d, sq);
        }
        sq += __shfl_xor(sq, 1, 64);
        sq += __shfl_xor(sq, 2, 64);
        sq += __shfl_xor(sq, 4, 64);
        sq += __shfl_xor(sq, 8, 64);
        // v_mfma_f64_16x16x4_f64: lane l, register v holds D[(l/16) + 4v][l%16]
        const int row = r0 + wave * 16 * RB + 16 * rb + (lane >> 4) + 4 * v;
        if ((lane & 15) == 0 && row < nrow) part[(int64_t)blockIdx.x * kpad + row] = sq;
      }
  }
}

// quad[s] = sum over workgroups of part[wg][s], fixed order.
__global__ void k_qta_reduce(const double *__restrict__ part, int nwg, int kpad, int kmax,
                             const DevState *st, double *__restrict__ quad) {
  int nrow = st ? st->t : kmax;
  if (nrow > kmax) nrow = kmax;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nrow) return;
  double acc = 0.0;
  for (int w = 0; w < nwg; ++w) acc += part[(int64_t)w * kpad + s];
  quad[s] = acc;
}

// obj[s+1] = F0 - sum_{x<=s} quad[x] for s < t (the objective from exact decrements)
__global__ void k_obj_from_quad(const double *F0, const double *quad, const DevState *st,
                                double *obj) {
  if (threadIdx.x != 0) return;
  const int t = st->t;
  double F = *F0;
  for (int s = 0; s < t; ++s) {
    F -= quad[s];
    obj[s + 1] = F;
  }
}

size_t qta_scratch_bytes(int64_t n, int kmax) {
  const int64_t nwg = (n + 63) / 64;
  return (size_t)(nwg * kmax + kmax + 64) * sizeof(double);
}

hipError_t launch_qta(const double *Q, int64_t ldq, int kmax, const DevState *st,
                      const AView &A, double *scratch, double *quad, hipStream_t s) {
  const int nwg = (int)((A.n + 63) / 64);
  double *part = scratch;
  switch (A.dtype) {
    case DT_F32:
      hipLaunchKernelGGL((k_qta_rowsq<DT_F32, 2>), dim3(nwg), dim3(256), 0, s, Q, ldq, kmax, st, A, part, kmax);
      break;
    case DT_BF16:
      hipLaunchKernelGGL((k_qta_rowsq<DT_BF16, 2>), dim3(nwg), dim3(256), 0, s, Q, ldq, kmax, st, A, part, kmax);
      break;
    case DT_FP8:
      hipLaunchKernelGGL((k_qta_rowsq<DT_FP8, 2>), dim3(nwg), dim3(256), 0, s, Q, ldq, kmax, st, A, part, kmax);
      break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_qta_reduce, dim3((unsigned)((kmax + 255) / 256)), dim3(256), 0, s, part, nwg,
                     kmax, kmax, st, quad);
  return hipGetLastError();
}

hipError_t launch_obj_from_quad(const double *F0, const double *quad, const DevState *st,
                                double *obj, hipStream_t s) {
  hipLaunchKernelGGL(k_obj_from_quad, dim3(1), dim3(64), 0, s, F0, quad, st, obj);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k values per LDS stage of the FP32 contractions: 16 (measured best for
// every kernel with double-buffered stages and operand reads issued one step
// ahead); the environment variable GCSS_MFMA_BK=32 selects the deeper stage.
static int mfma_bk(bool /*tri*/) {
  static const int bk = [] {
    const char *e = std::getenv("GCSS_MFMA_BK");
    return (e && std::atoi(e) == 32) ? 32 : 16;
  }();
  return bk;
}
// Double-buffered LDS stages (default); GCSS_MFMA_DB=0 selects one buffer.
static bool mfma_db() {
  static const bool db = [] {
    const char *e = std::getenv("GCSS_MFMA_DB");
    return !(e && std::atoi(e) == 0);
  }();
  return db;
}
constexpr int KC_ALIGN = 32;  // split-K chunks are multiples of every stage depth

template <int DT, int RB, int BKT, bool TRI>
static hipError_t init_t(const float *X, int64_t ldx, int64_t R, const AView &A, double *f0,
                         double *g0, uint8_t *mask0, hipStream_t s) {
  constexpr int NB = 4;
  // two buffers only where they fit the 160 KiB of LDS
  constexpr bool kFitsDB = 2 * (64 * RB + 16 * NB) * (BKT + 4) * 4 + 8 * 1024 <= 160 * 1024;
  const unsigned grid = (unsigned)((A.n + 16 * NB - 1) / (16 * NB));
  if constexpr (kFitsDB) {
    if (mfma_db()) {
      hipLaunchKernelGGL((k_init<DT, RB, NB, BKT, TRI, true>), dim3(grid), dim3(256), 0, s, X,
                         ldx, R, A, f0, g0, mask0);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_init<DT, RB, NB, BKT, TRI, false>), dim3(grid), dim3(256), 0, s, X, ldx,
                     R, A, f0, g0, mask0);
  return hipGetLastError();
}

template <int DT, int BKT>
static hipError_t init_bk(const float *X, int64_t ldx, int64_t R, const AView &A, double *f0,
                          double *g0, uint8_t *mask0, bool gram, hipStream_t s) {
  if (gram) return init_t<DT, 4, BKT, true>(X, ldx, R, A, f0, g0, mask0, s);
  if (R <= 64) return init_t<DT, 1, BKT, false>(X, ldx, R, A, f0, g0, mask0, s);
  if (R <= 128) return init_t<DT, 2, BKT, false>(X, ldx, R, A, f0, g0, mask0, s);
  if (R <= 256) return init_t<DT, 4, BKT, false>(X, ldx, R, A, f0, g0, mask0, s);
  return init_t<DT, 8, BKT, false>(X, ldx, R, A, f0, g0, mask0, s);
}

template <int DT>
static hipError_t init_dt(const float *X, int64_t ldx, int64_t R, const AView &A, double *f0,
                          double *g0, uint8_t *mask0, bool gram, hipStream_t s) {
  // large tiles once the row dimension fills them (GCSS_MFMA_INIT256=0: off)
  static const bool big_ok = [] {
    const char *e = std::getenv("GCSS_MFMA_INIT256");
    return !(e && std::atoi(e) == 0);
  }();
  // narrow targets (64 <= R <= 128) on the BF16 matrix cores: 128-row chunks
  if (big_ok && mfma_x3() && !gram && R >= 64 && R <= 128 && A.n >= 1024) {
    const unsigned grid = (unsigned)((A.n + 255) / 256);
    hipLaunchKernelGGL((k_init_x3<false, DT, 128>), dim3(grid), dim3(kI2Threads), 0, s, X, ldx, R,
                       A, f0, g0, mask0);
    return hipGetLastError();
  }
  if (big_ok && R >= 192 && A.n >= 1024) {
    const unsigned grid = (unsigned)((A.n + 255) / 256);
    if (mfma_x3()) {
      if (gram)
        hipLaunchKernelGGL((k_init_x3<true, DT, 256>), dim3(grid), dim3(kI2Threads), 0, s, X, ldx,
                           R, A, f0, g0, mask0);
      else
        hipLaunchKernelGGL((k_init_x3<false, DT, 256>), dim3(grid), dim3(kI2Threads), 0, s, X, ldx,
                           R, A, f0, g0, mask0);
      return hipGetLastError();
    }
    if (gram)
      hipLaunchKernelGGL((k_init256<DT, true>), dim3(grid), dim3(kI2Threads), 0, s, X, ldx, R, A,
                         f0, g0, mask0);
    else
      hipLaunchKernelGGL((k_init256<DT, false>), dim3(grid), dim3(kI2Threads), 0, s, X, ldx, R, A,
                         f0, g0, mask0);
    return hipGetLastError();
  }
  if (mfma_bk(gram) == 16) return init_bk<DT, 16>(X, ldx, R, A, f0, g0, mask0, gram, s);
  return init_bk<DT, 32>(X, ldx, R, A, f0, g0, mask0, gram, s);
}

hipError_t launch_init_factor(const float *X, int64_t ldx, int64_t R, const AView &A,
                              double *f0, double *g0, uint8_t *mask0, hipStream_t s) {
  switch (A.dtype) {
    case DT_F32: return init_dt<DT_F32>(X, ldx, R, A, f0, g0, mask0, false, s);
    case DT_BF16: return init_dt<DT_BF16>(X, ldx, R, A, f0, g0, mask0, false, s);
    case DT_FP8: return init_dt<DT_FP8>(X, ldx, R, A, f0, g0, mask0, false, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_init_gram(const float *C, int64_t ldc, const AView &A, double *f0,
                            double *g0, uint8_t *mask0, hipStream_t s) {
  switch (A.dtype) {
    case DT_F32: return init_dt<DT_F32>(C, ldc, A.m, A, f0, g0, mask0, true, s);
    case DT_BF16: return init_dt<DT_BF16>(C, ldc, A.m, A, f0, g0, mask0, true, s);
    case DT_FP8: return init_dt<DT_FP8>(C, ldc, A.m, A, f0, g0, mask0, true, s);
  }
  return hipErrorInvalidValue;
}

// Tiling of a split-K product: tile edge (128, or 256 for the large-tile
// kernel), tile grid, k splits.  The split count fills whole rounds of
// resident workgroups as far as the partial-sum budget allows.  Plans depend
// only on the shapes (a fixed CU count), so the workspace sized from a plan
// always matches the launch.
struct KPlan {
  int tile, ntm, ntile, nsplit;
  int64_t kchunk;
};
constexpr int kPlanSlots256 = 256;  // resident large-tile workgroups (one per CU)

static int64_t pick_split(int64_t T, int64_t n, int64_t cap_sp, int64_t slots) {
  int64_t max_sp = (n + 255) / 256;  // every split at least 256 columns
  if (max_sp > cap_sp) max_sp = cap_sp;
  if (max_sp < 1) max_sp = 1;
  int64_t best = 1;
  double best_eff = -1.0;
  for (int64_t sp = 1; sp <= max_sp; ++sp) {
    const int64_t w = T * sp, rounds = (w + slots - 1) / slots;
    const double eff = (double)w / (double)(rounds * slots);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = sp;
    }
  }
  return best;
}

static void finish_plan(int64_t n, int64_t sp, KPlan *p) {
  int64_t kc = (n + sp - 1) / sp;
  kc = ((kc + KC_ALIGN - 1) / KC_ALIGN) * KC_ALIGN;
  p->kchunk = kc;
  p->nsplit = (int)((n + kc - 1) / kc);
}

static KPlan gram_plan(int64_t m, int64_t n) {
  KPlan p{};
  const int64_t ldp = ((m + 3) / 4) * 4;
  if (m >= 256) {
    p.tile = 256;
    const int64_t nt = (m + 255) / 256;
    const int64_t T = nt * (nt + 1) / 2;
    int64_t cap = (int64_t)(1LL << 30) / (ldp * m * (int64_t)sizeof(float));
    if (cap < 1) cap = 1;
    p.ntm = (int)nt;
    p.ntile = (int)T;
    finish_plan(n, pick_split(T, n, cap, kPlanSlots256), &p);
  } else {
    p.tile = 128;
    const int64_t nt = (m + 127) / 128;
    const int64_t T = nt * (nt + 1) / 2;
    int64_t sp = (8LL * 256 + T - 1) / T;
    if (sp > 8) sp = 8;
    if (sp < 1) sp = 1;
    p.ntm = (int)nt;
    p.ntile = (int)T;
    finish_plan(n, sp, &p);
  }
  return p;
}

size_t gram_scratch_bytes(int64_t m, int64_t n, int64_t ldc, int num_cu) {
  (void)ldc;
  (void)num_cu;
  const KPlan p = gram_plan(m, n);
  const int64_t ldp = ((m + 3) / 4) * 4;
  return (size_t)p.nsplit * ldp * m * sizeof(float);
}

hipError_t launch_gram(const AView &A, float *C, int64_t ldc, void *scratch, int num_cu,
                       hipStream_t s) {
  (void)num_cu;
  const KPlan pl = gram_plan(A.m, A.n);
  const int64_t ldp = ((A.m + 3) / 4) * 4;
  float *P = (float *)scratch;
  const int nt = pl.ntile, sp = pl.nsplit;
  const int64_t kc = pl.kchunk;
  const dim3 grid((unsigned)(nt * sp));
  if (pl.tile == 256) {
    switch (A.dtype) {
      case DT_F32:
        if (mfma_x3())
          hipLaunchKernelGGL(k_gram_x3, grid, dim3(kG2Threads), 0, s, A, P, ldp, nt, kc);
        else
          hipLaunchKernelGGL((k_gemm256<DT_F32, 16, 0>), grid, dim3(kG2Threads), 0, s, A, nullptr, 0, P, ldp, pl.ntm, nt, kc, 0u, 0u, 0u);
        break;
      case DT_BF16: hipLaunchKernelGGL((k_gemm256<DT_BF16, 16, 0>), grid, dim3(kG2Threads), 0, s, A, nullptr, 0, P, ldp, pl.ntm, nt, kc, 0u, 0u, 0u); break;
      case DT_FP8: hipLaunchKernelGGL((k_gemm256<DT_FP8, 16, 0>), grid, dim3(kG2Threads), 0, s, A, nullptr, 0, P, ldp, pl.ntm, nt, kc, 0u, 0u, 0u); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const bool bk16 = mfma_bk(false) == 16, db = mfma_db();
    switch (A.dtype) {
#define GCSS_GRAM(DTV)                                                                        \
  if (bk16 && db)                                                                             \
    hipLaunchKernelGGL((k_gram<DTV, 16, true>), grid, dim3(256), 0, s, A, P, ldp, nt, kc);    \
  else if (bk16)                                                                              \
    hipLaunchKernelGGL((k_gram<DTV, 16, false>), grid, dim3(256), 0, s, A, P, ldp, nt, kc);   \
  else if (db)                                                                                \
    hipLaunchKernelGGL((k_gram<DTV, 32, true>), grid, dim3(256), 0, s, A, P, ldp, nt, kc);    \
  else                                                                                        \
    hipLaunchKernelGGL((k_gram<DTV, 32, false>), grid, dim3(256), 0, s, A, P, ldp, nt, kc);   \
  break;
      case DT_F32: GCSS_GRAM(DT_F32)
      case DT_BF16: GCSS_GRAM(DT_BF16)
      case DT_FP8: GCSS_GRAM(DT_FP8)
#undef GCSS_GRAM
      default: return hipErrorInvalidValue;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nb64 = (A.m + 63) / 64;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)(nb64 * (nb64 + 1) / 2)), dim3(256), 0, s, P,
                     ldp, A.m, sp, C, ldc);
  return hipGetLastError();
}

// Narrow targets (64 <= r <= 128) on the BF16-split projection take tiles of
// 256 rows x 128 columns when m >= 256 (k_proj_x3<.., 128>).
static bool proj_narrow(int64_t m, int64_t r) { return m >= 256 && r >= 64 && r <= 128; }

static KPlan proj_plan(int64_t m, int64_t n, int64_t r, bool force256 = false,
                       bool narrow = false) {
  KPlan p{};
  // keep the partials within ~128 MiB and every split at least 256 columns long
  const int64_t ldp = ((m + 3) / 4) * 4;
  const int64_t per = ldp * r * (int64_t)sizeof(float);
  int64_t cap = (int64_t)(128LL << 20) / (per > 0 ? per : 1);
  if (cap < 1) cap = 1;
  if (narrow) {
    p.tile = 256;  // 256 rows x 128 columns, one column tile
    const int64_t tm = (m + 255) / 256;
    p.ntm = (int)tm;
    p.ntile = (int)tm;
    finish_plan(n, pick_split(tm, n, cap, kPlanSlots256), &p);
  } else if (force256 || (m >= 256 && r >= 192)) {
    p.tile = 256;
    const int64_t tm = (m + 255) / 256, tn = (r + 255) / 256;
    p.ntm = (int)tm;
    p.ntile = (int)(tm * tn);
    finish_plan(n, pick_split(tm * tn, n, cap, kPlanSlots256), &p);
  } else {
    p.tile = 128;
    const int64_t tm = (m + 127) / 128, tn = (r + 127) / 128;
    const int64_t T = tm * tn;
    int64_t sp = (8LL * 256 + T - 1) / T;
    if (sp > cap) sp = cap;
    if (sp > (n + 255) / 256) sp = (n + 255) / 256;
    if (sp < 1) sp = 1;
    p.ntm = (int)tm;
    p.ntile = (int)T;
    finish_plan(n, sp, &p);
  }
  return p;
}

size_t proj_scratch_bytes(int64_t m, int64_t n, int64_t r, int num_cu) {
  (void)num_cu;
  const KPlan p = proj_plan(m, n, r), p2 = proj_plan(m, n, r, true);
  const int64_t ldp = ((m + 3) / 4) * 4;
  int64_t sp = p.nsplit > p2.nsplit ? p.nsplit : p2.nsplit;
  if (proj_narrow(m, r)) {
    const KPlan p3 = proj_plan(m, n, r, false, true);
    if (p3.nsplit > sp) sp = p3.nsplit;
  }
  return (size_t)sp * ldp * r * sizeof(float);
}

hipError_t launch_proj_reduce(const float *P, int64_t ldp, int64_t m, int64_t r, int nsplit,
                              float *B, int64_t ldb, hipStream_t s) {
  const int64_t total = m * r;
  hipLaunchKernelGGL(k_proj_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, P,
                     ldp, m, r, nsplit, B, ldb);
  return hipGetLastError();
}

// B = A Omega with the random sign Omega generated inside the large-tile
// MFMA kernel (dense Omega: every entry +-1, or any density).
hipError_t launch_project_sign_dense(const AView &A, uint32_t k0, uint32_t k1, uint32_t thr,
                                     int64_t r, float *B, int64_t ldb, void *scratch,
                                     hipStream_t s) {
  const KPlan pl = proj_plan(A.m, A.n, r, true);
  const int64_t ldp = ((A.m + 3) / 4) * 4;
  float *P = (float *)scratch;
  const dim3 grid((unsigned)(pl.ntile * pl.nsplit));
  switch (A.dtype) {
    case DT_F32: hipLaunchKernelGGL((k_gemm256<DT_F32, 16, 2>), grid, dim3(kG2Threads), 0, s, A, nullptr, r, P, ldp, pl.ntm, pl.ntile, pl.kchunk, k0, k1, thr); break;
    case DT_BF16: hipLaunchKernelGGL((k_gemm256<DT_BF16, 16, 2>), grid, dim3(kG2Threads), 0, s, A, nullptr, r, P, ldp, pl.ntm, pl.ntile, pl.kchunk, k0, k1, thr); break;
    case DT_FP8: hipLaunchKernelGGL((k_gemm256<DT_FP8, 16, 2>), grid, dim3(kG2Threads), 0, s, A, nullptr, r, P, ldp, pl.ntm, pl.ntile, pl.kchunk, k0, k1, thr); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_proj_reduce(P, ldp, A.m, r, pl.nsplit, B, ldb, s);
}

hipError_t launch_project(const AView &A, const float *omega, int64_t r, float *B,
                          int64_t ldb, void *scratch, int num_cu, hipStream_t s) {
  (void)num_cu;
  const int64_t ldp = ((A.m + 3) / 4) * 4;
  float *P = (float *)scratch;
  // (k_proj_x3 forms its load addresses as 32-bit offsets from the stage's
  // first k: 32 columns of A and 32 rows of Omega must span under 2^31 bytes)
  const int64_t es = A.dtype == DT_F32 ? 4 : A.dtype == DT_BF16 ? 2 : 1;
  const bool off32 = 32 * A.lda * es < (1LL << 31) && 32 * r * 4 < (1LL << 31);
  const bool x3 = mfma_x3() && A.m % 4 == 0 && r % 4 == 0 && off32;
  if (x3 && proj_narrow(A.m, r)) {
    const KPlan pn = proj_plan(A.m, A.n, r, false, true);
    const dim3 gn((unsigned)(pn.ntile * pn.nsplit));
    switch (A.dtype) {
      case DT_F32: hipLaunchKernelGGL((k_proj_x3<DT_F32, 128>), gn, dim3(kG2Threads), 0, s, A, omega, r, P, ldp, pn.ntm, pn.ntile, pn.kchunk); break;
      case DT_BF16: hipLaunchKernelGGL((k_proj_x3<DT_BF16, 128>), gn, dim3(kG2Threads), 0, s, A, omega, r, P, ldp, pn.ntm, pn.ntile, pn.kchunk); break;
      case DT_FP8: hipLaunchKernelGGL((k_proj_x3<DT_FP8, 128>), gn, dim3(kG2Threads), 0, s, A, omega, r, P, ldp, pn.ntm, pn.ntile, pn.kchunk); break;
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_proj_reduce(P, ldp, A.m, r, pn.nsplit, B, ldb, s);
  }
  const KPlan pl = proj_plan(A.m, A.n, r);
  const int tm = pl.ntm, nt = pl.ntile, sp = pl.nsplit;
  const int tn = nt / tm;
  const int64_t kc = pl.kchunk;
  const dim3 grid((unsigned)(nt * sp));
  if (pl.tile == 256) {
    if (x3) {
      switch (A.dtype) {
        case DT_F32: hipLaunchKernelGGL((k_proj_x3<DT_F32, 256>), grid, dim3(kG2Threads), 0, s, A, omega, r, P, ldp, tm, nt, kc); break;
        case DT_BF16: hipLaunchKernelGGL((k_proj_x3<DT_BF16, 256>), grid, dim3(kG2Threads), 0, s, A, omega, r, P, ldp, tm, nt, kc); break;
        case DT_FP8: hipLaunchKernelGGL((k_proj_x3<DT_FP8, 256>), grid, dim3(kG2Threads), 0, s, A, omega, r, P, ldp, tm, nt, kc); break;
        default: return hipErrorInvalidValue;
      }
    } else
    switch (A.dtype) {
      case DT_F32: hipLaunchKernelGGL((k_gemm256<DT_F32, 16, 1>), grid, dim3(kG2Threads), 0, s, A, omega, r, P, ldp, tm, nt, kc, 0u, 0u, 0u); break;
      case DT_BF16: hipLaunchKernelGGL((k_gemm256<DT_BF16, 16, 1>), grid, dim3(kG2Threads), 0, s, A, omega, r, P, ldp, tm, nt, kc, 0u, 0u, 0u); break;
      case DT_FP8: hipLaunchKernelGGL((k_gemm256<DT_FP8, 16, 1>), grid, dim3(kG2Threads), 0, s, A, omega, r, P, ldp, tm, nt, kc, 0u, 0u, 0u); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const bool bk16 = mfma_bk(false) == 16, db = mfma_db();
    switch (A.dtype) {
#define GCSS_PROJ(DTV)                                                                        \
  if (bk16 && db)                                                                             \
    hipLaunchKernelGGL((k_project<DTV, 16, true>), grid, dim3(256), 0, s, A, omega, r, P, ldp, \
                       tm, tn, kc);                                                           \
  else if (bk16)                                                                              \
    hipLaunchKernelGGL((k_project<DTV, 16, false>), grid, dim3(256), 0, s, A, omega, r, P,     \
                       ldp, tm, tn, kc);                                                      \
  else if (db)                                                                                \
    hipLaunchKernelGGL((k_project<DTV, 32, true>), grid, dim3(256), 0, s, A, omega, r, P, ldp, \
                       tm, tn, kc);                                                           \
  else                                                                                        \
    hipLaunchKernelGGL((k_project<DTV, 32, false>), grid, dim3(256), 0, s, A, omega, r, P,     \
                       ldp, tm, tn, kc);                                                      \
  break;
      case DT_F32: GCSS_PROJ(DT_F32)
      case DT_BF16: GCSS_PROJ(DT_BF16)
      case DT_FP8: GCSS_PROJ(DT_FP8)
#undef GCSS_PROJ
      default: return hipErrorInvalidValue;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = A.m * r;
  hipLaunchKernelGGL(k_proj_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, P,
                     ldp, A.m, r, sp, B, ldb);
  return hipGetLastError();
}

}  // namespace gcss
