// Dense contractions of the selection, on the CDNA matrix cores
// (v_mfma_f32_16x16x4_f32, FP32 in / FP32 accumulate):
//
//   init scores (Algorithm 3, first line):   f_i = || X^T A_i ||^2,
//       X = B (m x r), the epilogue sums the squares so the r x n product is
//       never stored; g_i = || A_i ||^2 is accumulated from the same A tiles.
//   init scores, Gram target (B = A enters only through C = A A^T):
//       f_i = A_i^T C A_i = || A^T A_i ||^2, epilogue dot with A_i.
//   Gram matrix C = A A^T (symmetric rank-n update, upper tiles, split-K).
//   Projection B = A Omega (Section 5.1), split-K with a fixed-order reduce.
//
// All tiles are staged in LDS in "k-major" layout (each row of the tile
// holds 16 consecutive k values, pitch 20 floats).  A lane feeds the 16x16x4
// instruction from one 16-byte LDS read per operand: lane l takes rows
// l%16 and the k quad 4*(l/16)..+3, and the four instructions s = 0..3 use
// element s of that quad, so the four lane groups cover all 16 k values.
// Output layout of v_mfma_f32_16x16x4_f32: lane l, register v holds
// D[4*(l/16) + v][l%16].
#include "gcss_device.h"

namespace gcss {

constexpr int BK = 16;   // k values per LDS stage
constexpr int PIT = 20;  // LDS row pitch in floats

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// acc[rb][nb] += X_rows(rb) * Y_cols(nb) over one BK stage.
template <int RB, int NB>
__device__ __forceinline__ void mma_stage(const float *Xs, int xrow0, const float *Ys, int ycol0,
                                          int lane, f32x4 (&acc)[RB][NB]) {
  const int r = lane & 15, kq = (lane >> 4) * 4;
  float4 xa[RB], yb[NB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) xa[rb] = *(const float4 *)(Xs + (xrow0 + 16 * rb + r) * PIT + kq);
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) yb[nb] = *(const float4 *)(Ys + (ycol0 + 16 * nb + r) * PIT + kq);
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
// RT = 64*RB; the column results are accumulated across chunks.
template <int DT, int RB, int NB, bool GRAM>
__global__ __launch_bounds__(256) void k_init(const float *__restrict__ X, int64_t ldx,
                                              int64_t R, AView A, double *__restrict__ f0,
                                              double *__restrict__ g0,
                                              uint8_t *__restrict__ mask0) {
  constexpr int RT = 64 * RB, NT = 16 * NB;
  constexpr int ES = EInfo<DT>::esize, EPC = EInfo<DT>::epc;
  constexpr int CPC = ES;  // 16-byte chunks per column per stage (16 k values)
  __shared__ __align__(16) float Xs[RT * PIT];
  __shared__ __align__(16) float Ys[NT * PIT];
  __shared__ double red[4][NT];
  __shared__ double gs[NT];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m = A.m, n = A.n;
  const int64_t j0 = (int64_t)blockIdx.x * NT;
  const char *abase = (const char *)A.a;
  const int64_t colb = A.lda * ES;

  // Y loader: thread -> (column, chunk)
  const int ycol = tid / CPC, ych = tid % CPC;
  const bool yact = tid < NT * CPC;
  const bool ycolv = yact && (j0 + ycol) < n;
  double gacc = 0.0;

  double colacc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) colacc[nb] = 0.0;

  const int64_t nchunks = (R + RT - 1) / RT;
  const int64_t ksteps = (m + BK - 1) / BK;
  for (int64_t rc = 0; rc < nchunks; ++rc) {
    const int64_t r0 = rc * RT;
    f32x4 acc[RB][NB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    float4 xr[RB];
    uint4 yr = make_uint4(0u, 0u, 0u, 0u);
    auto gload = [&](int64_t k0) {
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int q = tid + 256 * u;
        const int row = q >> 2, kq = (q & 3) * 4;
        const int64_t gr = r0 + row, gk = k0 + kq;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gr < R && gk < m) {
          v = *(const float4 *)(X + gr * ldx + gk);
          if (gk + 4 > m) {
            if (gk + 1 >= m) v.y = 0.f;
            if (gk + 2 >= m) v.z = 0.f;
            if (gk + 3 >= m) v.w = 0.f;
          }
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
      for (int u = 0; u < RB; ++u) {
        const int q = tid + 256 * u;
        const int row = q >> 2, kq = (q & 3) * 4;
        *(float4 *)(Xs + row * PIT + kq) = xr[u];
      }
      if (yact) {
        float v[EPC];
        decode16<DT>(yr, v);
        const int64_t gk = k0 + ych * EPC;
#pragma unroll
        for (int e = 0; e < EPC; ++e)
          if (gk + e >= m) v[e] = 0.f;
        if (rc == 0) {
#pragma unroll
          for (int e = 0; e < EPC; ++e) gacc = fma((double)v[e], (double)v[e], gacc);
        }
#pragma unroll
        for (int e = 0; e < EPC; e += 4)
          *(float4 *)(Ys + ycol * PIT + ych * EPC + e) = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
      }
    };

    gload(0);
    for (int64_t ks = 0; ks < ksteps; ++ks) {
      __syncthreads();
      sstore(ks * BK);
      __syncthreads();
      if (ks + 1 < ksteps) gload((ks + 1) * BK);
      mma_stage<RB, NB>(Xs, wave * 16 * RB, Ys, 0, lane, acc);
    }

    // epilogue of this row chunk
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t j = j0 + 16 * nb + (lane & 15);
      double s = 0.0;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int64_t i = r0 + wave * 16 * RB + 16 * rb + 4 * (lane >> 4);
        if constexpr (GRAM) {
          float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
          if (j < n && i < m) {
            a = load4<DT>(A.a, j * A.lda + i);
            if (i + 1 >= m) a.y = 0.f;
            if (i + 2 >= m) a.z = 0.f;
            if (i + 3 >= m) a.w = 0.f;
          }
          s += (double)acc[rb][nb][0] * a.x + (double)acc[rb][nb][1] * a.y +
               (double)acc[rb][nb][2] * a.z + (double)acc[rb][nb][3] * a.w;
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v) s += (double)acc[rb][nb][v] * (double)acc[rb][nb][v];
        }
      }
      colacc[nb] += s;
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
  // g: sum over the CPC threads of a column
  double gsum = gacc;
  if constexpr (CPC >= 2) gsum += __shfl_xor(gsum, 1, 64);
  if constexpr (CPC >= 4) gsum += __shfl_xor(gsum, 2, 64);
  if (yact && ych == 0) gs[ycol] = gsum;
  __syncthreads();
  if (tid < NT) {
    const int64_t j = j0 + tid;
    if (j < n) {
      const double fv = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      const double sc = col_scale(A, j);
      const double f = sc * sc * fv, g = sc * sc * gs[tid];
      f0[j] = f;
      g0[j] = g;
      mask0[j] = (g > 0.0 && isfinite(g) && isfinite(f)) ? 0 : 2;
    }
  }
}

// ---------------------------------------------------------------------------
// 128 x 128 output tiles, 4 waves in a 2 x 2 arrangement of 64 x 64.
// X[k][i] = A[i, k]: for each k (a column of A) the tile's rows are
// consecutive in memory; they are decoded, scaled by the column scale and
// written transposed into the k-major LDS tile.
template <int DT>
__device__ __forceinline__ void load_at_tile(const AView &A, int64_t i0, int64_t k0,
                                             int64_t kend, int tid, uint4 (&raw)[2],
                                             int (&kk)[2], int (&ii)[2], bool (&ok)[2]) {
  constexpr int ES = EInfo<DT>::esize, EPC = EInfo<DT>::epc;
  constexpr int CPK = 128 / EPC;  // chunks per k (128 rows)
  const char *abase = (const char *)A.a;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = tid + 256 * u;
    kk[u] = q / CPK;
    ii[u] = (q % CPK) * EPC;
    ok[u] = q < 16 * CPK && (k0 + kk[u]) < kend && (i0 + ii[u]) < A.m;
    raw[u] = ok[u] ? *(const uint4 *)(abase + ((k0 + kk[u]) * A.lda + i0 + ii[u]) * ES)
                   : make_uint4(0u, 0u, 0u, 0u);
  }
}

template <int DT>
__device__ __forceinline__ void store_at_tile(const AView &A, float *Ts, int64_t i0, int64_t k0,
                                              int tid, const uint4 (&raw)[2], const int (&kk)[2],
                                              const int (&ii)[2], const bool (&ok)[2]) {
  constexpr int EPC = EInfo<DT>::epc;
  constexpr int CPK = 128 / EPC;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = tid + 256 * u;
    if (q >= 16 * CPK) continue;
    float v[EPC];
    decode16<DT>(raw[u], v);
    float sc = 1.f;
    if constexpr (DT == DT_FP8) sc = ok[u] ? A.scale[k0 + kk[u]] : 0.f;
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
      const bool in = ok[u] && (i0 + ii[u] + e) < A.m;
      Ts[(ii[u] + e) * PIT + kk[u]] = in ? v[e] * sc : 0.f;
    }
  }
}

template <int DT>
__global__ __launch_bounds__(256) void k_gram(AView A, float *__restrict__ P, int64_t ldp,
                                              int ntile, int64_t kchunk) {
  __shared__ __align__(16) float Xs[128 * PIT];
  __shared__ __align__(16) float Ys[128 * PIT];
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

  uint4 xr[2], yr[2];
  int xk[2], xi[2], yk[2], yi[2];
  bool xo[2], yo[2];
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  if (kb < ke) load_at_tile<DT>(A, i0, kb, ke, tid, xr, xk, xi, xo);
  if (kb < ke) load_at_tile<DT>(A, j0, kb, ke, tid, yr, yk, yi, yo);
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();
    store_at_tile<DT>(A, Xs, i0, k0, tid, xr, xk, xi, xo);
    store_at_tile<DT>(A, Ys, j0, k0, tid, yr, yk, yi, yo);
    __syncthreads();
    if (k0 + BK < ke) {
      load_at_tile<DT>(A, i0, k0 + BK, ke, tid, xr, xk, xi, xo);
      load_at_tile<DT>(A, j0, k0 + BK, ke, tid, yr, yk, yi, yo);
    }
    mma_stage<4, 4>(Xs, wr, Ys, wc, lane, acc);
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int64_t i = i0 + wr + 16 * rb + 4 * (lane >> 4);
      const int64_t j = j0 + wc + 16 * nb + (lane & 15);
      if (j < m)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (i + v < m) Pout[j * ldp + i + v] = acc[rb][nb][v];
    }
}

// C[i,j] = sum_s P_s[min, max] (upper tiles only were computed; exact symmetry)
__global__ void k_gram_reduce(const float *__restrict__ P, int64_t ldp, int64_t m, int nsplit,
                              float *__restrict__ C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  const int64_t j = e / m, i = e % m;
  const int64_t src = (i <= j) ? (j * ldp + i) : (i * ldp + j);
  float s = 0.f;
  for (int x = 0; x < nsplit; ++x) s += P[x * ldp * m + src];
  C[j * ldc + i] = s;
}

// B = A Omega: X[k][i] = A[i, k], Y[k][j] = Omega[k, j] (row-major n x r).
template <int DT>
__global__ __launch_bounds__(256) void k_project(AView A, const float *__restrict__ Om,
                                                 int64_t r, float *__restrict__ P, int64_t ldp,
                                                 int ntm, int ntn, int64_t kchunk) {
  __shared__ __align__(16) float Xs[128 * PIT];
  __shared__ __align__(16) float Ys[128 * PIT];
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

  uint4 xr[2];
  int xk[2], xi[2];
  bool xo[2];
  float4 yv[2];
  auto yload = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
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
  auto ystore = [&]() {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = tid + 256 * u;
      const int kk = q >> 5, jj = (q & 31) * 4;
      Ys[(jj + 0) * PIT + kk] = yv[u].x;
      Ys[(jj + 1) * PIT + kk] = yv[u].y;
      Ys[(jj + 2) * PIT + kk] = yv[u].z;
      Ys[(jj + 3) * PIT + kk] = yv[u].w;
    }
  };
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  if (kb < ke) {
    load_at_tile<DT>(A, i0, kb, ke, tid, xr, xk, xi, xo);
    yload(kb);
  }
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();
    store_at_tile<DT>(A, Xs, i0, k0, tid, xr, xk, xi, xo);
    ystore();
    __syncthreads();
    if (k0 + BK < ke) {
      load_at_tile<DT>(A, i0, k0 + BK, ke, tid, xr, xk, xi, xo);
      yload(k0 + BK);
    }
    mma_stage<4, 4>(Xs, wr, Ys, wc, lane, acc);
  }
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int64_t i = i0 + wr + 16 * rb + 4 * (lane >> 4);
      const int64_t j = j0 + wc + 16 * nb + (lane & 15);
      if (j < r)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (i + v < A.m) Pout[j * ldp + i + v] = acc[rb][nb][v];
    }
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
template <int DT, int RB, bool GRAM>
static hipError_t init_t(const float *X, int64_t ldx, int64_t R, const AView &A, double *f0,
                         double *g0, uint8_t *mask0, hipStream_t s) {
  constexpr int NB = 4;
  const unsigned grid = (unsigned)((A.n + 16 * NB - 1) / (16 * NB));
  hipLaunchKernelGGL((k_init<DT, RB, NB, GRAM>), dim3(grid), dim3(256), 0, s, X, ldx, R, A, f0,
                     g0, mask0);
  return hipGetLastError();
}

template <int DT>
static hipError_t init_dt(const float *X, int64_t ldx, int64_t R, const AView &A, double *f0,
                          double *g0, uint8_t *mask0, bool gram, hipStream_t s) {
  if (gram) return init_t<DT, 4, true>(X, ldx, R, A, f0, g0, mask0, s);
  if (R <= 64) return init_t<DT, 1, false>(X, ldx, R, A, f0, g0, mask0, s);
  if (R <= 128) return init_t<DT, 2, false>(X, ldx, R, A, f0, g0, mask0, s);
  if (R <= 256) return init_t<DT, 4, false>(X, ldx, R, A, f0, g0, mask0, s);
  return init_t<DT, 8, false>(X, ldx, R, A, f0, g0, mask0, s);
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

static void gram_plan(int64_t m, int64_t n, int num_cu, int *ntile, int *nsplit,
                      int64_t *kchunk) {
  const int64_t nt = (m + 127) / 128;
  const int64_t T = nt * (nt + 1) / 2;
  int64_t sp = (8LL * num_cu + T - 1) / T;
  if (sp > 8) sp = 8;
  if (sp < 1) sp = 1;
  int64_t kc = (n + sp - 1) / sp;
  kc = ((kc + BK - 1) / BK) * BK;
  sp = (n + kc - 1) / kc;
  *ntile = (int)T;
  *nsplit = (int)sp;
  *kchunk = kc;
}

size_t gram_scratch_bytes(int64_t m, int64_t n, int64_t ldc, int num_cu) {
  int nt, sp;
  int64_t kc;
  gram_plan(m, n, num_cu, &nt, &sp, &kc);
  (void)ldc;
  const int64_t ldp = ((m + 3) / 4) * 4;
  return (size_t)sp * ldp * m * sizeof(float);
}

hipError_t launch_gram(const AView &A, float *C, int64_t ldc, void *scratch, int num_cu,
                       hipStream_t s) {
  int nt, sp;
  int64_t kc;
  gram_plan(A.m, A.n, num_cu, &nt, &sp, &kc);
  const int64_t ldp = ((A.m + 3) / 4) * 4;
  float *P = (float *)scratch;
  const dim3 grid((unsigned)(nt * sp));
  switch (A.dtype) {
    case DT_F32: hipLaunchKernelGGL(k_gram<DT_F32>, grid, dim3(256), 0, s, A, P, ldp, nt, kc); break;
    case DT_BF16: hipLaunchKernelGGL(k_gram<DT_BF16>, grid, dim3(256), 0, s, A, P, ldp, nt, kc); break;
    case DT_FP8: hipLaunchKernelGGL(k_gram<DT_FP8>, grid, dim3(256), 0, s, A, P, ldp, nt, kc); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = A.m * A.m;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, P,
                     ldp, A.m, sp, C, ldc);
  return hipGetLastError();
}

static void proj_plan(int64_t m, int64_t n, int64_t r, int num_cu, int *ntm, int *ntn,
                      int *nsplit, int64_t *kchunk) {
  const int64_t tm = (m + 127) / 128, tn = (r + 127) / 128;
  const int64_t T = tm * tn;
  int64_t sp = (8LL * num_cu + T - 1) / T;
  // keep the partials within ~128 MiB and every split at least 256 columns long
  const int64_t ldp = ((m + 3) / 4) * 4;
  const int64_t per = ldp * r * (int64_t)sizeof(float);
  int64_t cap = (int64_t)(128LL << 20) / (per > 0 ? per : 1);
  if (cap < 1) cap = 1;
  if (sp > cap) sp = cap;
  if (sp > (n + 255) / 256) sp = (n + 255) / 256;
  if (sp < 1) sp = 1;
  int64_t kc = (n + sp - 1) / sp;
  kc = ((kc + BK - 1) / BK) * BK;
  sp = (n + kc - 1) / kc;
  *ntm = (int)tm;
  *ntn = (int)tn;
  *nsplit = (int)sp;
  *kchunk = kc;
}

size_t proj_scratch_bytes(int64_t m, int64_t n, int64_t r, int num_cu) {
  int tm, tn, sp;
  int64_t kc;
  proj_plan(m, n, r, num_cu, &tm, &tn, &sp, &kc);
  const int64_t ldp = ((m + 3) / 4) * 4;
  return (size_t)sp * ldp * r * sizeof(float);
}

hipError_t launch_project(const AView &A, const float *omega, int64_t r, float *B,
                          int64_t ldb, void *scratch, int num_cu, hipStream_t s) {
  int tm, tn, sp;
  int64_t kc;
  proj_plan(A.m, A.n, r, num_cu, &tm, &tn, &sp, &kc);
  const int64_t ldp = ((A.m + 3) / 4) * 4;
  float *P = (float *)scratch;
  const dim3 grid((unsigned)(tm * tn * sp));
  switch (A.dtype) {
    case DT_F32:
      hipLaunchKernelGGL(k_project<DT_F32>, grid, dim3(256), 0, s, A, omega, r, P, ldp, tm, tn, kc);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(k_project<DT_BF16>, grid, dim3(256), 0, s, A, omega, r, P, ldp, tm, tn, kc);
      break;
    case DT_FP8:
      hipLaunchKernelGGL(k_project<DT_FP8>, grid, dim3(256), 0, s, A, omega, r, P, ldp, tm, tn, kc);
      break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = A.m * r;
  hipLaunchKernelGGL(k_proj_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, P,
                     ldp, A.m, r, sp, B, ldb);
  return hipGetLastError();
}

}  // namespace gcss
