// Fused streaming pass of one greedy step (Theorem 4 in the q/z form).
//
// For every column i of A, one coalesced read gives
//     omega_i = s_i * (A_i . q),   gamma_i = s_i * (A_i . z)
// (s_i = FP8 column scale, 1 otherwise), then in FP64
//     f_i <- f_i - 2 omega_i gamma_i + ||upsilon||^2 omega_i^2
//     g_i <- g_i - omega_i^2
// and the column's score f_i / g_i enters the argmax of the next pick.
// The last workgroup to finish reduces the per-workgroup winners and writes
// the next pick into the device state.
//
// Work mapping (CDNA4, 64-lane wavefronts, 256-thread workgroups):
//   * a "team" of W wavefronts owns a group of G consecutive columns; wave
//     w of the team reads rows [w*S, (w+1)*S) of each column, S = 64*NJ
//     16-byte chunks, so every load instruction of a wave covers 1 KiB of
//     one column, fully coalesced;
//   * q and z for those rows live in registers (NJ * EPC floats each);
//   * after each column the two partial dots are summed across the wave,
//     and lane c keeps the result of column c of the group;
//   * the FP64 epilogue runs with one column per lane.
#include "gcss_device.h"

namespace gcss {

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

template <int DT, int NJ, int W>
__global__ __launch_bounds__(256) void k_stream(AView A, int G, const float *__restrict__ q32,
                                                const float *__restrict__ z32,
                                                double *__restrict__ f, double *__restrict__ g,
                                                const double *__restrict__ g0,
                                                const uint8_t *__restrict__ mask,
                                                ArgPart *__restrict__ part, DevState *st,
                                                int score_only) {
  constexpr int EPC = Elem<DT>::epc;
  constexpr int TEAMS = 4 / W;
  constexpr int U = (16 / NJ) > 0 ? (16 / NJ) : 1;  // columns in flight per wave
  __shared__ float red[2][4][64];
  __shared__ double bs[4];
  __shared__ int64_t bi_s[4];

  if (st->done) return;
  const bool rescore = score_only || st->skip;
  const double u2 = st->u2;
  const double tau = st->tau;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int team = wave / W;
  const int ws = wave % W;
  const int64_t m = A.m, n = A.n;
  const int64_t ngroups = (n + G - 1) / G;
  const int64_t nsuper = (ngroups + TEAMS - 1) / TEAMS;
  const char *abase = (const char *)A.a;
  const int64_t col_bytes = A.lda * Elem<DT>::esize;

  // q, z for this lane's rows
  float qv[NJ][EPC], zv[NJ][EPC];
  int valid[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t ci = (int64_t)ws * 64 * NJ + j * 64 + lane;
    const int64_t e0 = ci * EPC;
    valid[j] = (int)(e0 < m ? (m - e0 < EPC ? m - e0 : EPC) : 0);
#pragma unroll
    for (int e = 0; e < EPC; e += 4) {
      float4 a = *(const float4 *)(q32 + e0 + e);
      float4 b = *(const float4 *)(z32 + e0 + e);
      qv[j][e] = a.x;
      qv[j][e + 1] = a.y;
      qv[j][e + 2] = a.z;
      qv[j][e + 3] = a.w;
      zv[j][e] = b.x;
      zv[j][e + 1] = b.y;
      zv[j][e + 2] = b.z;
      zv[j][e + 3] = b.w;
    }
  }

  double best = -INFINITY;
  int64_t besti = kNoIdx;

  for (int64_t sg = blockIdx.x; sg < nsuper; sg += gridDim.x) {
    const int64_t grp = sg * TEAMS + team;
    const int64_t col0 = grp * G;
    const int ncol = grp < ngroups ? (int)((n - col0) < G ? (n - col0) : G) : 0;
    float mw = 0.f, mz = 0.f;
    if (!rescore) {
      for (int c0 = 0; c0 < ncol; c0 += U) {
        uint4 raw[U][NJ];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool cv = (c0 + u) < ncol;
          const char *cp = abase + (col0 + c0 + u) * col_bytes;
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const int64_t ci = (int64_t)ws * 64 * NJ + j * 64 + lane;
            if (cv && valid[j] > 0)
              raw[u][j] = *(const uint4 *)(cp + ci * 16);
            else
              raw[u][j] = make_uint4(0u, 0u, 0u, 0u);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          float dq = 0.f, dz = 0.f;
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            float v[EPC];
            decode_chunk<DT>(raw[u][j], v);
            if (valid[j] < EPC) {
#pragma unroll
              for (int e = 0; e < EPC; ++e)
                if (e >= valid[j]) v[e] = 0.f;
            }
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
              dq = fmaf(v[e], qv[j][e], dq);
              dz = fmaf(v[e], zv[j][e], dz);
            }
          }
          dq = wave_sum(dq);
          dz = wave_sum(dz);
          if (lane == c0 + u) {
            mw = dq;
            mz = dz;
          }
        }
      }
    }
    if constexpr (W > 1) {
      red[0][wave][lane] = mw;
      red[1][wave][lane] = mz;
      __syncthreads();
      if (ws == 0) {
        float sw = 0.f, sz = 0.f;
#pragma unroll
        for (int x = 0; x < W; ++x) {
          sw += red[0][wave + x][lane];
          sz += red[1][wave + x][lane];
        }
        mw = sw;
        mz = sz;
      }
      __syncthreads();
    }
    if (ws == 0 && lane < ncol) {
      const int64_t col = col0 + lane;
      double fv = f[col], gv = g[col];
      if (!rescore) {
        const double s = (DT == DT_FP8) ? (double)A.scale[col] : 1.0;
        const double w = s * (double)mw, y = s * (double)mz;
        fv = fv - 2.0 * w * y + u2 * w * w;
        gv = gv - w * w;
        f[col] = fv;
        g[col] = gv;
      }
      if (mask[col] == 0 && gv > tau * g0[col] && isfinite(fv) && isfinite(gv)) {
        const double sc = fv / gv;
        if (better(sc, col, best, besti)) {
          best = sc;
          besti = col;
        }
      }
    }
  }

  // workgroup winner
  wave_argmax(best, besti);
  if (lane == 0) {
    bs[wave] = best;
    bi_s[wave] = besti;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = bs[0];
    int64_t bi = bi_s[0];
    for (int x = 1; x < 4; ++x)
      if (better(bs[x], bi_s[x], b, bi)) {
        b = bs[x];
        bi = bi_s[x];
      }
    part[blockIdx.x].score = b;
    part[blockIdx.x].idx = bi;
  }
  if (!last_block_arrive(&st->cnt[0])) return;

  // last workgroup: winner over all workgroups -> next pick
  best = -INFINITY;
  besti = kNoIdx;
  for (int x = threadIdx.x; x < (int)gridDim.x; x += blockDim.x) {
    const double s = load_acquire_f64(&part[x].score);
    const int64_t i = load_acquire_i64(&part[x].idx);
    if (better(s, i, best, besti)) {
      best = s;
      besti = i;
    }
  }
  wave_argmax(best, besti);
  __syncthreads();
  if (lane == 0) {
    bs[wave] = best;
    bi_s[wave] = besti;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = bs[0];
    int64_t bi = bi_s[0];
    for (int x = 1; x < 4; ++x)
      if (better(bs[x], bi_s[x], b, bi)) {
        b = bs[x];
        bi = bi_s[x];
      }
    if (bi == kNoIdx) {
      st->p = -1;
      st->exhausted = 1;
      st->done = 1;
    } else {
      st->p = bi;
    }
    st->skip = 0;
    st->cnt[0] = 0;
  }
}

// ---------------------------------------------------------------------------
static int pow2_at_least(int64_t x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

StreamGeo stream_geometry(int64_t m, int64_t n, int dtype, int num_cu) {
  StreamGeo geo{};
  const int epc = 16 / dtype_bytes(dtype);
  const int nj_max = 32 / epc;  // q and z: at most 32 floats each per lane
  const int64_t chunks = (m + epc - 1) / epc;
  int w = 1;
  while (w < 4 && chunks > (int64_t)64 * w * nj_max) w <<= 1;
  if (chunks > (int64_t)64 * w * nj_max) {
    geo.nj = 0;  // unsupported
    return geo;
  }
  int nj = pow2_at_least((chunks + 64 * w - 1) / (64 * w));
  if (nj < 1) nj = 1;
  geo.nj = nj;
  geo.w = w;
  geo.qlen = w * 64 * nj * epc;
  const int teams = 4 / w;
  // column group size: 64 unless that leaves fewer than ~4 workgroups per CU
  int G = 64;
  while (G > 16 && ((n + G - 1) / G + teams - 1) / teams < 4LL * num_cu) G >>= 1;
  geo.g = G;
  const int64_t nsuper = (((n + G - 1) / G) + teams - 1) / teams;
  const int64_t cap = 16LL * num_cu;
  geo.grid = (int)(nsuper < cap ? nsuper : cap);
  if (geo.grid < 1) geo.grid = 1;
  return geo;
}

template <int DT, int NJ, int W>
static hipError_t launch_t(const StreamGeo &geo, const AView &A, const float *q32,
                           const float *z32, double *f, double *g, const double *g0,
                           uint8_t *mask, ArgPart *part, DevState *st, int score_only,
                           hipStream_t s) {
  hipLaunchKernelGGL((k_stream<DT, NJ, W>), dim3(geo.grid), dim3(256), 0, s, A, geo.g, q32, z32,
                     f, g, g0, mask, part, st, score_only);
  return hipGetLastError();
}

template <int DT, int NJ>
static hipError_t launch_w(const StreamGeo &geo, const AView &A, const float *q32,
                           const float *z32, double *f, double *g, const double *g0,
                           uint8_t *mask, ArgPart *part, DevState *st, int score_only,
                           hipStream_t s) {
  switch (geo.w) {
    case 1: return launch_t<DT, NJ, 1>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
    case 2: return launch_t<DT, NJ, 2>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
    case 4: return launch_t<DT, NJ, 4>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
  }
  return hipErrorInvalidValue;
}

template <int DT>
static hipError_t launch_nj(const StreamGeo &geo, const AView &A, const float *q32,
                            const float *z32, double *f, double *g, const double *g0,
                            uint8_t *mask, ArgPart *part, DevState *st, int score_only,
                            hipStream_t s) {
  constexpr int NJMAX = 32 / Elem<DT>::epc;
  switch (geo.nj) {
    case 1: return launch_w<DT, 1>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
    case 2:
      if constexpr (NJMAX >= 2)
        return launch_w<DT, 2>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
      break;
    case 4:
      if constexpr (NJMAX >= 4)
        return launch_w<DT, 4>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
      break;
    case 8:
      if constexpr (NJMAX >= 8)
        return launch_w<DT, 8>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
      break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stream(const StreamGeo &geo, const AView &A, const float *q32,
                         const float *z32, double *f, double *g, const double *g0,
                         uint8_t *mask, ArgPart *part, DevState *st, int score_only,
                         hipStream_t s) {
  switch (A.dtype) {
    case DT_F32: return launch_nj<DT_F32>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
    case DT_BF16: return launch_nj<DT_BF16>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
    case DT_FP8: return launch_nj<DT_FP8>(geo, A, q32, z32, f, g, g0, mask, part, st, score_only, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gcss
