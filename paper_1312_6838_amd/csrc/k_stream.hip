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

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16-byte load of a chunk of A; NT: non-temporal (A is read once per pass).
template <bool NT>
__device__ __forceinline__ uint4 load_chunk(const char *p) {
  u32x4 v;
  if constexpr (NT)
    v = __builtin_nontemporal_load((const u32x4 *)p);
  else
    v = *(const u32x4 *)p;
  return make_uint4(v[0], v[1], v[2], v[3]);
}

template <int DT, int NJ, int W, bool NT, bool QL>
__global__ __launch_bounds__(256) void k_stream(AView A, int G, const float *__restrict__ q32,
                                                const float *__restrict__ z32,
                                                double *__restrict__ f, double *__restrict__ g,
                                                const double *__restrict__ g0,
                                                const uint8_t *__restrict__ mask,
                                                ArgPart *__restrict__ part, DevState *st,
                                                double *__restrict__ ap64, int score_only) {
  constexpr int EPC = Elem<DT>::epc;
  constexpr int TEAMS = 4 / W;
  constexpr int U = (8 / NJ) > 0 ? (8 / NJ) : 1;  // columns per load group
  __shared__ float red[2][4][64];
  __shared__ double bs[4];
  __shared__ int64_t bi_s[4];
  __shared__ int64_t sg_s;

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

  // q, z for this lane's rows; chunk j of the lane is ci(j) = ws*64*NJ + 64*j + lane.
  // Registers (QL = false) or LDS (QL = true, for long columns).
  extern __shared__ float qz_lds[];
  constexpr int NR = QL ? 1 : NJ;
  float qv[NR][EPC], zv[NR][EPC];
  int valid[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t ci = (int64_t)ws * 64 * NJ + j * 64 + lane;
    const int64_t e0 = ci * EPC;
    valid[j] = (int)(e0 < m ? (m - e0 < EPC ? m - e0 : EPC) : 0);
  }
  const int qlen = W * 64 * NJ * EPC;
  if constexpr (QL) {
    for (int x = threadIdx.x * 4; x < qlen; x += 256 * 4) {
      *(float4 *)(qz_lds + x) = *(const float4 *)(q32 + x);
      *(float4 *)(qz_lds + qlen + x) = *(const float4 *)(z32 + x);
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int64_t e0 = ((int64_t)ws * 64 * NJ + j * 64 + lane) * EPC;
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
  }
  const char *lane_off[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
    lane_off[j] = abase + ((int64_t)ws * 64 * NJ + j * 64 + lane) * 16;

  double best = -INFINITY;
  int64_t besti = kNoIdx;

  for (;;) {
    // next super-group of TEAMS * G columns from the work queue
    if (threadIdx.x == 0) sg_s = (int64_t)atomicAdd(&st->cnt[3], 1u);
    __syncthreads();
    const int64_t sg = sg_s;
    __syncthreads();
    if (sg >= nsuper) break;
    const int64_t grp = sg * TEAMS + team;
    const int64_t col0 = grp * G;
    const int ncol = grp < ngroups ? (int)((n - col0) < G ? (n - col0) : G) : 0;
    float mw = 0.f, mz = 0.f;
    if (!rescore && ncol > 0) {
      uint4 cur[U][NJ], nxt[U][NJ];
      auto fetch = [&](int c0, uint4 (&buf)[U][NJ]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool cv = (c0 + u) < ncol;
          const int64_t cb = (col0 + c0 + u) * col_bytes;
#pragma unroll
          for (int j = 0; j < NJ; ++j)
            buf[u][j] = (cv && valid[j] > 0) ? load_chunk<NT>(lane_off[j] + cb)
                                             : make_uint4(0u, 0u, 0u, 0u);
        }
      };
      fetch(0, cur);
      for (int c0 = 0; c0 < ncol; c0 += U) {
        if (c0 + U < ncol) fetch(c0 + U, nxt);  // in flight while this group reduces
#pragma unroll
        for (int u = 0; u < U; ++u) {
          float dq = 0.f, dz = 0.f;
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            float v[EPC];
            decode_chunk<DT>(cur[u][j], v);
            if (valid[j] < EPC) {
#pragma unroll
              for (int e = 0; e < EPC; ++e)
                if (e >= valid[j]) v[e] = 0.f;
            }
            if constexpr (QL) {
              const int64_t e0 = ((int64_t)ws * 64 * NJ + j * 64 + lane) * EPC;
#pragma unroll
              for (int e = 0; e < EPC; e += 4) {
                const float4 a = *(const float4 *)(qz_lds + e0 + e);
                const float4 b = *(const float4 *)(qz_lds + qlen + e0 + e);
                dq = fmaf(v[e], a.x, dq);
                dq = fmaf(v[e + 1], a.y, dq);
                dq = fmaf(v[e + 2], a.z, dq);
                dq = fmaf(v[e + 3], a.w, dq);
                dz = fmaf(v[e], b.x, dz);
                dz = fmaf(v[e + 1], b.y, dz);
                dz = fmaf(v[e + 2], b.z, dz);
                dz = fmaf(v[e + 3], b.w, dz);
              }
            } else {
#pragma unroll
              for (int e = 0; e < EPC; ++e) {
                dq = fmaf(v[e], qv[j][e], dq);
                dz = fmaf(v[e], zv[j][e], dz);
              }
            }
          }
          dq = wave_sum(dq);
          dz = wave_sum(dz);
          if (lane == c0 + u) {
            mw = dq;
            mz = dz;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int j = 0; j < NJ; ++j) cur[u][j] = nxt[u][j];
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
    st->cnt[3] = 0;
    bi_s[0] = bi;
  }
  __syncthreads();
  // the next pick's column, decoded to FP64, for the next Gram-Schmidt step
  const int64_t pn = bi_s[0];
  if (pn != kNoIdx) {
    const double sp = col_scale(A, pn);
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) ap64[j] = sp * (double)load_elem(A, pn, j);
  }
}

// ---------------------------------------------------------------------------
static int pow2_at_least(int64_t x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

typedef void (*StreamFn)(AView, int, const float *, const float *, double *, double *,
                         const double *, const uint8_t *, ArgPart *, DevState *, double *, int);

template <int DT, int NJ, int W, bool QL>
static StreamFn pick_nt(bool nt) {
  return nt ? (StreamFn)k_stream<DT, NJ, W, true, QL> : (StreamFn)k_stream<DT, NJ, W, false, QL>;
}

template <int DT, int NJ, bool QL>
static StreamFn pick_w(int w, bool nt) {
  switch (w) {
    case 1: return pick_nt<DT, NJ, 1, QL>(nt);
    case 2: return pick_nt<DT, NJ, 2, QL>(nt);
    case 4: return pick_nt<DT, NJ, 4, QL>(nt);
  }
  return nullptr;
}

// Register-resident q, z: at most 32 floats each per lane.  LDS-resident:
// up to 16 chunks per lane per column.
template <int DT, bool QL>
static StreamFn pick_nj(int nj, int w, bool nt) {
  constexpr int NJMAX = QL ? 16 : 32 / Elem<DT>::epc;
  switch (nj) {
    case 1: return pick_w<DT, 1, QL>(w, nt);
    case 2:
      if constexpr (NJMAX >= 2) return pick_w<DT, 2, QL>(w, nt);
      break;
    case 4:
      if constexpr (NJMAX >= 4) return pick_w<DT, 4, QL>(w, nt);
      break;
    case 8:
      if constexpr (NJMAX >= 8) return pick_w<DT, 8, QL>(w, nt);
      break;
    case 16:
      if constexpr (NJMAX >= 16) return pick_w<DT, 16, QL>(w, nt);
      break;
  }
  return nullptr;
}

static StreamFn pick_kernel(int dtype, int nj, int w, bool nt, bool ql) {
  switch (dtype) {
    case DT_F32: return ql ? pick_nj<DT_F32, true>(nj, w, nt) : pick_nj<DT_F32, false>(nj, w, nt);
    case DT_BF16: return ql ? pick_nj<DT_BF16, true>(nj, w, nt) : pick_nj<DT_BF16, false>(nj, w, nt);
    case DT_FP8: return ql ? pick_nj<DT_FP8, true>(nj, w, nt) : pick_nj<DT_FP8, false>(nj, w, nt);
  }
  return nullptr;
}

static size_t stream_lds(const StreamGeo &geo) {
  return geo.ql ? (size_t)2 * geo.qlen * sizeof(float) : 0;
}

// Shape of the streaming pass: rows per lane, waves per column, column group
// size, and a persistent grid of as many workgroups as fit on the chip at
// once (work is handed out through an atomic queue, so uneven column counts
// do not leave a partial last round).  The grid is an upper bound until
// stream_finalize() knows the occupancy of the chosen kernel.
StreamGeo stream_geometry(int64_t m, int64_t n, int dtype, int num_cu, int ql) {
  StreamGeo geo{};
  const int epc = 16 / dtype_bytes(dtype);
  const int nj_max = ql ? 16 : 32 / epc;  // registers: q and z at most 32 floats each per lane
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
  geo.ql = ql;
  geo.qlen = w * 64 * nj * epc;
  geo.g = 64;
  geo.nt = 1;  // measured faster: A is read once per pass
  const int teams = 4 / w;
  const int64_t nsuper = (((n + geo.g - 1) / geo.g) + teams - 1) / teams;
  const int64_t cap = 8LL * num_cu;  // upper bound: 8 workgroups (32 waves) per CU
  geo.grid = (int)(nsuper < cap ? nsuper : cap);
  if (geo.grid < 1) geo.grid = 1;
  return geo;
}

hipError_t stream_finalize(StreamGeo &geo, int64_t n, int dtype, int num_cu) {
  StreamFn fn = pick_kernel(dtype, geo.nj, geo.w, geo.nt != 0, geo.ql != 0);
  if (!fn) return hipErrorInvalidValue;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, 256,
                                                              stream_lds(geo));
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int teams = 4 / geo.w;
  const int64_t nsuper = (((n + geo.g - 1) / geo.g) + teams - 1) / teams;
  int64_t want = (int64_t)per_cu * num_cu;
  if (want > nsuper) want = nsuper;
  if (want > geo.grid) want = geo.grid;  // never above the workspace's partial count
  geo.grid = (int)(want < 1 ? 1 : want);
  return hipSuccess;
}

hipError_t launch_stream(const StreamGeo &geo, const AView &A, const float *q32,
                         const float *z32, double *f, double *g, const double *g0,
                         uint8_t *mask, ArgPart *part, DevState *st, double *ap64,
                         int score_only, hipStream_t s) {
  StreamFn fn = pick_kernel(A.dtype, geo.nj, geo.w, geo.nt != 0, geo.ql != 0);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(geo.grid), dim3(256), stream_lds(geo), s, A, geo.g, q32, z32, f, g, g0, mask,
                     part, st, ap64, score_only);
  return hipGetLastError();
}

}  // namespace gcss
