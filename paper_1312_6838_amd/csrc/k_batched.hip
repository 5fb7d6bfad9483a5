// Algorithm 4 on one GPU: the column blocks of A are independent greedy
// problems that share the target B.  They advance together: every per-step
// kernel runs with gridDim.y = number of blocks (strided buffers), and the
// fused stream below walks a table of column groups, each group inside one
// block, so one launch streams all blocks' columns.  Each group writes its
// own argmax candidate; k_block_argmax then picks every block's next column.
#include <type_traits>

#include "gcss_device.h"

namespace gcss {

template <int DT>
struct BElem;
template <>
struct BElem<DT_F32> {
  static constexpr int esize = 4, epc = 4;
};
template <>
struct BElem<DT_BF16> {
  static constexpr int esize = 2, epc = 8;
};
template <>
struct BElem<DT_FP8> {
  static constexpr int esize = 1, epc = 16;
};

template <int DT>
__device__ __forceinline__ void bdecode(const uint4 &r, float *v) {
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

typedef uint32_t bu32x4 __attribute__((ext_vector_type(4)));

// 16-byte non-temporal load (A is read once per pass)
__device__ __forceinline__ uint4 bload(const char *p) {
  const bu32x4 v = __builtin_nontemporal_load((const bu32x4 *)p);
  return make_uint4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint32_t l = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t h = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)h << 32) | l);
}

template <int DT, int NJ, int W>
__global__ __launch_bounds__(256) void k_stream_b(AView A, const GroupEnt *__restrict__ groups,
                                                  int64_t ngroups, const float *__restrict__ q32,
                                                  const float *__restrict__ z32,
                                                  int64_t qstride, double *__restrict__ f,
                                                  double *__restrict__ g,
                                                  const double *__restrict__ g0,
                                                  const uint8_t *__restrict__ mask,
                                                  ArgPart *__restrict__ gpart,
                                                  const DevState *__restrict__ stb,
                                                  uint32_t *bcnt, int score_only) {
  constexpr int EPC = BElem<DT>::epc;
  constexpr int TEAMS = 4 / W;
  constexpr int U = (8 / NJ) > 0 ? (8 / NJ) : 1;
  __shared__ float red[2][4][64];
  __shared__ int64_t sg_s;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int team = wave / W;
  const int ws = wave % W;
  const int64_t m = A.m;
  const int64_t nsuper = (ngroups + TEAMS - 1) / TEAMS;
  const char *abase = (const char *)A.a;
  const int64_t col_bytes = A.lda * BElem<DT>::esize;
  // Every load is unconditional, so the waits for a load group are exact: a
  // chunk past the end of the column reads its last chunk (masked below), a
  // column past the end of the group reads this block's q (in L2; unused).
  const int64_t nchunk = (m + EPC - 1) / EPC;
  int valid[NJ];
  const char *lane_off[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t ci = (int64_t)ws * 64 * NJ + j * 64 + lane;
    const int64_t e0 = ci * EPC;
    valid[j] = (int)(e0 < m ? (m - e0 < EPC ? m - e0 : EPC) : 0);
    lane_off[j] = abase + (ci < nchunk ? ci : nchunk - 1) * 16;
  }
  // every chunk of every lane inside m: the loop instance without masking
  const bool full = m == (int64_t)64 * NJ * W * EPC;

  // super-groups come from a shared counter; the next one is claimed while
  // the current one's epilogue runs
  if (threadIdx.x == 0) sg_s = (int64_t)atomicAdd(&bcnt[1], 1u);
  __syncthreads();
  int64_t sg = sg_s;
  while (sg < nsuper) {
    const int64_t grp = sg * TEAMS + team;
    int ncol = 0, blk = 0;
    int64_t col0 = 0;
    bool live = false, rescore = true;
    double u2 = 0.0, tau = 0.0;
    // the epilogue's inputs, loaded before the stream loads (clamped column,
    // unconditional: waiting for the stream then never waits for these)
    double fv = 0.0, gv = 0.0, g0v = 0.0;
    float scv = 1.f;
    int mk = 1;
    if (grp < ngroups) {
      // one group per team: read back as wave-uniform values, so the column
      // loop and its loads stay under uniform control flow
      const GroupEnt ge = groups[grp];
      col0 = uniform_i64(ge.col0);
      ncol = __builtin_amdgcn_readfirstlane(ge.ncol);
      blk = __builtin_amdgcn_readfirstlane(ge.blk);
      const DevState *st = stb + blk;
      live = __builtin_amdgcn_readfirstlane(st->done) == 0;
      rescore = score_only || __builtin_amdgcn_readfirstlane(st->skip) != 0;
      u2 = st->u2;
      tau = st->tau;
      if (ws == 0) {
        const int64_t colc = col0 + (lane < ncol ? lane : 0);
        fv = f[colc];
        gv = g[colc];
        g0v = g0[colc];
        mk = mask[colc];
        if constexpr (DT == DT_FP8) scv = A.scale[colc];
      }
    }
    float mw = 0.f, mz = 0.f;
    if (live && !rescore) {
      // this block's q and z
      float qv[NJ][EPC], zv[NJ][EPC];
      const float *qb = q32 + blk * qstride, *zb = z32 + blk * qstride;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int64_t e0 = ((int64_t)ws * 64 * NJ + j * 64 + lane) * EPC;
#pragma unroll
        for (int e = 0; e < EPC; e += 4) {
          const float4 a = *(const float4 *)(qb + e0 + e);
          const float4 b = *(const float4 *)(zb + e0 + e);
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
      const char *dummy = (const char *)qb + lane * 16;
      // two load groups of U columns, used in turn: one in flight while the
      // other is reduced
      uint4 b0[U][NJ], b1[U][NJ];
      auto fetch = [&](int c0, uint4 (&buf)[U][NJ]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool cv = (c0 + u) < ncol;
          const int64_t cb = (col0 + c0 + u) * col_bytes;
#pragma unroll
          for (int j = 0; j < NJ; ++j) buf[u][j] = bload(cv ? lane_off[j] + cb : dummy);
        }
      };
      auto consume = [&](auto full_c, int c0, const uint4 (&buf)[U][NJ]) {
        constexpr bool FULL = decltype(full_c)::value;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          float dq = 0.f, dz = 0.f;
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            float v[EPC];
            bdecode<DT>(buf[u][j], v);
            if constexpr (!FULL) {
              if (valid[j] < EPC) {
#pragma unroll
                for (int e = 0; e < EPC; ++e)
                  if (e >= valid[j]) v[e] = 0.f;
              }
            }
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
              dq = fmaf(v[e], qv[j][e], dq);
              dz = fmaf(v[e], zv[j][e], dz);
            }
          }
          dq = wave_total(dq);
          dz = wave_total(dz);
          const bool me = lane == c0 + u;
          mw = me ? dq : mw;
          mz = me ? dz : mz;
        }
      };
      auto run = [&](auto full_c) {
        fetch(0, b0);
        for (int c0 = 0; c0 < ncol; c0 += 2 * U) {
          fetch(c0 + U, b1);
          consume(full_c, c0, b0);
          if (c0 + U >= ncol) break;
          fetch(c0 + 2 * U, b0);
          consume(full_c, c0 + U, b1);
        }
      };
      if (full)
        run(std::true_type{});
      else
        run(std::false_type{});
    }
    // every thread has read sg_s: claim the next super-group
    __syncthreads();
    if (threadIdx.x == 0) sg_s = (int64_t)atomicAdd(&bcnt[1], 1u);
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
    if (ws == 0 && grp < ngroups) {
      double best = -INFINITY;
      int64_t besti = kNoIdx;
      if (live && lane < ncol) {
        const int64_t col = col0 + lane;
        if (!rescore) {
          const double s = (double)scv;
          const double w = s * (double)mw, y = s * (double)mz;
          fv = fv - 2.0 * w * y + u2 * w * w;
          gv = gv - w * w;
          f[col] = fv;
          g[col] = gv;
        }
        if (mk == 0 && gv > tau * g0v && isfinite(fv) && isfinite(gv)) {
          best = fv / gv;
          besti = col;
        }
      }
      wave_argmax(best, besti);
      if (lane == 0) {
        gpart[grp].score = best;
        gpart[grp].idx = besti;
      }
    }
    __syncthreads();
    sg = sg_s;
  }
  if (!last_block_arrive(&bcnt[0])) return;
  if (threadIdx.x == 0) {
    bcnt[0] = 0;
    bcnt[1] = 0;
  }
}

// One workgroup per block: winner over the block's groups -> the block's next
// pick, and that column decoded to FP64 for the next Gram-Schmidt step.
__global__ __launch_bounds__(256) void k_block_argmax(AView A, const ArgPart *__restrict__ gpart,
                                                      const int64_t *__restrict__ gfirst,
                                                      DevState *stb, double *ap64,
                                                      int64_t apstride) {
  __shared__ double bs[4];
  __shared__ int64_t bi_s[4];
  const int b = blockIdx.x;
  DevState *st = stb + b;
  if (st->done) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double best = -INFINITY;
  int64_t besti = kNoIdx;
  for (int64_t x = gfirst[b] + threadIdx.x; x < gfirst[b + 1]; x += blockDim.x) {
    const double s = gpart[x].score;
    const int64_t i = gpart[x].idx;
    if (better(s, i, best, besti)) {
      best = s;
      besti = i;
    }
  }
  wave_argmax(best, besti);
  if (lane == 0) {
    bs[wave] = best;
    bi_s[wave] = besti;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bb = bs[0];
    int64_t bi = bi_s[0];
    for (int x = 1; x < 4; ++x)
      if (better(bs[x], bi_s[x], bb, bi)) {
        bb = bs[x];
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
    bi_s[0] = bi;
  }
  __syncthreads();
  const int64_t pn = bi_s[0];
  if (pn != kNoIdx) {
    const double sp = col_scale(A, pn);
    double *ap = ap64 + b * apstride;
    for (int64_t j = threadIdx.x; j < A.m; j += blockDim.x) ap[j] = sp * (double)load_elem(A, pn, j);
  }
}

// Start of a batched selection: scores reset from the initial ones, every
// block's state cleared (block b wants kb[b] picks; a block with none is done
// from the start), outputs cleared (kbm entries per block).
__global__ void k_batch_begin(const double *__restrict__ f0, const double *__restrict__ g0,
                              const uint8_t *__restrict__ mask0, double *__restrict__ f,
                              double *__restrict__ g, uint8_t *__restrict__ mask, int64_t n,
                              DevState *stb, int nprob, const int32_t *__restrict__ kb, int kbm,
                              int64_t *idx, double *obj, int64_t iostride, const double *F0,
                              double tau, uint32_t *bcnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    f[i] = f0[i];
    g[i] = g0[i];
    mask[i] = mask0[i];
  }
  if (i < nprob) {
    DevState *st = stb + i;
    const int k = kb[i];
    st->t = 0;
    st->k = k;
    st->done = k < 1;
    st->exhausted = 0;
    st->skip = 0;
    st->n_reject = 0;
    st->pos = 0;
    st->dec_pending = 0;
    st->p = -1;
    st->F = *F0;
    st->u2 = 0.0;
    st->enorm2 = 0.0;
    st->tau = tau;
    for (int x = 0; x < 16; ++x) st->cnt[x] = 0;
    for (int x = 0; x < kbm; ++x) idx[i * iostride + x] = -1;
    for (int x = 0; x <= kbm; ++x) obj[i * iostride + x] = *F0;
  }
  if (i == 0) {
    bcnt[0] = 0;
    bcnt[1] = 0;
  }
}

// The pool of Algorithm 4's second phase as fixed slots: slot b * kbm + j
// holds block b's j-th pick, or -1 past its last one.  Empty slots become
// zero columns in the gathered matrix, which are never candidates, so the
// merge sees the picks in block order, then pick order, as if compacted.
__global__ void k_pool(const DevState *__restrict__ stb, const int64_t *__restrict__ idx,
                       int64_t iostride, int kbm, int nprob, int64_t *__restrict__ pick) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (int64_t)nprob * kbm) return;
  const int b = (int)(x / kbm), j = (int)(x % kbm);
  pick[x] = j < stb[b].t ? idx[b * iostride + j] : -1;
}

// Global index of each merge pick: out[j] = pick[loc[j]] (-1 stays -1).
__global__ void k_merge_map(const int64_t *__restrict__ loc, const int64_t *__restrict__ pick,
                            int64_t npick, int km, int64_t *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= km) return;
  const int64_t l = loc[j];
  out[j] = (l >= 0 && l < npick) ? pick[l] : -1;
}

// Pooled matrix of Algorithm 4's second phase: A0[:, j] = A[:, pick[j]] (and
// the FP8 column scale).  One workgroup per pooled column.
// Column j of a0 = column pick[j] of A (whole stored column, pad included);
// a pick outside [0, n) gives a zero column (FP8 scale 1).
__global__ void k_gather_cols(const char *__restrict__ a, int64_t col_bytes, int64_t n,
                              const float *__restrict__ scale, const int64_t *__restrict__ pick,
                              char *__restrict__ a0, float *__restrict__ scale0) {
  const int64_t j = blockIdx.x;
  const int64_t src = pick[j];
  const bool ok = src >= 0 && src < n;
  uint4 *d4 = (uint4 *)(a0 + j * col_bytes);
  if (ok) {
    const uint4 *s4 = (const uint4 *)(a + src * col_bytes);
    for (int64_t x = threadIdx.x; x < col_bytes / 16; x += blockDim.x) d4[x] = s4[x];
  } else {
    for (int64_t x = threadIdx.x; x < col_bytes / 16; x += blockDim.x) d4[x] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (threadIdx.x == 0 && scale) scale0[j] = ok ? scale[src] : 1.f;
}

// ---------------------------------------------------------------------------
typedef void (*BStreamFn)(AView, const GroupEnt *, int64_t, const float *, const float *, int64_t,
                          double *, double *, const double *, const uint8_t *, ArgPart *,
                          const DevState *, uint32_t *, int);

template <int DT, int NJ>
static BStreamFn bpick_w(int w) {
  switch (w) {
    case 1: return k_stream_b<DT, NJ, 1>;
    case 2: return k_stream_b<DT, NJ, 2>;
    case 4: return k_stream_b<DT, NJ, 4>;
  }
  return nullptr;
}

template <int DT>
static BStreamFn bpick_nj(int nj, int w) {
  constexpr int NJMAX = 32 / BElem<DT>::epc;
  switch (nj) {
    case 1: return bpick_w<DT, 1>(w);
    case 2:
      if constexpr (NJMAX >= 2) return bpick_w<DT, 2>(w);
      break;
    case 4:
      if constexpr (NJMAX >= 4) return bpick_w<DT, 4>(w);
      break;
    case 8:
      if constexpr (NJMAX >= 8) return bpick_w<DT, 8>(w);
      break;
  }
  return nullptr;
}

static BStreamFn bpick(int dtype, int nj, int w) {
  switch (dtype) {
    case DT_F32: return bpick_nj<DT_F32>(nj, w);
    case DT_BF16: return bpick_nj<DT_BF16>(nj, w);
    case DT_FP8: return bpick_nj<DT_FP8>(nj, w);
  }
  return nullptr;
}

hipError_t batched_stream_grid(const StreamGeo &geo, int dtype, int num_cu, int64_t ngroups,
                               int wg_per_cu, int *grid) {
  BStreamFn fn = bpick(dtype, geo.nj, geo.w);
  if (!fn) return hipErrorInvalidValue;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, 256, 0);
  if (e != hipSuccess) return e;
  if (wg_per_cu > 0 && per_cu > wg_per_cu) per_cu = wg_per_cu;
  if (per_cu < 1) per_cu = 1;
  const int teams = 4 / geo.w;
  const int64_t nsuper = (ngroups + teams - 1) / teams;
  int64_t want = (int64_t)per_cu * num_cu;
  if (want > nsuper) want = nsuper;
  *grid = (int)(want < 1 ? 1 : want);
  return hipSuccess;
}

hipError_t launch_stream_batched(const StreamGeo &geo, int grid, const AView &A,
                                 const GroupEnt *groups, int64_t ngroups, const float *q32,
                                 const float *z32, int64_t qstride, double *f, double *g,
                                 const double *g0, const uint8_t *mask, ArgPart *gpart,
                                 const DevState *stb, uint32_t *bcnt, int score_only,
                                 hipStream_t s) {
  BStreamFn fn = bpick(A.dtype, geo.nj, geo.w);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, s, A, groups, ngroups, q32, z32, qstride, f, g,
                     g0, mask, gpart, stb, bcnt, score_only);
  return hipGetLastError();
}

hipError_t launch_block_argmax(const AView &A, const ArgPart *gpart, const int64_t *gfirst,
                               int nprob, DevState *stb, double *ap64, int64_t apstride,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_block_argmax, dim3(nprob), dim3(256), 0, s, A, gpart, gfirst, stb, ap64,
                     apstride);
  return hipGetLastError();
}

hipError_t launch_batch_begin(const double *f0, const double *g0, const uint8_t *mask0,
                              double *f, double *g, uint8_t *mask, int64_t n, DevState *stb,
                              int nprob, const int32_t *kb, int kbm, int64_t *idx, double *obj,
                              int64_t iostride, const double *F0, double tau, uint32_t *bcnt,
                              hipStream_t s) {
  const int64_t total = n > nprob ? n : nprob;
  hipLaunchKernelGGL(k_batch_begin, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, f0, g0,
                     mask0, f, g, mask, n, stb, nprob, kb, kbm, idx, obj, iostride, F0, tau, bcnt);
  return hipGetLastError();
}

hipError_t launch_pool(const DevState *stb, const int64_t *idx, int64_t iostride, int kbm,
                       int nprob, int64_t *pick, hipStream_t s) {
  const int64_t total = (int64_t)nprob * kbm;
  if (total < 1) return hipSuccess;
  hipLaunchKernelGGL(k_pool, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, stb, idx,
                     iostride, kbm, nprob, pick);
  return hipGetLastError();
}

hipError_t launch_merge_map(const int64_t *loc, const int64_t *pick, int64_t npick, int km,
                            int64_t *out, hipStream_t s) {
  if (km < 1) return hipSuccess;
  hipLaunchKernelGGL(k_merge_map, dim3((unsigned)((km + 255) / 256)), dim3(256), 0, s, loc, pick,
                     npick, km, out);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const AView &A, const int64_t *pick, int64_t npick, void *a0,
                              float *scale0, hipStream_t s) {
  const int64_t col_bytes = A.lda * dtype_bytes(A.dtype);
  if (npick < 1) return hipSuccess;
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)npick), dim3(256), 0, s, (const char *)A.a,
                     col_bytes, A.n, A.dtype == DT_FP8 ? A.scale : nullptr, pick, (char *)a0,
                     scale0);
  return hipGetLastError();
}

}  // namespace gcss
