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
// Work mapping (CDNA4, 64-lane wavefronts, 512-thread workgroups, one per CU):
//   * a "team" of W wavefronts streams a sequence of work units of ucol
//     consecutive columns; wave w of the team reads rows [w*S, (w+1)*S) of
//     each column, S = 64*NJ 16-byte chunks, so every load instruction of a
//     wave covers 1 KiB of one column, fully coalesced;
//   * q and z for those rows live in registers (NJ * EPC elements each);
//   * loads run ahead of the reduction through a ring of load groups;
//   * after each column the two partial dots are summed across the wave,
//     and lane c keeps the result of column c of the unit;
//   * the FP64 epilogue runs with one column per lane.
#include <type_traits>

#include "gcss_device.h"

namespace gcss {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16-byte non-temporal load of a chunk of A (A is read once per pass).
__device__ __forceinline__ uint4 load_chunk(const char *p) {
  const u32x4 v = __builtin_nontemporal_load((const u32x4 *)p);
  return make_uint4(v[0], v[1], v[2], v[3]);
}

// One workgroup of 8 waves per CU (at the kernel's occupancy of two waves per
// SIMD): two 4-wave workgroups on one CU split its bandwidth unevenly (the
// older one's loads win), which left the younger finishing alone.
constexpr int kStreamWaves = 8;
constexpr int kStreamThreads = 64 * kStreamWaves;

__device__ __forceinline__ double sum_waves(const double (&v)[kStreamWaves]) {
  double s = 0.0;
#pragma unroll
  for (int x = 0; x < kStreamWaves; ++x) s += v[x];
  return s;
}

// (FP64 sums, EX only, keep the shuffle butterfly: DPP on both halves of each
// double measured no faster)
__device__ __forceinline__ double wave_total(double v) { return wave_sum(v); }

// EX (Gram target B = A): omega_i = A_i . q is formed in FP64 from the FP64
// basis vector (every product of a decoded element and q is exact before the
// FP64 accumulation), and the pass also returns sum_i omega_i^2 = ||A^T q||^2,
// the exact decrease of the objective, in quad[t - 1].
template <int DT, int NJ, int W, int PD, bool EX>
__global__ __launch_bounds__(512) void k_stream(AView A, int ucol, const float *__restrict__ q32,
                                                const double *__restrict__ q64,
                                                const float *__restrict__ z32,
                                                double *__restrict__ f, double *__restrict__ g,
                                                const double *__restrict__ g0,
                                                const uint8_t *__restrict__ mask,
                                                ArgPart *__restrict__ part, DevState *st,
                                                double *__restrict__ ap64, int score_only,
                                                double *__restrict__ qpart,
                                                double *__restrict__ quad,
                                                float *__restrict__ emb, int64_t ldw) {
  constexpr int EPC = Elem<DT>::epc;
  constexpr int TEAMS = kStreamWaves / W;
  constexpr int U = (8 / NJ) > 0 ? (8 / NJ) : 1;  // columns per load group
  typedef typename std::conditional<EX, double, float>::type QT;  // q and omega type
  __shared__ QT redq[kStreamWaves][64];
  __shared__ float redz[kStreamWaves][64];
  __shared__ double bs[kStreamWaves];
  __shared__ int64_t bi_s[kStreamWaves];
  __shared__ double qs[kStreamWaves];

  // after the last pick (done) one more pass runs for that pick's exact
  // decrease (EX) or its row of the embedding, without scores or a next pick
  const bool qonly = (EX || emb != nullptr) && st->done && st->dec_pending;
  if (st->done && !qonly) return;
  const bool rescore = score_only || st->skip;
  // embedding: row t - 1 of W = Q^T A receives omega = A^T q_t
  float *const wrow = (emb != nullptr && !rescore) ? emb + (int64_t)(st->t - 1) * ldw : nullptr;
  const double u2 = st->u2;
  const double tau = st->tau;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int team = wave / W;
  const int ws = wave % W;
  const int64_t m = A.m, n = A.n;
  // Work units: unit su holds TEAMS * ucol consecutive columns, ucol per team
  // (ucol <= 64, a multiple of (PD + 1) * U); workgroup b takes the units
  // b * per .. b * per + per - 1 in order.  A team's loads run ahead across
  // unit boundaries, so one unit's loads are in flight while the previous
  // one is reduced.  (Shared queues of units balanced the workgroups better
  // but cost more in waits and atomics than the imbalance.)
  const int64_t nsu = (n + (int64_t)TEAMS * ucol - 1) / ((int64_t)TEAMS * ucol);
  const int64_t per = (nsu + gridDim.x - 1) / gridDim.x;
  auto unit_of = [&](int64_t kth) -> int64_t {
    const int64_t su = (int64_t)blockIdx.x * per + kth;
    return (kth < per && su < nsu) ? su : nsu;
  };
  const int gpu = ucol / U;  // load groups per unit
  const char *abase = (const char *)A.a;
  const int64_t col_bytes = A.lda * Elem<DT>::esize;

  // q, z for this lane's rows (registers); chunk j of the lane is
  // ci(j) = ws*64*NJ + 64*j + lane.
  QT qv[NJ][EPC];
  float zv[NJ][EPC];
  int valid[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t ci = (int64_t)ws * 64 * NJ + j * 64 + lane;
    const int64_t e0 = ci * EPC;
    valid[j] = (int)(e0 < m ? (m - e0 < EPC ? m - e0 : EPC) : 0);
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t e0 = ((int64_t)ws * 64 * NJ + j * 64 + lane) * EPC;
#pragma unroll
    for (int e = 0; e < EPC; e += 4) {
      if constexpr (EX) {
        const double2 a0 = *(const double2 *)(q64 + e0 + e);
        const double2 a1 = *(const double2 *)(q64 + e0 + e + 2);
        qv[j][e] = a0.x;
        qv[j][e + 1] = a0.y;
        qv[j][e + 2] = a1.x;
        qv[j][e + 3] = a1.y;
      } else {
        const float4 a = *(const float4 *)(q32 + e0 + e);
        qv[j][e] = a.x;
        qv[j][e + 1] = a.y;
        qv[j][e + 2] = a.z;
        qv[j][e + 3] = a.w;
      }
      const float4 b = *(const float4 *)(z32 + e0 + e);
      zv[j][e] = b.x;
      zv[j][e + 1] = b.y;
      zv[j][e + 2] = b.z;
      zv[j][e + 3] = b.w;
    }
  }
  // Every load is issued unconditionally (no branches around loads, so the
  // waits for a load group are exact): chunks past the end of a column read
  // its last chunk, and load groups past the end of the range read q (both
  // cache hits); their values are masked or unused.
  const int64_t nchunk = (m + EPC - 1) / EPC;
  const char *lane_off[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int64_t ci = (int64_t)ws * 64 * NJ + j * 64 + lane;
    lane_off[j] = abase + (ci < nchunk ? ci : nchunk - 1) * 16;
  }

  double best = -INFINITY;
  int64_t besti = kNoIdx;
  // loads past the last column read q (resident in L2); unused
  const char *dummy = (const char *)q32 + lane * 16;

  int64_t kth = 0;
  int64_t su_cur = unit_of(0), su_nxt = unit_of(1);

  // ring of PD + 1 load groups of U columns: PD groups stay in flight while
  // one is reduced, across unit boundaries
  uint4 buf[PD + 1][U][NJ];
  auto fetch = [&](int64_t su, int x, uint4 (&b)[U][NJ]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t col = (su * TEAMS + team) * ucol + x * U + u;
      const bool ok = su < nsu && col < n;
      const int64_t cb = col * col_bytes;
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[u][j] = load_chunk(ok ? lane_off[j] + cb : dummy);
    }
  };
  QT mw = 0;
  float mz = 0.f;
  double qacc = 0.0;  // EX: sum of omega^2 over this lane's columns
  // FULL: every chunk of every lane lies inside m, so no element is masked
  auto consume = [&](auto full_c, int x, const uint4 (&b)[U][NJ]) {
    constexpr bool FULL = decltype(full_c)::value;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      QT dq = 0;
      float dz = 0.f;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        float v[EPC];
        decode_chunk<DT>(b[u][j], v);
        if constexpr (!FULL) {
          if (valid[j] < EPC) {
#pragma unroll
            for (int e = 0; e < EPC; ++e)
              if (e >= valid[j]) v[e] = 0.f;
          }
        }
#pragma unroll
        for (int e = 0; e < EPC; ++e) {
          dq = fma((QT)v[e], qv[j][e], dq);
          dz = fmaf(v[e], zv[j][e], dz);
        }
      }
      dq = wave_total(dq);
      dz = wave_total(dz);
      const bool me = lane == x * U + u;
      mw = me ? dq : mw;
      mz = me ? dz : mz;
    }
  };
  // one instance of the unit loop for full-height chunks, one for a ragged m
  auto run = [&](auto full_c) {
  if (!rescore) {
#pragma unroll
    for (int d = 0; d < PD; ++d) fetch(su_cur, d, buf[d]);
  }

  while (su_cur < nsu) {
    const int64_t c0 = (su_cur * TEAMS + team) * ucol;  // this team's first column
    const int ncol = (int)(c0 < n ? ((n - c0) < ucol ? (n - c0) : ucol) : 0);
    // this unit's scores and state, loaded before its stream loads so that
    // using them does not wait for loads issued later
    // (unconditional loads from a clamped column: no branch, so no copies of
    // in-flight registers at a join)
    const bool mine = ws == 0 && lane < ncol;
    const int64_t col = c0 + (lane < ncol ? lane : 0);
    const int64_t colc = col < n ? col : n - 1;
    double fv = f[colc], gv = g[colc];
    const double g0v = g0[colc];
    const int mk = mask[colc];
    float sc = 1.f;
    if constexpr (DT == DT_FP8) sc = A.scale[colc];
    mw = 0;
    mz = 0.f;
    if (!rescore) {
      for (int x0 = 0; x0 < gpu; x0 += PD + 1) {
#pragma unroll
        for (int d = 0; d <= PD; ++d) {
          // x0 is a multiple of PD + 1, so load group x0 + d sits in slot d;
          // the group PD ahead may belong to the next unit
          const int xt = x0 + d + PD;
          const bool nx = xt >= gpu;
          fetch(nx ? su_nxt : su_cur, nx ? xt - gpu : xt, buf[(d + PD) % (PD + 1)]);
          consume(full_c, x0 + d, buf[d]);
          // keeps the scheduler from hoisting later loads into renamed
          // registers, which would force a full drain at the loop head
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    if constexpr (W > 1) {
      redq[wave][lane] = mw;
      redz[wave][lane] = mz;
      __syncthreads();
      if (ws == 0) {
        QT sw = 0;
        float sz = 0.f;
#pragma unroll
        for (int x = 0; x < W; ++x) {
          sw += redq[wave + x][lane];
          sz += redz[wave + x][lane];
        }
        mw = sw;
        mz = sz;
      }
    }
    // scores of this unit's columns; the preloaded values are used on every
    // path (only the stores are predicated), so their waits stay exact
    if (!rescore) {
      const double s = (double)sc;
      const double ww = s * (double)mw, y = s * (double)mz;
      fv = fv - 2.0 * ww * y + u2 * ww * ww;
      gv = gv - ww * ww;
      if constexpr (EX) qacc += mine ? ww * ww : 0.0;
      if (wrow != nullptr && mine) wrow[col] = (float)ww;
    }
    const bool elig = mine && mk == 0 && gv > tau * g0v && isfinite(fv) && isfinite(gv);
    const double scv = fv / gv;
    if (mine && !rescore && !qonly) {
      f[col] = fv;
      g[col] = gv;
    }
    if (elig && better(scv, col, best, besti)) {
      best = scv;
      besti = col;
    }
    ++kth;
    su_cur = su_nxt;
    su_nxt = unit_of(kth + 1);
    if constexpr (W > 1) __syncthreads();  // redq/redz are rewritten by the next unit
  }
  };
  if (m == (int64_t)64 * NJ * W * EPC)
    run(std::true_type{});
  else
    run(std::false_type{});

  // workgroup winner (and, EX, the workgroup's sum of omega^2, fixed order)
  wave_argmax(best, besti);
  if constexpr (EX) qacc = wave_sum(qacc);
  if (lane == 0) {
    bs[wave] = best;
    bi_s[wave] = besti;
    if constexpr (EX) qs[wave] = qacc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = bs[0];
    int64_t bi = bi_s[0];
    for (int x = 1; x < kStreamWaves; ++x)
      if (better(bs[x], bi_s[x], b, bi)) {
        b = bs[x];
        bi = bi_s[x];
      }
    part[blockIdx.x].score = b;
    part[blockIdx.x].idx = bi;
    if constexpr (EX) qpart[blockIdx.x] = sum_waves(qs);
  }
  if (!last_block_arrive(&st->cnt[0])) return;

  // last workgroup: the exact decrease of this step (EX) ...
  if constexpr (EX) {
    if (!rescore) {
      double a = 0.0;
      for (int x = threadIdx.x; x < (int)gridDim.x; x += blockDim.x) a += qpart[x];
      a = wave_sum(a);
      if (lane == 0) qs[wave] = a;
      __syncthreads();
      if (threadIdx.x == 0) {
        quad[st->t - 1] = sum_waves(qs);
        st->dec_pending = 0;
      }
    }
  }
  if (qonly) {
    if (threadIdx.x == 0) {
      st->dec_pending = 0;
      st->cnt[0] = 0;
    }
    return;
  }
  // a pass with a new basis vector settles its pick (the final pass above
  // then has nothing left to do)
  if (!EX && !rescore && threadIdx.x == 0) st->dec_pending = 0;
  // ... and the winner over all workgroups -> next pick
  best = -INFINITY;
  besti = kNoIdx;
  for (int x = threadIdx.x; x < (int)gridDim.x; x += blockDim.x) {
    const double s = part[x].score;  // visible after last_block_arrive
    const int64_t i = part[x].idx;
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
    for (int x = 1; x < kStreamWaves; ++x)
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
  // (16-byte chunks, four loads per thread in flight before any is used)
  const int64_t pn = bi_s[0];
  if (pn != kNoIdx) {
    const double sp = col_scale(A, pn);
    const char *colp = abase + pn * col_bytes;
    constexpr int UNR = 4;
    for (int64_t c0 = threadIdx.x; c0 < nchunk; c0 += kStreamThreads * UNR) {
      uint4 r[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int64_t c = c0 + kStreamThreads * u;
        r[u] = c < nchunk ? *(const uint4 *)(colp + c * 16) : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int64_t c = c0 + kStreamThreads * u;
        if (c < nchunk) {
          float v[EPC];
          decode_chunk<DT>(r[u], v);
#pragma unroll
          for (int e = 0; e < EPC; ++e)
            if (c * EPC + e < m) ap64[c * EPC + e] = sp * (double)v[e];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
static int pow2_at_least(int64_t x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

typedef void (*StreamFn)(AView, int, const float *, const double *, const float *, double *,
                         double *, const double *, const uint8_t *, ArgPart *, DevState *, double *,
                         int, double *, double *, float *, int64_t);

template <int DT, int NJ, int W, bool EX>
static StreamFn pick_pd(int pd) {
  return pd >= 2 ? (StreamFn)k_stream<DT, NJ, W, 2, EX> : (StreamFn)k_stream<DT, NJ, W, 1, EX>;
}

template <int DT, int NJ, bool EX>
static StreamFn pick_w(int w, int pd) {
  switch (w) {
    case 1: return pick_pd<DT, NJ, 1, EX>(pd);
    case 2: return pick_pd<DT, NJ, 2, EX>(pd);
    case 4: return pick_pd<DT, NJ, 4, EX>(pd);
  }
  return nullptr;
}

// q and z live in registers: at most 32 elements each per lane.
template <int DT, bool EX>
static StreamFn pick_nj(int nj, int w, int pd) {
  constexpr int NJMAX = 32 / Elem<DT>::epc;
  switch (nj) {
    case 1: return pick_w<DT, 1, EX>(w, pd);
    case 2:
      if constexpr (NJMAX >= 2) return pick_w<DT, 2, EX>(w, pd);
      break;
    case 4:
      if constexpr (NJMAX >= 4) return pick_w<DT, 4, EX>(w, pd);
      break;
    case 8:
      if constexpr (NJMAX >= 8) return pick_w<DT, 8, EX>(w, pd);
      break;
  }
  return nullptr;
}

static StreamFn pick_kernel(int dtype, int nj, int w, int pd, bool ex) {
  switch (dtype) {
    case DT_F32: return ex ? pick_nj<DT_F32, true>(nj, w, pd) : pick_nj<DT_F32, false>(nj, w, pd);
    case DT_BF16: return ex ? pick_nj<DT_BF16, true>(nj, w, pd) : pick_nj<DT_BF16, false>(nj, w, pd);
    case DT_FP8: return ex ? pick_nj<DT_FP8, true>(nj, w, pd) : pick_nj<DT_FP8, false>(nj, w, pd);
  }
  return nullptr;
}

// Shape of the streaming pass: rows per lane, waves per column, and a grid of
// as many workgroups as fit on the chip at once; workgroup b streams its own
// consecutive work units (about upw of them).  The grid is an upper bound
// until stream_finalize() knows the occupancy of the chosen kernels.
StreamGeo stream_geometry(int64_t m, int64_t n, int dtype, int num_cu) {
  StreamGeo geo{};
  const int epc = 16 / dtype_bytes(dtype);
  const int nj_max = 32 / epc;  // registers: q and z at most 32 elements each per lane
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
  geo.g = 64;  // column groups of the batched pass
  geo.pd = 1;
  geo.upw = 4;
  const int teams = 4 / w;
  const int64_t need = (n + teams - 1) / teams;
  const int64_t cap = 8LL * num_cu;  // upper bound: 8 workgroups (32 waves) per CU
  geo.grid = (int)(need < cap ? need : cap);
  if (geo.grid < 1) geo.grid = 1;
  geo.grid_ex = geo.grid;
  return geo;
}

// grid = occupancy x CUs (at most the partial count of the workspace), and
// the unit size for about upw units per workgroup, a multiple of the ring
static hipError_t finalize_one(const StreamGeo &geo, int64_t n, int dtype, int num_cu, bool ex,
                               int *grid, int *ucol) {
  StreamFn fn = pick_kernel(dtype, geo.nj, geo.w, geo.pd, ex);
  if (!fn) return hipErrorInvalidValue;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, kStreamThreads, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int teams = kStreamWaves / geo.w;
  const int64_t need = (n + teams - 1) / teams;
  int64_t want = (int64_t)per_cu * num_cu;
  if (want > need) want = need;
  if (want > *grid) want = *grid;
  *grid = (int)(want < 1 ? 1 : want);
  const int U = geo.nj >= 8 ? 1 : 8 / geo.nj;
  const int quantum = (geo.pd + 1) * U;
  const int64_t per = (int64_t)*grid * teams * (geo.upw > 0 ? geo.upw : 1);
  int64_t uc = (n + per - 1) / per;
  uc = ((uc + quantum - 1) / quantum) * quantum;
  const int64_t ucmax = (64 / quantum) * quantum;
  if (uc > ucmax) uc = ucmax;
  if (uc < quantum) uc = quantum;
  *ucol = (int)uc;
  return hipSuccess;
}

hipError_t stream_finalize(StreamGeo &geo, int64_t n, int dtype, int num_cu) {
  hipError_t e = finalize_one(geo, n, dtype, num_cu, false, &geo.grid, &geo.ucol);
  if (!e) e = finalize_one(geo, n, dtype, num_cu, true, &geo.grid_ex, &geo.ucol_ex);
  return e;
}

hipError_t launch_stream(const StreamGeo &geo, const AView &A, const float *q32,
                         const double *q64, const float *z32, double *f, double *g,
                         const double *g0, uint8_t *mask, ArgPart *part, DevState *st,
                         double *ap64, int score_only, double *qpart, double *quad,
                         float *emb, int64_t ldw, hipStream_t s) {
  const bool ex = qpart != nullptr;
  StreamFn fn = pick_kernel(A.dtype, geo.nj, geo.w, geo.pd, ex);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(ex ? geo.grid_ex : geo.grid), dim3(kStreamThreads), 0, s, A,
                     ex ? geo.ucol_ex : geo.ucol, q32, q64, z32, f, g, g0, mask, part, st, ap64,
                     score_only, qpart, quad, emb, ldw);
  return hipGetLastError();
}

}  // namespace gcss
