// Per-step vector kernels of the greedy loop (steps between two streaming
// passes) and small helpers.
//
// One greedy step, q/z form (Theorem 4 restated with an orthonormal basis Q
// of the picks so far; P = Q Q^T):
//   e  = A_p - Q (Q^T A_p), repeated once on e     (Gram-Schmidt + re-orth)
//   q  = e / ||e||        -- rows final: checks ||e||^2 against tau * g0_p
//   upsilon = B^T q,  ||upsilon||^2 = the exact decrease of the objective
//   w  = B upsilon  (= B B^T q; with the Gram target w = (A A^T) q)
//   z  = w - Q (Q^T w)    -- rows final: records the pick and F_t
// "cols" kernels are the dot products Q^T v, B^T q; "rows" kernels are the
// updates v - Q c, B c.  All reductions have a fixed order.
#include <type_traits>

#include "gcss_device.h"

namespace gcss {

// Two consecutive elements of a column of M as doubles (M is FP64 or FP32).
template <typename MT>
__device__ __forceinline__ double2 load2(const MT *p) {
  if constexpr (sizeof(MT) == 8) {
    return *(const double2 *)p;
  } else {
    const float2 f = *(const float2 *)p;
    return make_double2((double)f.x, (double)f.y);
  }
}

// Column dots: one workgroup per output s; each thread owns pairs of rows
// (j, j+1) with j = 2*tid + 512*i, so a wave reads 512 contiguous bytes of
// FP32 or 1 KiB of FP64 per load and every load of a thread is issued before
// the first is used.
template <typename MT, int VSRC>
__global__ __launch_bounds__(256) void k_cols(const MT *__restrict__ M, int64_t ldm, int64_t m,
                                              int ns_from_t, int ns_add,
                                              const double *__restrict__ vec, AView A,
                                              double *__restrict__ out, int final_mode,
                                              StepBufs sb, BatchStride bs, ArgStride as) {
  __shared__ double red[4];
  {
    const int b = blockIdx.y;
    sb = shift_bufs(sb, bs, b);
    M += b * as.m;
    if (vec) vec += b * as.vec;
    out += b * as.out;
  }
  DevState *st = sb.st;
  if (st->done || st->skip) return;
  const int t = st->t;
  const int ns = (ns_from_t ? t : 0) + ns_add;
  const int s = blockIdx.x;
  if (s < ns) {
    const MT *col = M + (int64_t)s * ldm;
    double acc = 0.0;
    if constexpr (VSRC == VEC_ACOL) {
      const int64_t p = sb.pick_list ? sb.pick_list[st->pos] : st->p;
      const double ps = col_scale(A, p);
      for (int64_t j = threadIdx.x; j < m; j += 256)
        acc = fma((double)col[j], ps * (double)load_elem(A, p, j), acc);
    } else {
      const int64_t mp = m & ~(int64_t)1;
      double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
      for (int64_t j = 2 * threadIdx.x; j < mp; j += 512) {
        const double2 x = load2<MT>(col + j);
        const double2 y = *(const double2 *)(vec + j);
        a0 = fma(x.x, y.x, a0);
        a1 = fma(x.y, y.y, a1);
      }
      if ((m & 1) && threadIdx.x == 0) a0 = fma((double)col[m - 1], vec[m - 1], a0);
      acc = a0 + a1;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[s] = ((red[0] + red[1]) + red[2]) + red[3];
  }
  if (final_mode == CF_NONE) return;
  if (!last_block_arrive(&st->cnt[1])) return;
  // Last workgroup: the other workgroups' outputs are visible after the fence
  // and barrier of last_block_arrive; all threads read them (fixed-order sum).
  double u2;
  if (final_mode == CF_UPS) {
    double a = 0.0;
    for (int x = threadIdx.x; x < ns; x += blockDim.x) {
      const double v = out[x];
      a = fma(v, v, a);
    }
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    u2 = ((red[0] + red[1]) + red[2]) + red[3];
  } else {  // CF_GRAM_U2: the last coefficient is q . (C q)
    u2 = out[t];
  }
  if (threadIdx.x == 0) {
    st->u2 = u2;
    st->cnt[1] = 0;
  }
}

// Column dots, several outputs per workgroup: the vector stays in registers
// (PAIRS row pairs per thread, m <= 512 * PAIRS) and the workgroup streams
// CPW columns of M against it, so the vector is read once per CPW outputs
// instead of once per output.  Per-column partials meet in one fixed-order
// reduction at the end.
template <typename MT, int CPW, int PAIRS>
__global__ __launch_bounds__(256) void k_cols_multi(const MT *__restrict__ M, int64_t ldm,
                                                    int64_t m, int ns_from_t, int ns_add,
                                                    const double *__restrict__ vec, AView A,
                                                    double *__restrict__ out, int final_mode,
                                                    StepBufs sb, BatchStride bs, ArgStride as) {
  __shared__ double red[4][CPW];
  __shared__ double red4[4];
  {
    const int b = blockIdx.y;
    sb = shift_bufs(sb, bs, b);
    M += b * as.m;
    if (vec) vec += b * as.vec;
    out += b * as.out;
  }
  DevState *st = sb.st;
  if (st->done || st->skip) return;
  const int t = st->t;
  const int ns = (ns_from_t ? t : 0) + ns_add;
  const int s0 = blockIdx.x * CPW;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (s0 < ns) {
    double2 v[PAIRS];
#pragma unroll
    for (int i = 0; i < PAIRS; ++i) {
      const int64_t j = 2 * threadIdx.x + 512 * i;
      v[i] = j + 1 < m ? *(const double2 *)(vec + j)
                       : make_double2(j < m ? vec[j] : 0.0, 0.0);
    }
    // every load is issued before any is used: clamped (valid) columns and
    // rows, raw element pairs kept until the FMA, no branches around loads
    typedef typename std::conditional<sizeof(MT) == 8, double2, float2>::type MT2;
    MT2 xr[CPW][PAIRS];
    const int64_t jmax = m >= 2 ? ((m - 2) & ~(int64_t)1) : 0;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int sc = (s0 + c) < ns ? (s0 + c) : (ns - 1);
      const MT *col = M + (int64_t)sc * ldm;
#pragma unroll
      for (int i = 0; i < PAIRS; ++i) {
        const int64_t j = 2 * threadIdx.x + 512 * i;
        xr[c][i] = *(const MT2 *)(col + (j + 1 < m ? j : jmax));
      }
    }
    double acc[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int i = 0; i < PAIRS; ++i) {
        const int64_t j = 2 * threadIdx.x + 512 * i;
        if (j + 1 < m) {
          a0 = fma((double)xr[c][i].x, v[i].x, a0);
          a1 = fma((double)xr[c][i].y, v[i].y, a1);
        }
      }
      acc[c] = (s0 + c) < ns ? a0 + a1 : 0.0;
    }
    if (m & 1) {  // odd m: the last row (its pair is (m - 1, m)), by the thread owning it
#pragma unroll
      for (int i = 0; i < PAIRS; ++i) {
        const int64_t j = 2 * threadIdx.x + 512 * i;
        if (j == m - 1) {
#pragma unroll
          for (int c = 0; c < CPW; ++c)
            if (s0 + c < ns) acc[c] = fma((double)M[(int64_t)(s0 + c) * ldm + j], v[i].x, acc[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double w = wave_sum(acc[c]);
      if (lane == 0) red[wave][c] = w;
    }
    __syncthreads();
    if (threadIdx.x < CPW && s0 + (int)threadIdx.x < ns) {
      const int c = threadIdx.x;
      out[s0 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
  }
  if (final_mode == CF_NONE) return;
  if (!last_block_arrive(&st->cnt[1])) return;
  // last workgroup: the outputs of all workgroups are visible after the
  // fence and barrier of last_block_arrive (fixed-order sum over threads)
  double u2;
  if (final_mode == CF_UPS) {
    double a = 0.0;
    for (int x = threadIdx.x; x < ns; x += blockDim.x) {
      const double w = out[x];
      a = fma(w, w, a);
    }
    a = wave_sum(a);
    if (lane == 0) red4[wave] = a;
    __syncthreads();
    u2 = ((red4[0] + red4[1]) + red4[2]) + red4[3];
  } else {
    u2 = out[t];
  }
  if (threadIdx.x == 0) {
    st->u2 = u2;
    st->cnt[1] = 0;
  }
}

// Row updates: a workgroup owns 128 rows (each lane two consecutive rows) and
// its 16 waves split the sum over s; partial sums meet in LDS in a fixed
// order.  VSRC: -1 no base vector, VEC_F64, VEC_ACOL.
constexpr int kRowsWaves = 16;
constexpr int kRowsUnroll = 8;

template <typename MT, int VSRC>
__global__ __launch_bounds__(1024) void k_rows(const MT *__restrict__ M, int64_t ldm, int64_t m,
                                               int ns_from_t, int ns_add,
                                               const double *__restrict__ vec, AView A,
                                               const double *__restrict__ c, double *out64,
                                               float *out32, int final_mode, StepBufs sb,
                                               BatchStride bs, ArgStride as) {
  __shared__ double2 red[kRowsWaves][64];
  __shared__ double wsq[2];
  __shared__ double nrm;
  __shared__ int ok;
  {
    const int b = blockIdx.y;
    sb = shift_bufs(sb, bs, b);
    M += b * as.m;
    if (vec) vec += b * as.vec;
    c += b * as.c;
    if (out64) out64 += b * as.out;
    if (out32) out32 += b * bs.q32;
  }
  DevState *st = sb.st;
  if (st->done || st->skip) return;
  const int t = st->t;
  const int ns = (ns_from_t ? t : 0) + ns_add;
  int64_t p = 0;
  double ps = 1.0;
  if constexpr (VSRC == VEC_ACOL) {
    p = sb.pick_list ? sb.pick_list[st->pos] : st->p;
    ps = col_scale(A, p);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 128 + 2 * lane;  // rows j, j+1
  const bool full = j + 1 < m;
  double a0 = 0.0, a1 = 0.0;
  if (j < m) {
    const MT *base = M + j;
    int s = wave;
    // kRowsUnroll loads per lane in flight before the first is used
    for (; s + (kRowsUnroll - 1) * kRowsWaves < ns; s += kRowsUnroll * kRowsWaves) {
      double2 x[kRowsUnroll];
      double cc[kRowsUnroll];
#pragma unroll
      for (int u = 0; u < kRowsUnroll; ++u) {
        const int64_t off = (int64_t)(s + u * kRowsWaves) * ldm;
        x[u] = full ? load2<MT>(base + off) : make_double2((double)base[off], 0.0);
        cc[u] = c[s + u * kRowsWaves];
      }
#pragma unroll
      for (int u = 0; u < kRowsUnroll; ++u) {
        a0 = fma(x[u].x, cc[u], a0);
        a1 = fma(x[u].y, cc[u], a1);
      }
    }
    for (; s < ns; s += kRowsWaves) {
      const int64_t off = (int64_t)s * ldm;
      const double2 x = full ? load2<MT>(base + off) : make_double2((double)base[off], 0.0);
      a0 = fma(x.x, c[s], a0);
      a1 = fma(x.y, c[s], a1);
    }
  }
  red[wave][lane] = make_double2(a0, a1);
  __syncthreads();
  if (wave == 0) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int x = 0; x < kRowsWaves; ++x) {
      s0 += red[x][lane].x;
      s1 += red[x][lane].y;
    }
    double o0 = 0.0, o1 = 0.0;
    if (j < m) {
      if constexpr (VSRC < 0) {
        o0 = s0;
        o1 = s1;
      } else {
        double v0, v1 = 0.0;
        if constexpr (VSRC == VEC_ACOL) {
          v0 = ps * (double)load_elem(A, p, j);
          if (full) v1 = ps * (double)load_elem(A, p, j + 1);
        } else {
          v0 = vec[j];
          if (full) v1 = vec[j + 1];
        }
        o0 = v0 - s0;
        o1 = full ? v1 - s1 : 0.0;
      }
      if (out64) {
        out64[j] = o0;
        if (full) out64[j + 1] = o1;
      }
      if (out32) {
        out32[j] = (float)o0;
        if (full) out32[j + 1] = (float)o1;
      }
    }
    const double sq = wave_sum(o0 * o0 + o1 * o1);
    if (lane == 0 && final_mode == RF_GS2) sb.part[blockIdx.x] = sq;
  }
  if (final_mode == RF_NONE) return;
  if (!last_block_arrive(&st->cnt[2])) return;

  if (final_mode == RF_GS2) {
    // ||e||^2, basis check, q = e / ||e||
    // (the other workgroups' partials are visible after the fence and barrier
    // of last_block_arrive; fixed-order sum over all threads)
    double a = 0.0;
    for (int x = threadIdx.x; x < (int)gridDim.x; x += blockDim.x) a += sb.part[x];
    a = wave_sum(a);
    if (lane == 0) red[wave][0].x = a;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s2 = 0.0;
      for (int x = 0; x < kRowsWaves; ++x) s2 += red[x][0].x;
      const int64_t pp = sb.pick_list ? sb.pick_list[st->pos] : st->p;
      const int good = isfinite(s2) && s2 > st->tau * sb.g0[pp];
      nrm = s2;
      ok = good;
      st->enorm2 = s2;
      if (!good && !sb.advance) {
        sb.mask[pp] = 2;
        st->skip = 1;
        st->n_reject += 1;
      }
      st->cnt[2] = 0;
    }
    __syncthreads();
    if (ok) {
      const double inv = 1.0 / sqrt(nrm);
      for (int64_t jj = threadIdx.x; jj < m; jj += blockDim.x) {
        const double qv = out64[jj] * inv;
        sb.Q[(int64_t)t * sb.ldq + jj] = qv;
        sb.q64[jj] = qv;
        sb.q32[jj] = (float)qv;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0 && sb.advance) {
      // basis-only mode: walk the caller's pick list; dependent columns add nothing
      if (ok) st->t = t + 1;
      st->pos += 1;
    }
  } else if (final_mode == RF_Z) {
    if (threadIdx.x == 0) {
      const int64_t pp = st->p;
      const double F = st->F - st->u2;
      st->F = F;
      sb.obj[t + 1] = F;
      sb.idx[t] = pp;
      sb.mask[pp] = 1;
      st->t = t + 1;
      st->dec_pending = 1;
      if (t + 1 >= st->k) st->done = 1;
      st->cnt[2] = 0;
    }
  }
  (void)wsq;
}

__global__ void k_select_begin(const double *__restrict__ f0, const double *__restrict__ g0,
                               const uint8_t *__restrict__ mask0, double *__restrict__ f,
                               double *__restrict__ g, uint8_t *__restrict__ mask, int64_t n,
                               StepBufs sb, int k, int kcap, const double *F0, double tau) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    f[i] = f0[i];
    g[i] = g0[i];
    mask[i] = mask0[i];
  }
  if (blockIdx.x == 0) {
    const double F = *F0;
    for (int x = threadIdx.x; x < kcap; x += blockDim.x) sb.idx[x] = -1;
    for (int x = threadIdx.x; x <= kcap; x += blockDim.x) sb.obj[x] = F;
    if (threadIdx.x == 0) {
      DevState *st = sb.st;
      st->t = 0;
      st->k = k;
      st->done = 0;
      st->exhausted = 0;
      st->skip = 0;
      st->n_reject = 0;
      st->pos = 0;
      st->dec_pending = 0;
      st->p = -1;
      st->F = F;
      st->u2 = 0.0;
      st->enorm2 = 0.0;
      st->tau = tau;
      for (int x = 0; x < 16; ++x) st->cnt[x] = 0;
    }
  }
}

__global__ void k_finish(StepBufs sb, int k, int64_t *idx_out, double *obj_out,
                         int32_t *nsel_out) {
  const int t = sb.st->t;
  for (int s = threadIdx.x; s < k; s += blockDim.x) {
    if (idx_out) idx_out[s] = s < t ? sb.idx[s] : -1;
    if (obj_out) obj_out[s + 1] = s < t ? sb.obj[s + 1] : sb.obj[t];
  }
  if (threadIdx.x == 0) {
    if (obj_out) obj_out[0] = sb.obj[0];
    if (nsel_out) *nsel_out = t;
  }
}

// Fixed-order FP64 sum by one workgroup.
__global__ __launch_bounds__(256) void k_sum_f64(const double *__restrict__ x, int64_t n,
                                                 double *out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// out[b] = fixed-order sum of x[off[b] .. off[b + 1]), one workgroup per segment
__global__ __launch_bounds__(256) void k_seg_sum(const double *__restrict__ x,
                                                 const int64_t *__restrict__ off,
                                                 double *__restrict__ out) {
  __shared__ double red[256];
  const int64_t b0 = off[blockIdx.x], b1 = off[blockIdx.x + 1];
  double s = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// part[b] = fixed-order sum of x[b * chunk .. (b + 1) * chunk)
__global__ __launch_bounds__(256) void k_sum_chunks(const double *__restrict__ x, int64_t n,
                                                    int64_t chunk, double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t b0 = (int64_t)blockIdx.x * chunk;
  const int64_t b1 = (b0 + chunk) < n ? (b0 + chunk) : n;
  double s = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// part[c] = fixed-order sum of squares of column c of B (m x r, ld ldb)
__global__ __launch_bounds__(256) void k_sumsq_cols(const float *__restrict__ B, int64_t m,
                                                    int64_t ldb, double *__restrict__ part) {
  __shared__ double red[256];
  const float *col = B + (int64_t)blockIdx.x * ldb;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < m; j += 256) {
    const double v = col[j];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_q_to_f32(const double *__restrict__ Q, int64_t ldq, int64_t m, int k,
                           float *__restrict__ Q32, int64_t ld32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = ld32 * k;
  if (i >= total) return;
  const int64_t s = i / ld32, j = i % ld32;
  Q32[i] = j < m ? (float)Q[s * ldq + j] : 0.f;
}

__global__ void k_copy_i64(const int64_t *__restrict__ src, int64_t *__restrict__ dst,
                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_gram_err(const double *trace, const double *quad, int k, double *err) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int x = 0; x < k; ++x) s += quad[x];
    *err = *trace - s;
  }
}

__global__ void k_zero_f32(float *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <typename MT>
static hipError_t cols_t(const MT *M, int64_t ldm, int64_t m, int ns_from_t, int ns_add,
                         int max_ns, int vsrc, const double *vec, const AView &A, double *out,
                         int final_mode, const StepBufs &sb, hipStream_t s, int nprob,
                         BatchStride bs, ArgStride as) {
  // FP32 matrices with many outputs (B^T q, C q): several outputs per
  // workgroup (32 element pairs per thread in flight), while keeping at
  // least 256 workgroups
  if constexpr (sizeof(MT) == 4) {
    // (measured: B^T q at m = 8192, r = 512 16.4 -> 12.7 us; with thousands
    // of outputs, C q, one output per workgroup already streams M at ~5 TB/s)
    if (vsrc == VEC_F64 && max_ns >= 512 && max_ns < 2048 && m <= 8192) {
      const int pairs = m <= 2048 ? 4 : (m <= 4096 ? 8 : 16);
      int cpw = 32 / pairs;
      while (cpw > 1 && (max_ns + cpw - 1) / cpw < 256) cpw >>= 1;
      const dim3 grid((unsigned)((max_ns + cpw - 1) / cpw), (unsigned)nprob);
#define GCSS_CM(CPW, PAIRS)                                                                    \
  hipLaunchKernelGGL((k_cols_multi<MT, CPW, PAIRS>), grid, dim3(256), 0, s, M, ldm, m,        \
                     ns_from_t, ns_add, vec, A, out, final_mode, sb, bs, as)
      if (pairs == 4) {
        if (cpw >= 8) GCSS_CM(8, 4); else if (cpw == 4) GCSS_CM(4, 4); else if (cpw == 2) GCSS_CM(2, 4); else GCSS_CM(1, 4);
      } else if (pairs == 8) {
        if (cpw >= 4) GCSS_CM(4, 8); else if (cpw == 2) GCSS_CM(2, 8); else GCSS_CM(1, 8);
      } else {
        if (cpw >= 2) GCSS_CM(2, 16); else GCSS_CM(1, 16);
      }
#undef GCSS_CM
      return hipGetLastError();
    }
  }
  const dim3 grid((unsigned)(max_ns > 0 ? max_ns : 1), (unsigned)nprob);
  if (vsrc == VEC_ACOL)
    hipLaunchKernelGGL((k_cols<MT, VEC_ACOL>), grid, dim3(256), 0, s, M, ldm, m, ns_from_t,
                       ns_add, vec, A, out, final_mode, sb, bs, as);
  else
    hipLaunchKernelGGL((k_cols<MT, VEC_F64>), grid, dim3(256), 0, s, M, ldm, m, ns_from_t,
                       ns_add, vec, A, out, final_mode, sb, bs, as);
  return hipGetLastError();
}

hipError_t launch_cols(const double *Mq, const float *Mf, int64_t ldm, int64_t m,
                       int ns_from_t, int ns_add, int max_ns, int vsrc, const double *vec,
                       const AView &A, double *out, int final_mode, const StepBufs &sb,
                       hipStream_t s, int nprob, BatchStride bs, ArgStride as) {
  if (Mq) return cols_t<double>(Mq, ldm, m, ns_from_t, ns_add, max_ns, vsrc, vec, A, out,
                                final_mode, sb, s, nprob, bs, as);
  return cols_t<float>(Mf, ldm, m, ns_from_t, ns_add, max_ns, vsrc, vec, A, out, final_mode,
                       sb, s, nprob, bs, as);
}

template <typename MT>
static hipError_t rows_t(const MT *M, int64_t ldm, int64_t m, int ns_from_t, int ns_add,
                         int vsrc, const double *vec, const AView &A, const double *c,
                         double *out64, float *out32, int final_mode, const StepBufs &sb,
                         hipStream_t s, int nprob, BatchStride bs, ArgStride as) {
  const dim3 grid(blocks_for(m, 128), (unsigned)nprob);
  const dim3 block(64 * kRowsWaves);
  if (vsrc == VEC_ACOL)
    hipLaunchKernelGGL((k_rows<MT, VEC_ACOL>), grid, block, 0, s, M, ldm, m, ns_from_t, ns_add,
                       vec, A, c, out64, out32, final_mode, sb, bs, as);
  else if (vsrc == VEC_F64)
    hipLaunchKernelGGL((k_rows<MT, VEC_F64>), grid, block, 0, s, M, ldm, m, ns_from_t, ns_add,
                       vec, A, c, out64, out32, final_mode, sb, bs, as);
  else
    hipLaunchKernelGGL((k_rows<MT, -1>), grid, block, 0, s, M, ldm, m, ns_from_t, ns_add, vec, A,
                       c, out64, out32, final_mode, sb, bs, as);
  return hipGetLastError();
}

hipError_t launch_rows(const double *Mq, const float *Mf, int64_t ldm, int64_t m,
                       int ns_from_t, int ns_add, int vsrc, const double *vec, const AView &A,
                       const double *c, double *out64, float *out32, int final_mode,
                       const StepBufs &sb, hipStream_t s, int nprob, BatchStride bs,
                       ArgStride as) {
  if (Mq) return rows_t<double>(Mq, ldm, m, ns_from_t, ns_add, vsrc, vec, A, c, out64, out32,
                                final_mode, sb, s, nprob, bs, as);
  return rows_t<float>(Mf, ldm, m, ns_from_t, ns_add, vsrc, vec, A, c, out64, out32,
                       final_mode, sb, s, nprob, bs, as);
}

hipError_t launch_select_begin(const double *f0, const double *g0, const uint8_t *mask0,
                               double *f, double *g, uint8_t *mask, int64_t n,
                               const StepBufs &sb, int k, int kcap, const double *F0,
                               double tau, hipStream_t s) {
  hipLaunchKernelGGL(k_select_begin, dim3(blocks_for(n, 256)), dim3(256), 0, s, f0, g0, mask0, f,
                     g, mask, n, sb, k, kcap, F0, tau);
  return hipGetLastError();
}

hipError_t launch_finish(const StepBufs &sb, int k, int64_t *idx_out, double *obj_out,
                         int32_t *nsel_out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, sb, k, idx_out, obj_out, nsel_out);
  return hipGetLastError();
}

// Long sums in two fixed-order levels: contiguous chunks, then the chunk sums.
hipError_t launch_sum_f64(const double *x, int64_t n, double *out, double *part, int npart,
                          hipStream_t s) {
  const int64_t chunk = 8192;
  const int64_t nb = (n + chunk - 1) / chunk;
  if (nb <= 1 || part == nullptr || nb > npart) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)nb), dim3(256), 0, s, x, n, chunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, s, part, nb, out);
  return hipGetLastError();
}

hipError_t launch_seg_sum(const double *x, const int64_t *off, int nseg, double *out,
                          hipStream_t s) {
  if (nseg < 1) return hipSuccess;
  hipLaunchKernelGGL(k_seg_sum, dim3((unsigned)nseg), dim3(256), 0, s, x, off, out);
  return hipGetLastError();
}

// ||B||_F^2: one workgroup per column, then the column sums in order
hipError_t launch_sumsq_f32(const float *B, int64_t m, int64_t r, int64_t ldb, double *out,
                            double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq_cols, dim3((unsigned)r), dim3(256), 0, s, B, m, ldb, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, s, part, r, out);
  return hipGetLastError();
}

hipError_t launch_q_to_f32(const double *Q, int64_t ldq, int64_t m, int k, float *Q32,
                           int64_t ld32, hipStream_t s) {
  hipLaunchKernelGGL(k_q_to_f32, dim3(blocks_for(ld32 * k, 256)), dim3(256), 0, s, Q, ldq, m, k,
                     Q32, ld32);
  return hipGetLastError();
}

hipError_t launch_copy_i64(const int64_t *src, int64_t *dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_i64, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_gram_err(const double *trace, const double *quad, int k, double *err,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_gram_err, dim3(1), dim3(64), 0, s, trace, quad, k, err);
  return hipGetLastError();
}

hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace gcss
