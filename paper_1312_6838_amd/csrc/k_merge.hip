// Algorithm 4's second phase (the selection over the pooled picks) for a
// small pool, in the recursive form of Algorithm 3 over the pool's own
// matrices (Theorem 4):
//   G = A0^T A0 (P x P) and H = A0^T B (P x r), once, in FP64;
//   initial scores f_i = ||H_i||^2, g_i = G_ii;
//   per step, with p the pick and wp_s = omega^(s)_p:
//     delta_i   = G_pi - sum_s omega^(s)_i wp_s        (residual Gram column)
//     upsilon_c = (H_pc - sum_s upsilon^(s)_c wp_s) / sqrt(delta_p)
//     omega_i   = delta_i / sqrt(delta_p)
//     hu_i      = H_i . upsilon - sum_s omega^(s)_i (upsilon^(s) . upsilon)
//     f_i      <- f_i - 2 omega_i hu_i + ||upsilon||^2 omega_i^2
//     g_i      <- g_i - omega_i^2
//   and the argmax of f_i / g_i for the next pick.
// A pick with delta_p <= tau g0_p (dependent up to rounding) is dropped and
// the search repeated, as in the main selection.  The whole step is one
// launch: every workgroup recomputes the few shared quantities (delta_p,
// upsilon, ||upsilon||^2, upsilon^(s) . upsilon) with identical code, so all
// of them see the same bits, updates its slice of candidates, and the last
// workgroup to finish reduces the argmax and records the pick.  The pool is
// small (its Gram matrix is read one row per step), so a step costs about
// one launch instead of a streaming pass plus six chain kernels.
#include "gcss_device.h"

namespace gcss {

constexpr int kMT = 64;  // Gram tile edge
constexpr int kMK = 32;  // contraction chunk
constexpr int kMergeCPW = 32;  // candidates per workgroup of a step (8 lanes each)

// Element k of pool column c as stored (binary32, or the BF16 / E4M3 code),
// and its decoded, scaled value.
template <int DT>
struct PoolRaw;
template <> struct PoolRaw<DT_F32> { using T = float; };
template <> struct PoolRaw<DT_BF16> { using T = uint16_t; };
template <> struct PoolRaw<DT_FP8> { using T = uint8_t; };
template <int DT>
__device__ __forceinline__ typename PoolRaw<DT>::T pool_raw(const MergeArgs &a, int64_t c, int64_t k) {
  return ((const typename PoolRaw<DT>::T *)a.a0)[c * a.lda + k];
}
// (sc: the column's FP8 scale; 1 otherwise)
template <int DT>
__device__ __forceinline__ double pool_dec(typename PoolRaw<DT>::T v, double sc) {
  if constexpr (DT == DT_F32) {
    return (double)v;
  } else if constexpr (DT == DT_BF16) {
    return (double)__uint_as_float((uint32_t)v << 16);
  } else {
    f32x2 d = __builtin_amdgcn_cvt_pk_f32_fp8((uint32_t)v, false);
    return sc * (double)d[0];
  }
}

// GH[i][j] = pool column i . Y_j, Y_j = pool column j (j < P) or target
// column j - P; 64 x 64 tiles, FP64, fixed summation order (chunks of 32
// rows in order).  G comes out exactly symmetric: entries (i, j) and (j, i)
// multiply the same pairs in the same order.  A chunk's loads come from
// clamped in-range addresses, all issued before any is used, and entries
// outside the matrices are zeroed as they go to LDS; a tile takes its Y
// columns from the pool, the target, or (the one tile that straddles
// j = P) both.
template <int DT>
__global__ __launch_bounds__(256) void k_pool_gh(MergeArgs a) {
  using RT = typename PoolRaw<DT>::T;
  __shared__ double xs[kMK][kMT + 1];
  __shared__ double ys[kMK][kMT + 1];
  const int64_t i0 = (int64_t)blockIdx.x * kMT, j0 = (int64_t)blockIdx.y * kMT;
  const int64_t P = a.P, m = a.m, ncol = a.P + a.r;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int lr = threadIdx.x & 31, lc = threadIdx.x >> 5;
  // (the same in the whole workgroup) where the tile's Y columns live
  const bool ypool = j0 + kMT <= P, ytarget = j0 >= P;
  // this thread's columns (clamped into range) and their FP8 scales
  int64_t xc[8], yc[8];
  double xsc[8], ysc[8];
#pragma unroll
  for (int x = 0; x < 8; ++x) {
    const int64_t ci = i0 + lc + 8 * x, cj = j0 + lc + 8 * x;
    xc[x] = ci < P ? ci : P - 1;
    yc[x] = cj < P ? cj : P - 1;
    xsc[x] = DT == DT_FP8 ? (double)a.sc0[xc[x]] : 1.0;
    ysc[x] = DT == DT_FP8 ? (double)a.sc0[yc[x]] : 1.0;
  }
  double acc[4][4] = {};
  for (int64_t kb = 0; kb < m; kb += kMK) {
    const int64_t k = kb + lr;
    const int64_t kc = k < m ? k : m - 1;
    RT xr[8], yp[8];
    float yb[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const int64_t cj = j0 + lc + 8 * x;
      xr[x] = pool_raw<DT>(a, xc[x], kc);
      if (!ytarget) yp[x] = pool_raw<DT>(a, yc[x], kc);
      if (!ypool) {
        const int64_t bj = cj < P ? 0 : (cj < ncol ? cj - P : a.r - 1);
        yb[x] = a.B[bj * a.ldb + kc];
      }
    }
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const int cc = lc + 8 * x;
      const int64_t ci = i0 + cc, cj = j0 + cc;
      xs[lr][cc] = (k < m && ci < P) ? pool_dec<DT>(xr[x], xsc[x]) : 0.0;
      double yv;
      if (ypool)
        yv = pool_dec<DT>(yp[x], ysc[x]);
      else if (ytarget)
        yv = (double)yb[x];
      else
        yv = cj < P ? pool_dec<DT>(yp[x], ysc[x]) : (double)yb[x];
      ys[lr][cc] = (k < m && cj < ncol) ? yv : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kMK; ++kk) {
      double u[4], v[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        u[x] = xs[kk][ty + 16 * x];
        v[x] = ys[kk][tx + 16 * x];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fma(u[x], v[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int64_t i = i0 + ty + 16 * x;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int64_t j = j0 + tx + 16 * y;
      if (i < P && j < ncol) a.GH[i * a.ldgh + j] = acc[x][y];
    }
  }
}

// Initial scores and state of the merge selection.
__global__ void k_merge_init(MergeArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.P) {
    const double *row = a.GH + i * a.ldgh;
    double f = 0.0;
    for (int c = 0; c < a.r; ++c) f = fma(row[a.P + c], row[a.P + c], f);
    a.f[i] = f;
    a.g[i] = row[i];
    a.g0[i] = row[i];
    a.excl[i] = 0;
  }
  if (blockIdx.x == 0) {
    const double F = *a.F0;
    for (int x = threadIdx.x; x < a.k; x += blockDim.x) a.loc[x] = -1;
    for (int x = threadIdx.x; x <= a.k; x += blockDim.x) a.obj[x] = F;
    if (threadIdx.x == 0) {
      DevState *st = a.st;
      st->t = 0;
      st->k = a.k;
      st->done = a.k < 1;
      st->exhausted = 0;
      st->skip = 0;
      st->n_reject = 0;
      st->pos = 0;
      st->dec_pending = 0;
      st->p = -1;
      st->F = F;
      st->u2 = 0.0;
      st->enorm2 = 0.0;
      st->tau = a.tau;
      for (int x = 0; x < 16; ++x) st->cnt[x] = 0;
      *a.ns = 0;
    }
  }
}

// The eight lanes of a candidate's group added by a butterfly (every lane of
// the group gets the same bits).
__device__ __forceinline__ double group_sum(double v) {
  v += __shfl_xor(v, 4, kWave);
  v += __shfl_xor(v, 2, kWave);
  v += __shfl_xor(v, 1, kWave);
  return v;
}

constexpr int kMPre = 16;  // history / target entries per lane held in registers

// A lane's share of a candidate's history: W[s][i] for s = gl + 8 u (u <
// kMPre), loaded at once; later entries are read when used.
struct HistRow {
  double v[kMPre];
};

__device__ __forceinline__ void hist_load(const double *__restrict__ W, int64_t P, int64_t i,
                                          int t, int gl, HistRow &h) {
#pragma unroll
  for (int u = 0; u < kMPre; ++u) {
    const int s = gl + 8 * u;
    h.v[u] = s < t ? W[(int64_t)s * P + i] : 0.0;
  }
}

// sum over s < t of W[s][i] c[s]: lane gl takes s = gl, gl + 8, ... in order
// (the first kMPre of them from h), then the group's butterfly
__device__ __forceinline__ double hist_dot(const HistRow &h, const double *__restrict__ W,
                                           int64_t P, int64_t i, const double *c, int t,
                                           int gl) {
  double d = 0.0;
#pragma unroll
  for (int u = 0; u < kMPre; ++u) {
    const int s = gl + 8 * u;
    if (s < t) d = fma(h.v[u], c[s], d);
  }
  for (int s = gl + 8 * kMPre; s < t; s += 8) d = fma(W[(int64_t)s * P + i], c[s], d);
  return group_sum(d);
}

// One step of the merge selection (see the file comment); grid: ceil(P / 32)
// workgroups of 256 threads, 8 lanes per candidate.  Every load that does
// not depend on this step's upsilon (the candidates' histories, rows of H
// and G, scores) is issued at the start, so the step costs a few dependent
// rounds: the pick's history, delta_p, upsilon, its products, the argmax.
__global__ __launch_bounds__(256) void k_merge_step(MergeArgs a) {
  extern __shared__ double sh[];  // wp (k), upsilon (r), y (k), upsilon halves (2r)
  __shared__ double wred[4];
  __shared__ double dps;
  __shared__ double bs[4];
  __shared__ int64_t bi_s[4];
  DevState *st = a.st;
  if (st->done) return;
  const int t = st->t;
  const int64_t p = st->p;
  const double tau = st->tau;
  const int64_t P = a.P;
  const int r = a.r;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = threadIdx.x >> 3, gl = threadIdx.x & 7;
  double *wp = sh, *ups = sh + a.k, *y = ups + r, *uh = y + a.k;
  const double *Gp = a.GH + (p >= 0 ? p : 0) * a.ldgh;  // row p: G_p., then H_p.

  // this workgroup's candidate (8 lanes each) and its loads
  const int64_t i = (int64_t)blockIdx.x * kMergeCPW + grp;
  const int64_t ic = i < P ? i : P - 1;
  double f = a.f[ic], g = a.g[ic];
  const double g0 = a.g0[ic];
  int ex = a.excl[ic];
  HistRow hw;
  double hv[kMPre];
  double gpi = 0.0;
  if (p >= 0) {
    hist_load(a.W, P, ic, t, gl, hw);
    const double *Hi = a.GH + ic * a.ldgh + P;
#pragma unroll
    for (int u = 0; u < kMPre; ++u) {
      const int c = gl + 8 * u;
      hv[u] = c < r ? Hi[c] : 0.0;
    }
    gpi = Gp[ic];
  }

  bool upd = false, rej = false;
  double un = 0.0, sq = 1.0;
  if (p >= 0) {
    for (int s2 = threadIdx.x; s2 < t; s2 += blockDim.x) wp[s2] = a.W[(int64_t)s2 * P + p];
    __syncthreads();
    if (grp == 0) {
      // delta_p, with the same lanes and order as the candidate p's own delta
      HistRow hp;
#pragma unroll
      for (int u = 0; u < kMPre; ++u) {
        const int s2 = gl + 8 * u;
        hp.v[u] = s2 < t ? wp[s2] : 0.0;
      }
      const double d = hist_dot(hp, a.W, P, p, wp, t, gl);
      if (gl == 0) dps = Gp[p] - d;
    }
    __syncthreads();
    const double dp = dps;
    if (!(isfinite(dp) && dp > tau * a.g0[p])) {
      rej = true;
    } else {
      upd = true;
      sq = sqrt(dp);
      // upsilon_c = (H_pc - sum_s U[s][c] wp[s]) / sqrt(delta_p): two threads
      // per c, each a half of the s range (sixteen loads in flight), halves
      // added in order
      const int half = (t + 1) / 2;
      for (int x = threadIdx.x; x < 2 * r; x += blockDim.x) {
        const int c = x % r, hh = x / r;
        const int s0 = hh * half, s1 = hh ? t : half;
        double v = 0.0;
        int s2 = s0;
        for (; s2 + 16 <= s1; s2 += 16) {
          double uv[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) uv[u] = a.U[(int64_t)(s2 + u) * r + c];
#pragma unroll
          for (int u = 0; u < 16; ++u) v = fma(wp[s2 + u], uv[u], v);
        }
        for (; s2 < s1; ++s2) v = fma(wp[s2], a.U[(int64_t)s2 * r + c], v);
        uh[hh * r + c] = v;
      }
      __syncthreads();
      for (int c = threadIdx.x; c < r; c += blockDim.x) ups[c] = (Gp[P + c] - (uh[c] + uh[r + c])) / sq;
      __syncthreads();
      // ||upsilon||^2, and y_s = upsilon^(s) . upsilon by eight lanes per s
      double q = 0.0;
      for (int c = threadIdx.x; c < r; c += blockDim.x) q = fma(ups[c], ups[c], q);
      q = wave_sum(q);
      if (lane == 0) wred[wave] = q;
      for (int s2 = grp; s2 < t; s2 += blockDim.x / 8) {
        const double *Us = a.U + (int64_t)s2 * r;
        double v = 0.0;
        int c = gl;
        for (; c + 8 * 7 < r; c += 8 * 8) {
          double uv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) uv[u] = Us[c + 8 * u];
#pragma unroll
          for (int u = 0; u < 8; ++u) v = fma(uv[u], ups[c + 8 * u], v);
        }
        for (; c < r; c += 8) v = fma(Us[c], ups[c], v);
        v = group_sum(v);
        if (gl == 0) y[s2] = v;
      }
      __syncthreads();
      un = ((wred[0] + wred[1]) + wred[2]) + wred[3];
      if (blockIdx.x == 0)
        for (int c = threadIdx.x; c < r; c += blockDim.x) a.U[(int64_t)t * r + c] = ups[c];
    }
  }
  // this workgroup's candidates
  double best = -INFINITY;
  int64_t bi = kNoIdx;
  if (i < P) {
    if (upd) {
      const double d = hist_dot(hw, a.W, P, i, wp, t, gl);
      const double w = (gpi - d) / sq;
      const double *Hi = a.GH + i * a.ldgh + P;
      double h1 = 0.0;
#pragma unroll
      for (int u = 0; u < kMPre; ++u) {
        const int c = gl + 8 * u;
        if (c < r) h1 = fma(hv[u], ups[c], h1);
      }
      for (int c = gl + 8 * kMPre; c < r; c += 8) h1 = fma(Hi[c], ups[c], h1);
      h1 = group_sum(h1);
      const double h2 = hist_dot(hw, a.W, P, i, y, t, gl);
      const double hu = h1 - h2;
      f = f - 2.0 * w * hu + un * w * w;
      g = g - w * w;
      if (i == p) ex = 1;
      if (gl == 0) {
        a.f[i] = f;
        a.g[i] = g;
        a.W[(int64_t)t * P + i] = w;
        if (i == p) a.excl[i] = 1;
      }
    }
    if (rej && i == p) {
      ex = 2;
      if (gl == 0) a.excl[i] = 2;
    }
    if (gl == 0 && ex == 0 && g0 > 0.0 && isfinite(f) && isfinite(g) && g > tau * g0) {
      best = f / g;
      bi = i;
    }
  }
  wave_argmax(best, bi);
  if (lane == 0) {
    bs[wave] = best;
    bi_s[wave] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = bs[0];
    int64_t x = bi_s[0];
    for (int w = 1; w < 4; ++w)
      if (better(bs[w], bi_s[w], b, x)) {
        b = bs[w];
        x = bi_s[w];
      }
    a.part[blockIdx.x].score = b;
    a.part[blockIdx.x].idx = x;
  }
  if (!last_block_arrive(&st->cnt[0])) return;
  // last workgroup: the next pick over all workgroups, and this step's record
  best = -INFINITY;
  bi = kNoIdx;
  for (int x = threadIdx.x; x < (int)gridDim.x; x += blockDim.x) {
    const double sc = a.part[x].score;
    const int64_t ix = a.part[x].idx;
    if (better(sc, ix, best, bi)) {
      best = sc;
      bi = ix;
    }
  }
  wave_argmax(best, bi);
  __syncthreads();
  if (lane == 0) {
    bs[wave] = best;
    bi_s[wave] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = bs[0];
    int64_t x = bi_s[0];
    for (int w = 1; w < 4; ++w)
      if (better(bs[w], bi_s[w], b, x)) {
        b = bs[w];
        x = bi_s[w];
      }
    int tn = t;
    if (upd) {
      const double F = st->F - un;
      st->F = F;
      st->u2 = un;
      a.obj[t + 1] = F;
      a.loc[t] = p;
      tn = t + 1;
      st->t = tn;
      *a.ns = tn;
    }
    if (rej) st->n_reject += 1;
    if (tn >= st->k) {
      st->done = 1;
    } else if (x == kNoIdx) {
      st->p = -1;
      st->exhausted = 1;
      st->done = 1;
    } else {
      st->p = x;
    }
    st->cnt[0] = 0;
  }
}

// ---------------------------------------------------------------------------
size_t merge_gram_lds_bytes(int k, int r) { return (size_t)(2 * k + 3 * r) * sizeof(double); }

hipError_t launch_merge_gram(const MergeArgs &a, int dtype, hipStream_t s) {
  const dim3 tiles((unsigned)((a.P + kMT - 1) / kMT), (unsigned)((a.P + a.r + kMT - 1) / kMT));
  switch (dtype) {
    case DT_F32: hipLaunchKernelGGL(k_pool_gh<DT_F32>, tiles, dim3(256), 0, s, a); break;
    case DT_BF16: hipLaunchKernelGGL(k_pool_gh<DT_BF16>, tiles, dim3(256), 0, s, a); break;
    case DT_FP8: hipLaunchKernelGGL(k_pool_gh<DT_FP8>, tiles, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e) return e;
  const int64_t nthr = a.P > a.k + 1 ? a.P : a.k + 1;
  hipLaunchKernelGGL(k_merge_init, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

int merge_step_groups(int64_t P) { return (int)((P + kMergeCPW - 1) / kMergeCPW); }

hipError_t launch_merge_step(const MergeArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_step, dim3((unsigned)merge_step_groups(a.P)), dim3(256),
                     merge_gram_lds_bytes(a.k, a.r), s, a);
  return hipGetLastError();
}

}  // namespace gcss
