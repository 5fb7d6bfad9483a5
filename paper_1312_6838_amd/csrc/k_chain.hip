// The steps of one greedy pick between two streaming passes: six kernels,
// for one selection problem or, along gridDim.z, for several at once (the
// blocks of Algorithm 4, each with its own state and buffers).
//
// With Q the orthonormal FP64 basis of the t picks so far, a the pick's
// column (decoded to FP64 by the previous streaming pass), V = [w_1 .. w_t]
// the history of the target vectors w_s = B B^T q_s (for B = A: (A A^T) q_s),
// and B the explicit target (for B = A, C = A A^T in its place):
//
//   K1  dots   c1 = Q^T a                          (partials over row blocks)
//   K2  rows   e1 = a - Q c1
//   K3  dots   c2 = Q^T e1
//   K4  rows   e2 = e1 - Q c2,  ||e2||^2 per workgroup
//   K5  dots   [B^T e2 ; V^T e2]                   (B = A: [C e2 ; V^T e2])
//   K6  rows   ||e2||^2 and the basis check; with q = e2 / ||e2||:
//              upsilon = B^T q, c3 = V^T q = Q^T (B B^T q), w = B upsilon
//              (B = A: w = C q), z = w - Q c3, V[:, t] = w, Q[:, t] = q;
//              the last workgroup to finish records the pick and the
//              objective decrease ||upsilon||^2 (B = A: q . w).
//
// This is Gram-Schmidt with one re-orthogonalisation (K1-K4) and the target
// operations of Theorem 4 in the q/z form (K5-K6): omega = A^T q and
// gamma = A^T z then come from one streaming pass.  c3 is formed as V^T q
// (equal to Q^T w, since q_s^T B B^T q = w_s^T q), so it needs no reduction
// after w is known.
//
// Latency is what these kernels spend: each one reads the device state, then
// issues every load it needs at once (partials of the previous kernel, the
// rows of Q, B or V it multiplies), so a kernel costs about two memory round
// trips.  Dot kernels: workgroup (x, y) forms kDotCols column sums over rows
// [1024 y, 1024 (y + 1)), written as partials P[y][c]; a consumer adds the
// ceil(m / 1024) <= kMaxRB partials of an entry in order.  Row kernels: a
// workgroup of 1024 threads owns 32 rows and its 32 groups of 32 lanes split
// the sum over columns; partial sums meet in LDS in a fixed order.  Every
// reduction has a fixed order, so results do not depend on scheduling.
#include "gcss_device.h"

namespace gcss {

constexpr int kDotRows = 1024;  // rows per block of the dot kernels (4 consecutive per thread)
constexpr int kDotCols = 4;     // columns per dot workgroup
constexpr int kMaxRB = 8;       // row blocks of the dot kernels (m <= 8192)
constexpr int kRowRB = 32;      // rows per row-kernel workgroup
constexpr int kRowGroups = 32;  // column groups per row-kernel workgroup
constexpr int kRowThreads = kRowRB * kRowGroups;  // 1024
constexpr int kRowU = 16;       // columns per thread loaded in one round (t <= 512: one round)

template <typename T>
__device__ __forceinline__ double to_f64(T v) {
  if constexpr (sizeof(T) == 2) return (double)__uint_as_float((uint32_t)v << 16);  // bfloat16
  else return (double)v;
}

// sum over y < nrb (in order) of P[y * lp + c]: all loads in flight at once
// (unconditional: y >= nrb reads row nrb - 1 again, nrb >= 1).
__device__ __forceinline__ double psum(const double *P, int64_t lp, int nrb, int64_t c) {
  double v[kMaxRB];
#pragma unroll
  for (int y = 0; y < kMaxRB; ++y) v[y] = P[(int64_t)(y < nrb ? y : nrb - 1) * lp + c];
  double s = 0.0;
#pragma unroll
  for (int y = 0; y < kMaxRB; ++y)
    if (y < nrb) s += v[y];
  return s;
}

// Fixed-order sum of one double per thread over a 1024-thread workgroup:
// wave sums, then the 16 waves in order.  Every thread gets the total.
__device__ __forceinline__ double block_sum(double v, double *wsum) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int x = 0; x < kRowThreads / 64; ++x) s += wsum[x];
  __syncthreads();
  return s;
}

// Raw loads of four consecutive elements (p aligned to four elements), kept
// as loaded until raw_f64 turns them into doubles.
template <typename T> struct Quad;
template <> struct Quad<float> { float4 v; };
template <> struct Quad<uint16_t> { uint2 v; };  // bfloat16
template <> struct Quad<double> { double2 a, b; };
__device__ __forceinline__ void raw_load(const float *p, Quad<float> &q) { q.v = *(const float4 *)p; }
__device__ __forceinline__ void raw_load(const uint16_t *p, Quad<uint16_t> &q) { q.v = *(const uint2 *)p; }
__device__ __forceinline__ void raw_load(const double *p, Quad<double> &q) {
  q.a = *(const double2 *)p;
  q.b = *(const double2 *)(p + 2);
}
__device__ __forceinline__ void raw_f64(const Quad<float> &q, double (&o)[4]) {
  o[0] = q.v.x;
  o[1] = q.v.y;
  o[2] = q.v.z;
  o[3] = q.v.w;
}
__device__ __forceinline__ void raw_f64(const Quad<uint16_t> &q, double (&o)[4]) {
  o[0] = (double)__uint_as_float(q.v.x << 16);
  o[1] = (double)__uint_as_float(q.v.x & 0xFFFF0000u);
  o[2] = (double)__uint_as_float(q.v.y << 16);
  o[3] = (double)__uint_as_float(q.v.y & 0xFFFF0000u);
}
__device__ __forceinline__ void raw_f64(const Quad<double> &q, double (&o)[4]) {
  o[0] = q.a.x;
  o[1] = q.a.y;
  o[2] = q.b.x;
  o[3] = q.b.y;
}

// The partial dots of one workgroup: P[y * lp + c] for its kDotCols columns
// c0 .. (< cend) of one matrix M (type T, ld ldm, column c - cbase), rows of
// block y.  Every load (the column quads, then x) is issued before the first
// is used.
template <typename T>
__device__ __forceinline__ void dots_block(const T *__restrict__ M, int64_t ldm, int cbase, int c0,
                                           int cend, const double *__restrict__ x, int64_t m,
                                           double *__restrict__ P, int64_t lp,
                                           double (&red)[4][kDotCols]) {
  // four consecutive rows per thread (one 16- or 32-byte load per column);
  // a quad past m reads the last quad of the column (every leading
  // dimension is a multiple of four elements) and its terms are dropped
  const int64_t jq = (int64_t)blockIdx.y * kDotRows + 4 * threadIdx.x;
  const int64_t jb = jq < m ? jq : (m - 1) & ~(int64_t)3;
  Quad<T> raw[kDotCols];
#pragma unroll
  for (int c = 0; c < kDotCols; ++c) {
    const int cc = c0 + c < cend ? c0 + c : cend - 1;
    raw_load(M + (int64_t)(cc - cbase) * ldm + jb, raw[c]);
  }
  Quad<double> xq;
  raw_load(x + jb, xq);
  double xv[4];
  raw_f64(xq, xv);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // (a row block wholly inside m uses every term unconditionally, so no load
  // is moved under a condition)
  const bool full = (int64_t)(blockIdx.y + 1) * kDotRows <= m;
#pragma unroll
  for (int c = 0; c < kDotCols; ++c) {
    double mv[4];
    raw_f64(raw[c], mv);
    double a = 0.0;
    if (full) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a = fma(mv[u], xv[u], a);
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (jq + u < m) a = fma(mv[u], xv[u], a);
    }
    a = wave_sum(a);
    if (lane == 0) red[wave][c] = a;
  }
  __syncthreads();
  if (threadIdx.x < kDotCols && c0 + (int)threadIdx.x < cend) {
    const int c = threadIdx.x;
    P[(int64_t)blockIdx.y * lp + c0 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
  }
}

// Number of column workgroups of k_dots: the columns of M1 and those of M2
// are never mixed in one workgroup.
inline int dots_col_blocks(int nfix, int kmax) {
  return (nfix + kDotCols - 1) / kDotCols + (kmax + kDotCols - 1) / kDotCols;
}

// P[y * lp + c] = sum over rows j of block y of M_c[j] * x[j] for c < ncols,
// ncols = nfix + t: column c < nfix is column c of M1 (type T1, ld ld1; the
// target B, or C for B = A), column c >= nfix is column c - nfix of M2 (FP64,
// ld ld2).  Workgroups x < ceil(nfix / 4) take four columns of M1 each, the
// rest four columns of M2.
template <typename T1>
__global__ __launch_bounds__(256) void k_dots(const T1 *__restrict__ M1, int64_t ld1, int nfix,
                                              const double *__restrict__ M2, int64_t ld2,
                                              const double *__restrict__ x, int64_t m,
                                              double *__restrict__ P, int64_t lp,
                                              const DevState *st, int64_t s_m2, int64_t s_x,
                                              int64_t s_p) {
  __shared__ double red[4][kDotCols];
  {  // problem blockIdx.z (M1 is shared)
    const int b = blockIdx.z;
    M2 += b * s_m2;
    x += b * s_x;
    P += b * s_p;
    st += b;
  }
  if (st->done || st->skip) return;
  const int ncols = nfix + st->t;
  const int nb1 = (nfix + kDotCols - 1) / kDotCols;
  if ((int)blockIdx.x < nb1) {
    dots_block(M1, ld1, 0, (int)blockIdx.x * kDotCols, nfix, x, m, P, lp, red);
  } else {
    const int c0 = nfix + ((int)blockIdx.x - nb1) * kDotCols;
    if (c0 >= ncols) return;
    dots_block(M2, ld2, nfix, c0, ncols, x, m, P, lp, red);
  }
}

// Loads of one round of a thread's row sum: M[j + s ld] for the columns
// s = s0 + 32 u (u < kRowU), raw, all issued before any is used; a column
// s >= ns reads column ns - 1 instead, and is dropped by the caller (ns <= 0:
// nothing is read).
template <typename T>
__device__ __forceinline__ void row_loads(const T *__restrict__ col0, int64_t ld, int s0, int ns,
                                          T (&raw)[kRowU]) {
  if (ns <= 0) {  // (the same in the whole workgroup)
#pragma unroll
    for (int u = 0; u < kRowU; ++u) raw[u] = T(0);
    return;
  }
#pragma unroll
  for (int u = 0; u < kRowU; ++u) {
    const int s = s0 + kRowGroups * u;
    raw[u] = col0[(int64_t)(s < ns ? s : ns - 1) * ld];
  }
}

// The row sum of one thread: sum over columns s = g, g + 32, ... < ns of
// M[j + s ld] * c[s], the first kRowU terms from preloaded values, the rest
// (ns > 32 kRowU) loaded in further rounds.
template <typename T>
__device__ __forceinline__ double row_sum(const T *__restrict__ col0, int64_t ld, int g, int ns,
                                          const double (&pre)[kRowU], const double *c) {
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < kRowU; ++u) {
    const int s = g + kRowGroups * u;
    if (s < ns) acc = fma(pre[u], c[s], acc);
  }
  for (int s0 = g + kRowGroups * kRowU; s0 < ns; s0 += kRowGroups * kRowU) {
    T raw[kRowU];
    row_loads(col0, ld, s0, ns, raw);
#pragma unroll
    for (int u = 0; u < kRowU; ++u) {
      const int s = s0 + kRowGroups * u;
      if (s < ns) acc = fma(to_f64(raw[u]), c[s], acc);
    }
  }
  return acc;
}

// The first kRowU values of a thread's row sum (columns g + 32 u < ns; the
// others 0).  The loads are unconditional (clamped columns), so they are all
// in flight together instead of each waited for inside its own branch.
template <typename T>
__device__ __forceinline__ void row_convert(const T (&raw)[kRowU], int g, int ns,
                                            double (&pre)[kRowU]) {
#pragma unroll
  for (int u = 0; u < kRowU; ++u) pre[u] = g + kRowGroups * u < ns ? to_f64(raw[u]) : 0.0;
}
template <typename T>
__device__ __forceinline__ void row_preload(const T *__restrict__ col0, int64_t ld, int g, int ns,
                                            double (&pre)[kRowU]) {
  T raw[kRowU];
  row_loads(col0, ld, g, ns, raw);
  row_convert(raw, g, ns, pre);
}

// out = v - Q c for this workgroup's 32 rows, c[s] = sum_y P[y * lp + s]
// (s < t); NORM: Pn[blockIdx.x] = sum of out^2 over its rows.
template <bool NORM>
__global__ __launch_bounds__(1024) void k_rows_sub(const double *__restrict__ Q, int64_t ldq,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ P, int64_t lp,
                                                   int nrb, double *__restrict__ out,
                                                   double *__restrict__ Pn, int64_t m,
                                                   const DevState *st, int64_t s_q,
                                                   int64_t s_vec, int64_t s_p, int64_t s_pn) {
  extern __shared__ double cs[];  // t coefficients
  __shared__ double red[kRowGroups][kRowRB + 1];
  {  // problem blockIdx.z
    const int b = blockIdx.z;
    Q += b * s_q;
    v += b * s_vec;
    P += b * s_p;
    out += b * s_vec;
    if (NORM) Pn += b * s_pn;
    st += b;
  }
  if (st->done || st->skip) return;
  const int t = st->t;
  const int r = threadIdx.x & (kRowRB - 1), g = threadIdx.x / kRowRB;
  const int64_t j = (int64_t)blockIdx.x * kRowRB + r;
  const int64_t jc = j < m ? j : m - 1;
  // loads: this thread's first columns of Q, the base value, the coefficients
  double pre[kRowU];
  row_preload(Q + jc, ldq, g, t, pre);
  const double vj = v[jc];
  for (int s = threadIdx.x; s < t; s += kRowThreads) cs[s] = psum(P, lp, nrb, s);
  __syncthreads();
  red[g][r] = row_sum(Q + jc, ldq, g, t, pre, cs);
  __syncthreads();
  if (threadIdx.x < 64) {  // wave 0: lanes 0..31 own the rows
    double o = 0.0;
    if (threadIdx.x < kRowRB && j < m) {
      double sum = 0.0;
      for (int x = 0; x < kRowGroups; ++x) sum += red[x][r];
      o = vj - sum;
      out[j] = o;
    }
    if constexpr (NORM) {
      const double sq = wave_sum(o * o);
      if (threadIdx.x == 0) Pn[blockIdx.x] = sq;
    }
  }
}

// Arguments of the last kernel of the step (see the file comment).
struct ZArgs {
  double *Q;         // basis (read: columns < t; written: column t)
  int64_t ldq;
  double *V;         // w history, ld ldq
  const double *e2;
  const double *P;   // K5 partials: [B^T e2 ; V^T e2], or [C e2 ; V^T e2]
  int64_t lp;
  int nrb;
  const double *Pn;  // K4 norm partials
  int npn;
  double *Pu;        // q . w partials (B = A)
  const void *B;     // explicit target (TB)
  int64_t ldb;
  int r;             // explicit target width (B = A: 0)
  int nfix;          // entries of P before the V^T e2 block (r, or m for B = A)
  double *q64;
  float *q32, *z32;
  const double *g0;
  uint8_t *mask;
  int64_t *idx;
  double *obj;
  int64_t m;
  int64_t s_q, s_vec, s_p, s_pn, s_q32, s_io;  // per-problem strides (see ChainArgs)
};

// TB: element type of the explicit target (float or bfloat16 bits); GRAM:
// B = A through C = A A^T (w comes from K5's partials of C e2).
template <typename TB, bool GRAM>
__global__ __launch_bounds__(1024) void k_rows_z(ZArgs za, DevState *st) {
  extern __shared__ double sh[];  // upsilon (r) then c3 (t)
  __shared__ double redw[kRowGroups][kRowRB + 1];
  __shared__ double redz[kRowGroups][kRowRB + 1];
  __shared__ double wsum[kRowThreads / 64];
  __shared__ double wrow[kRowRB];
  {  // problem blockIdx.z (B, g0 and mask are shared)
    const int64_t b = blockIdx.z;
    za.Q += b * za.s_q;
    za.V += b * za.s_q;
    za.e2 += b * za.s_vec;
    za.q64 += b * za.s_vec;
    za.P += b * za.s_p;
    za.Pn += b * za.s_pn;
    if (za.Pu) za.Pu += b * za.s_pn;
    za.q32 += b * za.s_q32;
    za.z32 += b * za.s_q32;
    za.idx += b * za.s_io;
    za.obj += b * za.s_io;
    st += b;
  }
  if (st->done || st->skip) return;
  const int t = st->t;
  const int64_t p = st->p;
  const double thr = st->tau * za.g0[p];
  const int64_t m = za.m;
  const int r = GRAM ? 0 : za.r;
  const int rr = threadIdx.x & (kRowRB - 1), g = threadIdx.x / kRowRB;
  const int64_t j0 = (int64_t)blockIdx.x * kRowRB;
  const int64_t j = j0 + rr;
  const int64_t jc = j < m ? j : m - 1;
  // every load of the kernel at once: rows of B and Q (kept raw until the
  // row sums), e2, the norm partials, the coefficient partials
  TB braw[kRowU];
  double qraw[kRowU];
  row_loads(za.Q + jc, za.ldq, g, t, qraw);
  if constexpr (!GRAM) row_loads((const TB *)za.B + jc, za.ldb, g, r, braw);
  const double e2j = za.e2[jc];
  double pn = 0.0;
  for (int x = threadIdx.x; x < za.npn; x += kRowThreads) pn += za.Pn[x];
  double *ups = sh, *c3 = sh + r;
  for (int c = threadIdx.x; c < r; c += kRowThreads) ups[c] = psum(za.P, za.lp, za.nrb, c);
  for (int s = threadIdx.x; s < t; s += kRowThreads) c3[s] = psum(za.P, za.lp, za.nrb, za.nfix + s);
  if constexpr (GRAM)
    if (threadIdx.x < kRowRB) wrow[threadIdx.x] = psum(za.P, za.lp, za.nrb, jc);
  // ||e2||^2 in a fixed order (the same in every workgroup)
  const double nrm2 = block_sum(pn, wsum);
  // the basis check: a pick whose exact residual is at most tau * g0_p is
  // dropped (every workgroup takes the same decision from the same sum)
  if (!(isfinite(nrm2) && nrm2 > thr)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      za.mask[p] = 2;
      st->skip = 1;
      st->n_reject += 1;
      st->enorm2 = nrm2;
    }
    return;
  }
  const double inv = 1.0 / sqrt(nrm2);
  for (int c = threadIdx.x; c < r; c += kRowThreads) ups[c] *= inv;
  for (int s = threadIdx.x; s < t; s += kRowThreads) c3[s] *= inv;
  __syncthreads();
  // w = B upsilon and Q c3 for this workgroup's rows
  double bpre[kRowU], qpre[kRowU];
  if constexpr (!GRAM) {
    row_convert(braw, g, r, bpre);
    redw[g][rr] = row_sum((const TB *)za.B + jc, za.ldb, g, r, bpre, ups);
  }
  row_convert(qraw, g, t, qpre);
  redz[g][rr] = row_sum(za.Q + jc, za.ldq, g, t, qpre, c3);
  __syncthreads();
  if (threadIdx.x < 64) {
    double qw = 0.0;
    if (threadIdx.x < kRowRB && j < m) {
      double wj, qc = 0.0;
      if constexpr (GRAM) {
        wj = wrow[rr] * inv;
      } else {
        wj = 0.0;
        for (int x = 0; x < kRowGroups; ++x) wj += redw[x][rr];
      }
      for (int x = 0; x < kRowGroups; ++x) qc += redz[x][rr];
      const double qv = e2j * inv;
      za.Q[(int64_t)t * za.ldq + j] = qv;
      za.q64[j] = qv;
      za.q32[j] = (float)qv;
      za.V[(int64_t)t * za.ldq + j] = wj;
      za.z32[j] = (float)(wj - qc);
      qw = qv * wj;
    }
    if constexpr (GRAM) {
      const double sq = wave_sum(qw);
      if (threadIdx.x == 0) za.Pu[blockIdx.x] = sq;
    }
  }
  // the last workgroup records the pick
  if (!last_block_arrive(&st->cnt[4])) return;
  double u2;
  if constexpr (GRAM) {
    // q . w over all workgroups (visible after last_block_arrive)
    double a = 0.0;
    for (int x = threadIdx.x; x < (int)gridDim.x; x += kRowThreads) a += za.Pu[x];
    u2 = block_sum(a, wsum);
  } else {
    double a = 0.0;
    for (int c = threadIdx.x; c < r; c += kRowThreads) a = fma(ups[c], ups[c], a);
    u2 = block_sum(a, wsum);
  }
  if (threadIdx.x == 0) {
    const double F = st->F - u2;
    st->u2 = u2;
    st->enorm2 = nrm2;
    st->F = F;
    za.obj[t + 1] = F;
    za.idx[t] = p;
    za.mask[p] = 1;
    st->t = t + 1;
    st->dec_pending = 1;
    if (t + 1 >= st->k) st->done = 1;
    st->cnt[4] = 0;
  }
}

// ---------------------------------------------------------------------------
// The whole step of one small problem in one workgroup (blockIdx.x = the
// problem): for Algorithm 4's blocks, whose m, t and r are small, one
// workgroup per block does the six kernels' work with barriers in place of
// kernel boundaries, so a step of all blocks is one launch of nprob
// workgroups instead of six launches of thousands.  Same operations as
// K1-K6 (Gram-Schmidt with one re-orthogonalisation, the basis check,
// upsilon = B^T q, c3 = V^T q, w = B upsilon, z = w - Q c3, the pick's
// record); dot products are wave sums over the rows, row sums run over the
// columns in order, so every result has a fixed summation order.
constexpr int kBlkThreads = 1024;
constexpr int kBlkWaves = kBlkThreads / 64;
constexpr int kBlkMaxM = 2048;  // rows held in LDS

// sum over waves (in order) of one double per wave; every thread gets it
__device__ __forceinline__ double blk_sum(double v, double *wsum) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int x = 0; x < kBlkWaves; ++x) s += wsum[x];
  __syncthreads();
  return s;
}

// out[c] = sum_j M_c[j] x[j] for c < nc (M_c column c, ld ldm, element type
// T): wave w takes four columns at a time (w * 4 + 64 u ..), lanes stride
// the rows, sixteen loads in flight per lane.
template <typename T>
__device__ __forceinline__ void blk_dots(const T *__restrict__ M, int64_t ldm, int nc,
                                         const double *x, int64_t m, double *out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c0 = wave * 4; c0 < nc; c0 += 4 * kBlkWaves) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t j0 = lane; j0 < m; j0 += 256) {
      double xv[4];
      T v[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = j0 + 64 * u;
        xv[u] = j < m ? x[j] : 0.0;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const int c = c0 + cc < nc ? c0 + cc : nc - 1;
          v[cc][u] = M[(int64_t)c * ldm + (j < m ? j : m - 1)];
        }
      }
#pragma unroll
      for (int cc = 0; cc < 4; ++cc)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[cc] = fma(to_f64(v[cc][u]), xv[u], acc[cc]);
    }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      const double a = wave_sum(acc[cc]);
      if (lane == 0 && c0 + cc < nc) out[c0 + cc] = a;
    }
  }
}

// sum over s < ns (in order) of M[j + s ldm] * c[s], sixteen loads in flight
template <typename T>
__device__ __forceinline__ double blk_row(const T *__restrict__ M, int64_t ldm, int ns, int64_t j,
                                          const double *c) {
  double acc = 0.0;
  int s = 0;
  for (; s + 16 <= ns; s += 16) {
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = M[(int64_t)(s + u) * ldm + j];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc = fma(to_f64(v[u]), c[s + u], acc);
  }
  for (; s < ns; ++s) acc = fma(to_f64(M[(int64_t)s * ldm + j]), c[s], acc);
  return acc;
}

template <typename TB>
__global__ __launch_bounds__(kBlkThreads) void k_chain_block(ChainArgs ca) {
  extern __shared__ double lds[];  // vec (m), coefficients (kmax + 1), upsilon (r)
  __shared__ double wsum[kBlkWaves];
  const int64_t b = blockIdx.x;
  DevState *st = ca.st + b;
  if (st->done || st->skip) return;
  const int t = st->t;
  const int64_t p = st->p;
  const int64_t m = ca.m;
  const int r = (int)ca.r;
  const double *Q = ca.Q + b * ca.s_q;
  double *Qw = ca.Q + b * ca.s_q;
  double *V = ca.V + b * ca.s_q;
  const double *a = ca.a + b * ca.s_vec;
  const TB *B = (const TB *)ca.B;
  double *vec = lds, *cf = lds + m, *ups = cf + (ca.kmax + 1);
  for (int64_t j = threadIdx.x; j < m; j += kBlkThreads) vec[j] = a[j];
  __syncthreads();
  // Gram-Schmidt twice: vec <- vec - Q (Q^T vec)
  double nrm2 = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    blk_dots(Q, ca.ldq, t, vec, m, cf);
    __syncthreads();
    double sq = 0.0;
    for (int64_t j = threadIdx.x; j < m; j += kBlkThreads) {
      const double e = vec[j] - blk_row(Q, ca.ldq, t, j, cf);
      vec[j] = e;
      sq = fma(e, e, sq);
    }
    __syncthreads();
    if (pass == 1) nrm2 = blk_sum(sq, wsum);
  }
  // the basis check (the same rule as the chain's K6)
  const double thr = st->tau * ca.g0[p];
  if (!(isfinite(nrm2) && nrm2 > thr)) {
    if (threadIdx.x == 0) {
      ca.mask[p] = 2;
      st->skip = 1;
      st->n_reject += 1;
      st->enorm2 = nrm2;
    }
    return;
  }
  const double inv = 1.0 / sqrt(nrm2);
  double *q64 = ca.q64 + b * ca.s_vec;
  float *q32 = ca.q32 + b * ca.s_q32;
  for (int64_t j = threadIdx.x; j < m; j += kBlkThreads) {
    const double qv = vec[j] * inv;
    vec[j] = qv;
    Qw[(int64_t)t * ca.ldq + j] = qv;
    q64[j] = qv;
    q32[j] = (float)qv;
  }
  __syncthreads();
  // upsilon = B^T q, c3 = V^T q
  blk_dots(B, ca.ldb, r, vec, m, ups);
  blk_dots((const double *)V, ca.ldq, t, vec, m, cf);
  __syncthreads();
  double a2 = 0.0;
  for (int c = threadIdx.x; c < r; c += kBlkThreads) a2 = fma(ups[c], ups[c], a2);
  const double u2 = blk_sum(a2, wsum);
  // w = B upsilon, z = w - Q c3
  float *z32 = ca.z32 + b * ca.s_q32;
  for (int64_t j = threadIdx.x; j < m; j += kBlkThreads) {
    const double wj = blk_row(B, ca.ldb, r, j, ups);
    const double qc = blk_row(Q, ca.ldq, t, j, cf);
    V[(int64_t)t * ca.ldq + j] = wj;
    z32[j] = (float)(wj - qc);
  }
  if (threadIdx.x == 0) {
    const double F = st->F - u2;
    st->u2 = u2;
    st->enorm2 = nrm2;
    st->F = F;
    ca.obj[b * ca.s_io + t + 1] = F;
    ca.idx[b * ca.s_io + t] = p;
    ca.mask[p] = 1;
    st->t = t + 1;
    st->dec_pending = 1;
    if (t + 1 >= st->k) st->done = 1;
  }
}

size_t chain_block_lds_bytes(int64_t m, int64_t r, int kmax) {
  return (size_t)(m + kmax + 1 + r) * sizeof(double);
}

bool chain_block_fits(int64_t m, int64_t r, int kmax, size_t lds_max) {
  return m <= kBlkMaxM && chain_block_lds_bytes(m, r, kmax) <= lds_max;
}

hipError_t launch_chain_block(const ChainArgs &ca, hipStream_t s) {
  const size_t lds = chain_block_lds_bytes(ca.m, ca.r, ca.kmax);
  const unsigned np = (unsigned)(ca.nprob > 0 ? ca.nprob : 1);
  if (ca.b_bf16)
    hipLaunchKernelGGL((k_chain_block<uint16_t>), dim3(np), dim3(kBlkThreads), lds, s, ca);
  else
    hipLaunchKernelGGL((k_chain_block<float>), dim3(np), dim3(kBlkThreads), lds, s, ca);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
int chain_row_blocks(int64_t m) { return (int)((m + kDotRows - 1) / kDotRows); }
int chain_row_groups(int64_t m) { return (int)((m + kRowRB - 1) / kRowRB); }

size_t chain_lds_bytes(int64_t r, int kmax) { return (size_t)(r + kmax + 1) * sizeof(double); }

bool chain_fits(int64_t m, int64_t r, int kmax, size_t lds_max) {
  return chain_row_blocks(m) <= kMaxRB && chain_lds_bytes(r, kmax) <= lds_max;
}

hipError_t launch_chain(const ChainArgs &ca, hipStream_t s) {
  const int64_t m = ca.m;
  const int nrb = chain_row_blocks(m), nrg = chain_row_groups(m);
  if (nrb > kMaxRB) return hipErrorInvalidValue;
  const unsigned qdots = (unsigned)dots_col_blocks(0, ca.kmax);
  const size_t lds_t = (size_t)(ca.kmax + 1) * sizeof(double);
  const unsigned np = (unsigned)(ca.nprob > 0 ? ca.nprob : 1);
  // K1: c1 partials
  hipLaunchKernelGGL((k_dots<float>), dim3(qdots, nrb, np), dim3(256), 0, s, (const float *)nullptr,
                     (int64_t)0, 0, ca.Q, ca.ldq, ca.a, m, ca.P, ca.lp, ca.st, ca.s_q, ca.s_vec,
                     ca.s_p);
  // K2: e1 = a - Q c1
  hipLaunchKernelGGL((k_rows_sub<false>), dim3(nrg, 1, np), dim3(kRowThreads), lds_t, s, ca.Q,
                     ca.ldq, ca.a, ca.P, ca.lp, nrb, ca.e1, (double *)nullptr, m, ca.st, ca.s_q,
                     ca.s_vec, ca.s_p, ca.s_pn);
  // K3: c2 partials
  hipLaunchKernelGGL((k_dots<float>), dim3(qdots, nrb, np), dim3(256), 0, s, (const float *)nullptr,
                     (int64_t)0, 0, ca.Q, ca.ldq, ca.e1, m, ca.P, ca.lp, ca.st, ca.s_q, ca.s_vec,
                     ca.s_p);
  // K4: e2 = e1 - Q c2, norm partials
  hipLaunchKernelGGL((k_rows_sub<true>), dim3(nrg, 1, np), dim3(kRowThreads), lds_t, s, ca.Q,
                     ca.ldq, ca.e1, ca.P, ca.lp, nrb, ca.e2, ca.Pn, m, ca.st, ca.s_q, ca.s_vec,
                     ca.s_p, ca.s_pn);
  // K5: [B^T e2 ; V^T e2] partials (B = A: [C e2 ; V^T e2])
  const int nfix = ca.gram ? (int)m : (int)ca.r;
  const unsigned tdots = (unsigned)dots_col_blocks(nfix, ca.kmax);
  if (ca.b_bf16 && !ca.gram)
    hipLaunchKernelGGL((k_dots<uint16_t>), dim3(tdots, nrb, np), dim3(256), 0, s,
                       (const uint16_t *)ca.B, ca.ldb, nfix, ca.V, ca.ldq, ca.e2, m, ca.P, ca.lp,
                       ca.st, ca.s_q, ca.s_vec, ca.s_p);
  else
    hipLaunchKernelGGL((k_dots<float>), dim3(tdots, nrb, np), dim3(256), 0, s, (const float *)ca.B,
                       ca.ldb, nfix, ca.V, ca.ldq, ca.e2, m, ca.P, ca.lp, ca.st, ca.s_q, ca.s_vec,
                       ca.s_p);
  // K6
  ZArgs za{};
  za.Q = ca.Q;
  za.ldq = ca.ldq;
  za.V = ca.V;
  za.e2 = ca.e2;
  za.P = ca.P;
  za.lp = ca.lp;
  za.nrb = nrb;
  za.Pn = ca.Pn;
  za.npn = nrg;
  za.Pu = ca.Pu;
  za.B = ca.B;
  za.ldb = ca.ldb;
  za.r = ca.gram ? 0 : (int)ca.r;
  za.nfix = nfix;
  za.q64 = ca.q64;
  za.q32 = ca.q32;
  za.z32 = ca.z32;
  za.g0 = ca.g0;
  za.mask = ca.mask;
  za.idx = ca.idx;
  za.obj = ca.obj;
  za.m = m;
  za.s_q = ca.s_q;
  za.s_vec = ca.s_vec;
  za.s_p = ca.s_p;
  za.s_pn = ca.s_pn;
  za.s_q32 = ca.s_q32;
  za.s_io = ca.s_io;
  const size_t lds_z = (size_t)(za.r + ca.kmax + 1) * sizeof(double);
  const dim3 gz(nrg, 1, np);
  if (ca.gram)
    hipLaunchKernelGGL((k_rows_z<float, true>), gz, dim3(kRowThreads), lds_z, s, za, ca.st);
  else if (ca.b_bf16)
    hipLaunchKernelGGL((k_rows_z<uint16_t, false>), gz, dim3(kRowThreads), lds_z, s, za, ca.st);
  else
    hipLaunchKernelGGL((k_rows_z<float, false>), gz, dim3(kRowThreads), lds_z, s, za, ca.st);
  return hipGetLastError();
}

}  // namespace gcss
