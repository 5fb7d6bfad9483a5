// The steps of one greedy pick between two streaming passes, for a single
// selection problem: seven kernels.
//
// With Q the orthonormal FP64 basis of the t picks so far, a the pick's
// column (decoded to FP64 by the previous streaming pass), V = [w_1 .. w_t]
// the history of the target vectors w_s = B B^T q_s (for B = A: (A A^T) q_s),
// and B the explicit target:
//
//   K0  dots   c1 = Q^T a                      (partials over row blocks)
//   K1  rows   e1 = a - Q c1
//   K2  dots   c2 = Q^T e1
//   K3  rows   e2 = e1 - Q c2,  partial ||e2||^2 per workgroup
//   K4  dots   [B^T e2 ; V^T e2]               (B = A: V^T e2 only)
//   K5  rows   ||e2||^2, the basis check; q = e2 / ||e2||, upsilon = B^T q,
//              c3 = V^T q = Q^T (B B^T q); w = B upsilon (B = A: w = (A A^T) q),
//              z = w - Q c3, V[:, t] = w
//   K6  one workgroup records the pick and the objective decrease
//              ||upsilon||^2 (B = A: q . w).
//
// This is Gram-Schmidt with one re-orthogonalisation (K0-K3) and the target
// operations of Theorem 4 in the q/z form (K4-K5): omega = A^T q and
// gamma = A^T z then come from one streaming pass.  c3 is formed as V^T q
// (V^T q = U^T upsilon with U = B^T Q, the upsilons so far), so z needs no
// reduction after w is known.
//
// Dot kernels: workgroup (x, y) forms kDotCols column sums over rows
// [1024 y, 1024 (y + 1)), written as partials P[y][c]; the consumer adds the
// ceil(m / 1024) partials of an entry in order.  Row kernels: a workgroup of
// 1024 threads owns 32 rows and its 32 groups of 32 lanes split the sum over
// columns (eight loads in flight per thread); partial sums meet in LDS in a
// fixed order.  Every reduction has a fixed order, so
// results do not depend on scheduling.
#include "gcss_device.h"

namespace gcss {

constexpr int kDotRows = 1024;  // rows per block of the dot kernels (4 per thread)
constexpr int kDotCols = 4;     // columns per dot workgroup
constexpr int kRowRB = 32;       // rows per row-kernel workgroup
constexpr int kRowGroups = 32;   // column groups per row-kernel workgroup
constexpr int kRowThreads = kRowRB * kRowGroups;  // 1024
constexpr int kRowUnroll = 8;    // loads in flight per thread in the column sums

template <typename T>
__device__ __forceinline__ double to_f64(T v) {
  if constexpr (sizeof(T) == 2) return (double)__uint_as_float((uint32_t)v << 16);  // bfloat16
  else return (double)v;
}

// P[y * lp + c] = sum over rows j of block y of M_c[j] * x[j] for c < ncols,
// ncols = nfix + t: column c < nfix is column c of M1 (type T1, ld ld1; the
// target B), column c >= nfix is column c - nfix of M2 (FP64, ld ld2).
template <typename T1>
__global__ __launch_bounds__(256) void k_dots(const T1 *__restrict__ M1, int64_t ld1, int nfix,
                                              const double *__restrict__ M2, int64_t ld2,
                                              const double *__restrict__ x, int64_t m,
                                              double *__restrict__ P, int64_t lp,
                                              const DevState *st) {
  __shared__ double red[4][kDotCols];
  if (st->done || st->skip) return;
  const int ncols = nfix + st->t;
  const int c0 = blockIdx.x * kDotCols;
  if (c0 >= ncols) return;
  const int64_t j0 = (int64_t)blockIdx.y * kDotRows + threadIdx.x;
  double xv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t j = j0 + 256 * u;
    xv[u] = j < m ? x[j] : 0.0;
  }
  // every load issued before the first use
  double mv[kDotCols][4];
#pragma unroll
  for (int c = 0; c < kDotCols; ++c) {
    const int cc = c0 + c < ncols ? c0 + c : ncols - 1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = j0 + 256 * u;
      const int64_t jj = j < m ? j : m - 1;
      mv[c][u] = cc < nfix ? to_f64(M1[(int64_t)cc * ld1 + jj]) : M2[(int64_t)(cc - nfix) * ld2 + jj];
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < kDotCols; ++c) {
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j0 + 256 * u < m) a = fma(mv[c][u], xv[u], a);
    a = wave_sum(a);
    if (lane == 0) red[wave][c] = a;
  }
  __syncthreads();
  if (threadIdx.x < kDotCols && c0 + (int)threadIdx.x < ncols) {
    const int c = threadIdx.x;
    P[(int64_t)blockIdx.y * lp + c0 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
  }
}

// sum over columns s < ns (s = g, g + 32, ...) of M[j + s ld] * c[s] for the
// thread's row j (clamped to a valid row): kRowUnroll loads in flight.
template <typename T>
__device__ __forceinline__ double row_sum(const T *__restrict__ col0, int64_t ld, int g, int ns,
                                          const double *c) {
  double acc = 0.0;
  int s = g;
  for (; s + (kRowUnroll - 1) * kRowGroups < ns; s += kRowUnroll * kRowGroups) {
    double x[kRowUnroll];
#pragma unroll
    for (int u = 0; u < kRowUnroll; ++u) x[u] = to_f64(col0[(int64_t)(s + u * kRowGroups) * ld]);
#pragma unroll
    for (int u = 0; u < kRowUnroll; ++u) acc = fma(x[u], c[s + u * kRowGroups], acc);
  }
  for (; s < ns; s += kRowGroups) acc = fma(to_f64(col0[(int64_t)s * ld]), c[s], acc);
  return acc;
}

// out = v - Q c for this workgroup's 32 rows, c[s] = sum_y P[y * lp + s]
// (s < t); NORM: Pn[blockIdx.x] = sum of out^2 over its rows.
template <bool NORM>
__global__ __launch_bounds__(1024) void k_rows_sub(const double *__restrict__ Q, int64_t ldq,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ P, int64_t lp,
                                                   int nrb, double *__restrict__ out,
                                                   double *__restrict__ Pn, int64_t m,
                                                   const DevState *st) {
  extern __shared__ double cs[];  // t coefficients
  __shared__ double red[kRowGroups][kRowRB + 1];
  if (st->done || st->skip) return;
  const int t = st->t;
  for (int s = threadIdx.x; s < t; s += kRowThreads) {
    double c = 0.0;
    for (int y = 0; y < nrb; ++y) c += P[(int64_t)y * lp + s];
    cs[s] = c;
  }
  __syncthreads();
  const int r = threadIdx.x & (kRowRB - 1), g = threadIdx.x / kRowRB;
  const int64_t j = (int64_t)blockIdx.x * kRowRB + r;
  const int64_t jc = j < m ? j : m - 1;
  red[g][r] = row_sum(Q + jc, ldq, g, t, cs);
  __syncthreads();
  if (threadIdx.x < 64) {  // wave 0: lanes 0..31 own the rows
    double o = 0.0;
    if (threadIdx.x < kRowRB && j < m) {
      double sum = 0.0;
      for (int x = 0; x < kRowGroups; ++x) sum += red[x][r];
      o = v[j] - sum;
      out[j] = o;
    }
    if constexpr (NORM) {
      const double sq = wave_sum(o * o);
      if (threadIdx.x == 0) Pn[blockIdx.x] = sq;
    }
  }
}

// The last kernel of the step (see the file comment).  TB: element type of
// the explicit target (float or bfloat16 bits); GRAM: B = A through C = A A^T.
struct ZArgs {
  const double *Qr;  // basis (read, columns < t)
  double *Qw;        // basis column t (written)
  int64_t ldq;
  double *V;         // w history, ld ldq
  const double *e2;
  const double *P;   // K4 partials
  int64_t lp;
  int nrb;
  const double *Pn;  // K3 norm partials
  int npn;
  double *Pu;        // u2 partials (B = A)
  const void *B;     // explicit target (TB), or C (float) for B = A
  int64_t ldb;
  int r;
  double *q64;
  float *q32, *z32;
  const double *g0;
  uint8_t *mask;
  int64_t *idx;
  double *obj;
  int64_t m;
};

template <typename TB, bool GRAM>
__global__ __launch_bounds__(1024) void k_rows_z(ZArgs za, DevState *st) {
  extern __shared__ double sh[];  // upsilon (r) then c3 (t)
  __shared__ double red[kRowGroups][kRowRB + 1];
  __shared__ double bc[2];
  if (st->done || st->skip) return;
  const int t = st->t;
  const int64_t p = st->p;
  const int64_t m = za.m;
  if (threadIdx.x < 64) {  // ||e2||^2 from K3's partials: one wave, fixed order
    double s2 = 0.0;
    for (int x = threadIdx.x; x < za.npn; x += 64) s2 += za.Pn[x];
    s2 = wave_sum(s2);
    if (threadIdx.x == 0) bc[0] = s2;
  }
  __syncthreads();
  const double nrm2 = bc[0];
  // the basis check: a pick whose exact residual is at most tau * g0_p is
  // dropped (every workgroup takes the same decision from the same sum)
  if (!(isfinite(nrm2) && nrm2 > st->tau * za.g0[p])) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      za.mask[p] = 2;
      st->skip = 1;
      st->n_reject += 1;
      st->enorm2 = nrm2;
    }
    return;
  }
  const double inv = 1.0 / sqrt(nrm2);
  const int r = GRAM ? 0 : za.r;
  double *ups = sh, *c3 = sh + r;
  for (int c = threadIdx.x; c < r + t; c += kRowThreads) {
    double a = 0.0;
    for (int y = 0; y < za.nrb; ++y) a += za.P[(int64_t)y * za.lp + c];
    sh[c] = a * inv;
  }
  __syncthreads();
  const int rr = threadIdx.x & (kRowRB - 1), g = threadIdx.x / kRowRB;
  const int64_t j0 = (int64_t)blockIdx.x * kRowRB;
  const int64_t j = j0 + rr;
  const int64_t jc = j < m ? j : m - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // w for this workgroup's rows
  double wj = 0.0;
  if constexpr (GRAM) {
    // w_j = (column j of C) . e2 / ||e2|| for the 32 columns j of this
    // workgroup: thread i reads e2[i] once and row i of those columns
    const float *C = (const float *)za.B;
    double acc[kRowRB];
#pragma unroll
    for (int x = 0; x < kRowRB; ++x) acc[x] = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += kRowThreads) {
      const double e = za.e2[i];
      float cv[kRowRB];
#pragma unroll
      for (int x = 0; x < kRowRB; ++x) {
        const int64_t jj = j0 + x < m ? j0 + x : m - 1;
        cv[x] = C[jj * za.ldb + i];
      }
#pragma unroll
      for (int x = 0; x < kRowRB; ++x) acc[x] = fma((double)cv[x], e, acc[x]);
    }
    // column sums: waves first, then the 16 waves in order
#pragma unroll
    for (int x = 0; x < kRowRB; ++x) {
      const double a = wave_sum(acc[x]);
      if (lane == 0) red[wave][x] = a;
    }
    __syncthreads();
    if (threadIdx.x < kRowRB) {
      double a = 0.0;
      for (int x = 0; x < kRowThreads / 64; ++x) a += red[x][threadIdx.x];
      red[kRowGroups - 1][threadIdx.x] = a * inv;  // row 31 is past the 16 wave rows
    }
    __syncthreads();
    wj = red[kRowGroups - 1][rr];
    __syncthreads();
  } else {
    red[g][rr] = row_sum((const TB *)za.B + jc, za.ldb, g, r, ups);
    __syncthreads();
    double sum = 0.0;
    for (int x = 0; x < kRowGroups; ++x) sum += red[x][rr];
    wj = sum;
    __syncthreads();
  }
  // Q c3 for this workgroup's rows
  red[g][rr] = row_sum(za.Qr + jc, za.ldq, g, t, c3);
  __syncthreads();
  if (threadIdx.x < 64) {
    double qw = 0.0;
    if (threadIdx.x < kRowRB && j < m) {
      double sum = 0.0;
      for (int x = 0; x < kRowGroups; ++x) sum += red[x][rr];
      const double qv = za.e2[j] * inv;
      za.Qw[(int64_t)t * za.ldq + j] = qv;
      za.q64[j] = qv;
      za.q32[j] = (float)qv;
      za.V[(int64_t)t * za.ldq + j] = wj;
      za.z32[j] = (float)(wj - sum);
      qw = qv * wj;
    }
    if constexpr (GRAM) {
      const double sq = wave_sum(qw);
      if (threadIdx.x == 0) za.Pu[blockIdx.x] = sq;
    }
  }
  if constexpr (!GRAM) {
    // ||upsilon||^2 (every workgroup holds upsilon; the first one stores it)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      double u2 = 0.0;
      for (int c = 0; c < r; ++c) u2 = fma(ups[c], ups[c], u2);
      za.Pu[0] = u2;
    }
  }
}

// K6 (one workgroup, after K5): the objective decrease of the pick and the
// pick itself.  The decrease is ||upsilon||^2 (B = A: q . w, the sum of K5's
// partials in order).  Nothing to do when K5 dropped the pick.
__global__ __launch_bounds__(64) void k_chain_record(const double *__restrict__ Pu, int npu,
                                                     int gram, const double *__restrict__ Pn,
                                                     int npn, uint8_t *__restrict__ mask,
                                                     int64_t *__restrict__ idx,
                                                     double *__restrict__ obj, DevState *st) {
  if (st->done || st->skip) return;
  const int lane = threadIdx.x;
  double u2 = 0.0, s2 = 0.0;
  if (gram)
    for (int x = lane; x < npu; x += 64) u2 += Pu[x];
  else if (lane == 0)
    u2 = Pu[0];
  for (int x = lane; x < npn; x += 64) s2 += Pn[x];
  u2 = wave_sum(u2);
  s2 = wave_sum(s2);
  if (lane != 0) return;
  const int t = st->t;
  const int64_t p = st->p;
  const double F = st->F - u2;
  st->u2 = u2;
  st->enorm2 = s2;
  st->F = F;
  obj[t + 1] = F;
  idx[t] = p;
  mask[p] = 1;
  st->t = t + 1;
  st->dec_pending = 1;
  if (t + 1 >= st->k) st->done = 1;
}

// ---------------------------------------------------------------------------
int chain_row_blocks(int64_t m) { return (int)((m + kDotRows - 1) / kDotRows); }
int chain_row_groups(int64_t m) { return (int)((m + kRowRB - 1) / kRowRB); }

size_t chain_lds_bytes(int64_t r, int kmax) { return (size_t)(r + kmax + 1) * sizeof(double); }

hipError_t launch_chain(const ChainArgs &ca, hipStream_t s) {
  const int64_t m = ca.m;
  const int nrb = chain_row_blocks(m), nrg = chain_row_groups(m);
  const unsigned qdots = (unsigned)((ca.kmax + kDotCols - 1) / kDotCols);
  const size_t lds_t = (size_t)(ca.kmax + 1) * sizeof(double);
  // K0: c1 partials
  hipLaunchKernelGGL((k_dots<float>), dim3(qdots, nrb), dim3(256), 0, s, (const float *)nullptr,
                     (int64_t)0, 0, ca.Q, ca.ldq, ca.a, m, ca.P, ca.lp, ca.st);
  // K1: e1 = a - Q c1
  hipLaunchKernelGGL((k_rows_sub<false>), dim3(nrg), dim3(kRowThreads), lds_t, s, ca.Q, ca.ldq, ca.a, ca.P,
                     ca.lp, nrb, ca.e1, (double *)nullptr, m, ca.st);
  // K2: c2 partials
  hipLaunchKernelGGL((k_dots<float>), dim3(qdots, nrb), dim3(256), 0, s, (const float *)nullptr,
                     (int64_t)0, 0, ca.Q, ca.ldq, ca.e1, m, ca.P, ca.lp, ca.st);
  // K3: e2 = e1 - Q c2, norm partials
  hipLaunchKernelGGL((k_rows_sub<true>), dim3(nrg), dim3(kRowThreads), lds_t, s, ca.Q, ca.ldq, ca.e1, ca.P,
                     ca.lp, nrb, ca.e2, ca.Pn, m, ca.st);
  // K4: [B^T e2 ; V^T e2] partials (B = A: V^T e2)
  const int nfix = ca.gram ? 0 : (int)ca.r;
  const unsigned tdots = (unsigned)((nfix + ca.kmax + kDotCols - 1) / kDotCols);
  if (ca.b_bf16 && !ca.gram)
    hipLaunchKernelGGL((k_dots<uint16_t>), dim3(tdots, nrb), dim3(256), 0, s,
                       (const uint16_t *)ca.B, ca.ldb, nfix, ca.V, ca.ldq, ca.e2, m, ca.P, ca.lp,
                       ca.st);
  else
    hipLaunchKernelGGL((k_dots<float>), dim3(tdots, nrb), dim3(256), 0, s,
                       ca.gram ? (const float *)nullptr : (const float *)ca.B, ca.ldb, nfix, ca.V,
                       ca.ldq, ca.e2, m, ca.P, ca.lp, ca.st);
  // K5
  ZArgs za{};
  za.Qr = ca.Q;
  za.Qw = ca.Q;
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
  za.r = (int)ca.r;
  za.q64 = ca.q64;
  za.q32 = ca.q32;
  za.z32 = ca.z32;
  za.g0 = ca.g0;
  za.mask = ca.mask;
  za.idx = ca.idx;
  za.obj = ca.obj;
  za.m = m;
  const size_t lds_z = (size_t)(nfix + ca.kmax + 1) * sizeof(double);
  if (ca.gram)
    hipLaunchKernelGGL((k_rows_z<float, true>), dim3(nrg), dim3(kRowThreads), lds_z, s, za, ca.st);
  else if (ca.b_bf16)
    hipLaunchKernelGGL((k_rows_z<uint16_t, false>), dim3(nrg), dim3(kRowThreads), lds_z, s, za, ca.st);
  else
    hipLaunchKernelGGL((k_rows_z<float, false>), dim3(nrg), dim3(kRowThreads), lds_z, s, za, ca.st);
  // K6: record the pick (a workgroup-count handshake at the end of K5 would
  // serialise its ~m/32 workgroups on one atomic counter)
  hipLaunchKernelGGL(k_chain_record, dim3(1), dim3(64), 0, s, ca.Pu, nrg, ca.gram, ca.Pn, nrg,
                     ca.mask, ca.idx, ca.obj, ca.st);
  return hipGetLastError();
}

}  // namespace gcss
