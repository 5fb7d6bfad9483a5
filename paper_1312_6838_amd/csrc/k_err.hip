// Reconstruction error of an explicit target against a selection's basis
// (Problem 5's objective for the picks):  err = || B - Q (Q^T B) ||_F^2,
// with Q the m x t orthonormal FP64 basis of the picked columns and B the
// m x r binary32 target.  The residual is formed explicitly in FP64 (no
// ||B||^2 - ||Q^T B||^2 cancellation).
//
// Three tiled FP64 passes:
//   1. Y_part[x] = Q^T B over the rows of split x   (64 x 64 tiles of Y)
//   2. Y = sum over x of Y_part[x], in split order
//   3. per 64 x 64 tile of R = B - Q Y: the sum of its squares, one partial
//      per workgroup, then the partials in order (fixed-order sums
//      throughout, so the result does not depend on scheduling).
// Q and B are read once per 64-column tile of the other operand instead of
// once per target column.
#include "gcss_device.h"

namespace gcss {

constexpr int kET = 64;   // tile edge (outputs)
constexpr int kEK = 32;   // contraction chunk staged in LDS
constexpr int kEThreads = 256;

// Pass 1: Ypart[x][c * ky + s] = sum over rows j of split x of Q[j, s] B[j, c]
// for the 64 x 64 tile (s0.., c0..) of this workgroup; grid (s tiles, c tiles,
// splits).
__global__ __launch_bounds__(kEThreads) void k_err_qtb(const double *__restrict__ Q, int64_t ldq,
                                                       int64_t m, int k,
                                                       const float *__restrict__ B, int64_t ldb,
                                                       int r, int64_t rows_per_split,
                                                       double *__restrict__ Ypart, int64_t ky) {
  __shared__ double qs[kEK][kET + 1];
  __shared__ double bs[kEK][kET + 1];
  const int s0 = blockIdx.x * kET, c0 = blockIdx.y * kET;
  const int64_t j0 = (int64_t)blockIdx.z * rows_per_split;
  const int64_t j1 = j0 + rows_per_split < m ? j0 + rows_per_split : m;
  // thread (tx, ty) owns outputs (s0 + ty + 16 u, c0 + tx + 16 v), u, v < 4:
  // its LDS reads are conflict-free (consecutive tx, consecutive doubles)
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  // loader: 32 rows x 64 columns, 8 per thread (a wave covers two columns)
  const int lr = threadIdx.x & 31, lc = threadIdx.x >> 5;
  double acc[4][4] = {};
  for (int64_t jb = j0; jb < j1; jb += kEK) {
    const int64_t j = jb + lr;
    const bool jok = j < j1;
    // every load unconditional, from a clamped row and column (so all 16 are
    // in flight together); out-of-range values are zeroed at the LDS store
    const int64_t jc = jok ? j : j1 - 1;
    double qv[8];
    float bv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int cc = lc + 8 * i;
      const int s = s0 + cc, c = c0 + cc;
      qv[i] = Q[(int64_t)(s < k ? s : k - 1) * ldq + jc];
      bv[i] = B[(int64_t)(c < r ? c : r - 1) * ldb + jc];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int cc = lc + 8 * i;
      const int s = s0 + cc, c = c0 + cc;
      qs[lr][cc] = (jok && s < k) ? qv[i] : 0.0;
      bs[lr][cc] = (jok && c < r) ? (double)bv[i] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int jj = 0; jj < kEK; ++jj) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = qs[jj][ty + 16 * u];
        b[u] = bs[jj][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
  double *Yp = Ypart + (int64_t)blockIdx.z * ky * r;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int s = s0 + ty + 16 * u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = c0 + tx + 16 * v;
      if (s < k && c < r) Yp[(int64_t)c * ky + s] = acc[u][v];
    }
  }
}

// Pass 2: Y[c * ky + s] = sum over x < nsplit (in order) of Ypart[x][c * ky + s].
__global__ void k_err_ysum(const double *__restrict__ Ypart, int64_t ky, int k, int r, int nsplit,
                           double *__restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = ky * r;
  if (i >= total) return;
  if ((int)(i % ky) >= k) return;
  double s = 0.0;
  for (int x = 0; x < nsplit; ++x) s += Ypart[(int64_t)x * total + i];
  Y[i] = s;
}

// Pass 3: part[tile] = sum over the 64 x 64 tile (rows j0.., columns c0..) of
// (B[j, c] - sum_s Q[j, s] Y[s, c])^2; grid (row tiles, column tiles).
__global__ __launch_bounds__(kEThreads) void k_err_resid(const double *__restrict__ Q, int64_t ldq,
                                                         int64_t m, int k,
                                                         const float *__restrict__ B, int64_t ldb,
                                                         int r, const double *__restrict__ Y,
                                                         int64_t ky, double *__restrict__ part) {
  __shared__ double qs[kEK][kET + 1];  // [s][j]
  __shared__ double ys[kEK][kET + 1];  // [s][c]
  __shared__ double red[kEThreads / 64];
  const int64_t j0 = (int64_t)blockIdx.x * kET;
  const int c0 = blockIdx.y * kET;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  // loaders: Q as 64 rows x 32 s (a wave: one s, 64 rows), Y as 32 s x 64 c
  const int qj = threadIdx.x & 63, qs0 = threadIdx.x >> 6;
  const int ysl = threadIdx.x & 31, yc0 = threadIdx.x >> 5;
  const int64_t jq = j0 + qj;
  const int64_t jqc = jq < m ? jq : m - 1;
  for (int sb = 0; sb < k; sb += kEK) {
    // unconditional loads from clamped indices, zeroed at the LDS store
    double qv[8], yv[8];
    const int s2 = sb + ysl;
    const int s2c = s2 < k ? s2 : k - 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int s = sb + qs0 + 4 * i;
      const int c = c0 + yc0 + 8 * i;
      qv[i] = Q[(int64_t)(s < k ? s : k - 1) * ldq + jqc];
      yv[i] = Y[(int64_t)(c < r ? c : r - 1) * ky + s2c];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int sl = qs0 + 4 * i;
      const int s = sb + sl;
      qs[sl][qj] = (s < k && jq < m) ? qv[i] : 0.0;
      const int cl = yc0 + 8 * i;
      const int c = c0 + cl;
      ys[ysl][cl] = (s2 < k && c < r) ? yv[i] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int ss = 0; ss < kEK; ++ss) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = qs[ss][ty + 16 * u];
        b[u] = ys[ss][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
  // the tile's target values: 16 unconditional loads from clamped indices
  float bt[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t j = j0 + ty + 16 * u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = c0 + tx + 16 * v;
      bt[u][v] = B[(int64_t)(c < r ? c : r - 1) * ldb + (j < m ? j : m - 1)];
    }
  }
  double sq = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t j = j0 + ty + 16 * u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = c0 + tx + 16 * v;
      const double e = (double)bt[u][v] - acc[u][v];
      sq = (j < m && c < r) ? fma(e, e, sq) : sq;
    }
  }
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0)
    part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// ---------------------------------------------------------------------------
namespace {

struct ErrPlan {
  int64_t ky, rows_per_split, ypart, y, part, bytes;
  int nsplit, stiles, ctiles, rtiles;
};

inline int64_t up256(int64_t x) { return (x + 255) / 256 * 256; }

ErrPlan err_plan(int64_t m, int k, int64_t r, int nsplit) {
  ErrPlan p{};
  p.ky = ((int64_t)(k > 0 ? k : 1) + 3) / 4 * 4;
  p.stiles = (k + kET - 1) / kET;
  p.ctiles = (int)((r + kET - 1) / kET);
  p.rtiles = (int)((m + kET - 1) / kET);
  // whole kEK-row chunks per split
  const int64_t chunks = (m + kEK - 1) / kEK;
  const int64_t per = (chunks + nsplit - 1) / nsplit;
  p.rows_per_split = per * kEK;
  p.nsplit = (int)((m + p.rows_per_split - 1) / p.rows_per_split);
  p.ypart = 0;
  p.y = up256((int64_t)p.nsplit * p.ky * r * 8);
  p.part = p.y + up256(p.ky * r * 8);
  p.bytes = p.part + up256((int64_t)p.rtiles * p.ctiles * 8);
  return p;
}

// Splits of the rows for pass 1: enough workgroups to cover the chip (about
// 2 per CU), at most 16, and at most one per 128 rows.
int err_splits(int64_t m, int k, int64_t r, int num_cu) {
  const int64_t tiles = (int64_t)((k + kET - 1) / kET) * ((r + kET - 1) / kET);
  int64_t sp = tiles > 0 ? (2 * num_cu + tiles - 1) / tiles : 1;
  sp = sp < 1 ? 1 : (sp > 16 ? 16 : sp);
  const int64_t maxsp = (m + 127) / 128;
  if (sp > maxsp) sp = maxsp;
  return (int)(sp < 1 ? 1 : sp);
}

}  // namespace

size_t err_scratch_bytes(int64_t m, int k, int64_t r, int num_cu) {
  return (size_t)err_plan(m, k, r, err_splits(m, k, r, num_cu)).bytes;
}

hipError_t launch_err_tiled(const double *Q, int64_t ldq, int64_t m, int k, const float *B,
                            int64_t ldb, int64_t r, void *scratch, size_t scratch_bytes,
                            int num_cu, double *err, hipStream_t s) {
  ErrPlan p = err_plan(m, k, r, err_splits(m, k, r, num_cu));
  // fewer splits if the scratch is short (one split always fits a layout
  // sized by err_scratch_bytes for these arguments)
  while ((size_t)p.bytes > scratch_bytes && p.nsplit > 1) p = err_plan(m, k, r, p.nsplit / 2);
  if ((size_t)p.bytes > scratch_bytes) return hipErrorInvalidValue;
  char *base = (char *)scratch;
  double *Ypart = (double *)(base + p.ypart), *Y = (double *)(base + p.y),
         *part = (double *)(base + p.part);
  if (k > 0) {
    hipLaunchKernelGGL(k_err_qtb, dim3((unsigned)p.stiles, (unsigned)p.ctiles, (unsigned)p.nsplit),
                       dim3(kEThreads), 0, s, Q, ldq, m, k, B, ldb, (int)r, p.rows_per_split,
                       Ypart, p.ky);
    hipError_t e = hipGetLastError();
    if (e) return e;
    const int64_t total = p.ky * r;
    hipLaunchKernelGGL(k_err_ysum, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Ypart,
                       p.ky, k, (int)r, p.nsplit, Y);
    e = hipGetLastError();
    if (e) return e;
  }
  hipLaunchKernelGGL(k_err_resid, dim3((unsigned)p.rtiles, (unsigned)p.ctiles), dim3(kEThreads), 0,
                     s, Q, ldq, m, k, B, ldb, (int)r, Y, p.ky, part);
  hipError_t e = hipGetLastError();
  if (e) return e;
  return launch_sum_f64(part, (int64_t)p.rtiles * p.ctiles, err, nullptr, 0, s);
}

}  // namespace gcss
