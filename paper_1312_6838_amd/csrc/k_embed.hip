// Outputs built on the embedding W = Q^T A (Section 3, Eq. CSS_LowDim) that
// the streaming passes write row by row.
#include "gcss_device.h"

namespace gcss {

// Q-less R factor (Section 6): R[s][j] = W[s][idx[j]] on and above the
// diagonal, 0 below it; a pick outside [0, n) gives a NaN column.  One
// thread per entry of R, rows of R over blockIdx.y.
__global__ __launch_bounds__(256) void k_qless_r(const float *__restrict__ w, int64_t n,
                                                 int64_t ldw, const int64_t *__restrict__ idx,
                                                 int k, float *__restrict__ r, int64_t ldr) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= k) return;
  const int64_t p = idx[j];
  float v;
  if (p < 0 || p >= n)
    v = __builtin_nanf("");
  else
    v = s <= j ? w[(int64_t)s * ldw + p] : 0.f;
  r[(int64_t)s * ldr + j] = v;
}

hipError_t launch_qless_r(const float *w, int64_t n, int64_t ldw, const int64_t *idx, int k,
                          float *r, int64_t ldr, hipStream_t s) {
  if (k < 1) return hipSuccess;
  hipLaunchKernelGGL(k_qless_r, dim3((unsigned)((k + 255) / 256), (unsigned)k), dim3(256), 0, s,
                     w, n, ldw, idx, k, r, ldr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rank-k approximation inside span(A_S) (Section 3, after Boutsidis et al.):
// the SVD of the l x n embedding W comes from the eigen-decomposition of its
// l x l Gram matrix G = W W^T (FP64 sums of exact products of the binary32
// entries), G = U diag(lambda) U^T, sigma = sqrt(lambda).  Then
// U_A = Q U_k (m x k, FP64), V_A = W^T U_k Sigma_k^-1 (n x k, binary32).
//
// Eigen-decomposition: two-sided block Jacobi.  G is padded to L (a multiple
// of 64) with -1 on the padding's diagonal (sorted after every eigenvalue of
// the positive semidefinite G) and split into 2b blocks of 32 indices.  Each
// round pairs the blocks by the round-robin (circle) schedule; one workgroup
// per pair applies a sweep of cyclic Jacobi rotations to its 64 x 64
// subproblem in LDS, then G <- V^T G V and U <- U V with the block-diagonal V
// of the round.  A sweep is 2b - 1 rounds; sweeps repeat until every
// off-diagonal entry is negligible.
namespace {

constexpr int kJB = 32;       // indices per Jacobi block
constexpr int kJP = 2 * kJB;  // indices per block pair
constexpr int kJLd = kJP + 1;  // padded LDS row (doubles)
constexpr double kJacRel = 1e-14;  // |g_xy| <= kJacRel sqrt(|g_xx g_yy|) is zero
constexpr double kJacAbs = 1e-15;  // ... and so is |g_xy| <= kJacAbs * max_x g_xx

// Round-robin pairing of n2 players (n2 even): in round r, pair p meets
// (n2 - 1, r) for p = 0 and ((r + p) mod (n2 - 1), (r - p) mod (n2 - 1)).
__device__ __forceinline__ void rr_pair(int n2, int r, int p, int &u, int &v) {
  const int m1 = n2 - 1;
  if (p == 0) {
    u = n2 - 1;
    v = r % m1;
  } else {
    u = (r + p) % m1;
    v = (r - p + m1) % m1;
  }
}

__device__ __forceinline__ int pair_index(int u, int v, int e) {
  return e < kJB ? u * kJB + e : v * kJB + (e - kJB);
}

__device__ __forceinline__ int clamp_idx(int x, int l) { return (x >= 0 && x < l) ? x : 0; }

__device__ __forceinline__ bool negligible(double gxy, double gxx, double gyy, double fl) {
  const double a = fabs(gxy);
  return a <= fl || a <= kJacRel * sqrt(fabs(gxx) * fabs(gyy));
}

// Partial Gram tiles: workgroup (tile, split) sums W[64a.., c] V[64b.., c]
// over its column range for the upper tile pair (a, b), a <= b (V = W for
// the Gram matrix of W; otherwise a product known to be symmetric).
__global__ __launch_bounds__(256) void k_wgram_part(const float *__restrict__ w,
                                                    const float *__restrict__ v, int64_t ldw,
                                                    int l, int64_t n, int nt, int64_t chunk,
                                                    double *__restrict__ part) {
  __shared__ float wa[64][65];
  __shared__ float wb[64][65];
  const int tile = blockIdx.x % (unsigned)((nt * (nt + 1)) / 2);
  const int split = blockIdx.x / (unsigned)((nt * (nt + 1)) / 2);
  int a = 0, rem = tile;
  while (rem >= nt - a) {
    rem -= nt - a;
    ++a;
  }
  const int b = a + rem;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  const int64_t c0 = (int64_t)split * chunk;
  const int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
  for (int64_t cc = c0; cc < c1; cc += 64) {
#pragma unroll 4
    for (int e = 0; e < 16; ++e) {
      const int id = e * 256 + threadIdx.x;
      const int row = id >> 6, col = id & 63;
      const int64_t c = cc + col;
      const int ra = a * 64 + row, rb = b * 64 + row;
      wa[row][col] = (ra < l && c < c1) ? w[(int64_t)ra * ldw + c] : 0.f;
      wb[row][col] = (rb < l && c < c1) ? v[(int64_t)rb * ldw + c] : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int x = 0; x < 64; ++x) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        av[i] = (double)wa[ty * 4 + i][x];
        bv[i] = (double)wb[tx + 16 * i][x];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  double *o = part + ((int64_t)split * ((nt * (nt + 1)) / 2) + tile) * 4096;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) o[(ty * 4 + i) * 64 + tx + 16 * j] = acc[i][j];
}

// G (L x L, both triangles) = sum of the splits in order; padding rows and
// columns 0 with -1 on the diagonal; U = I.
__global__ __launch_bounds__(256) void k_wgram_reduce(const double *__restrict__ part, int nsplit,
                                                      int nt, int l, double *__restrict__ G,
                                                      double *__restrict__ U) {
  const int ntiles = (nt * (nt + 1)) / 2;
  const int tile = blockIdx.x;
  int a = 0, rem = tile;
  while (rem >= nt - a) {
    rem -= nt - a;
    ++a;
  }
  const int b = a + rem;
  const int L = nt * 64;
  for (int e = threadIdx.x; e < 4096; e += 256) {
    const int i = e >> 6, j = e & 63;
    const int x = a * 64 + i, y = b * 64 + j;
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += part[((int64_t)sp * ntiles + tile) * 4096 + e];
    if (x >= l || y >= l) s = (x == y) ? -1.0 : 0.0;
    G[(int64_t)x * L + y] = s;
    G[(int64_t)y * L + x] = s;
    U[(int64_t)x * L + y] = x == y ? 1.0 : 0.0;
    U[(int64_t)y * L + x] = x == y ? 1.0 : 0.0;
  }
}

// aux[0] = kJacAbs * max(0, max_x g_xx): the absolute zero of the sweeps.
__global__ __launch_bounds__(256) void k_jac_floor(const double *__restrict__ G, int L,
                                                   double *__restrict__ aux) {
  __shared__ double red[4];
  double mx = 0.0;
  for (int x = threadIdx.x; x < L; x += 256) mx = fmax(mx, G[(int64_t)x * L + x]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) aux[0] = kJacAbs * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// One workgroup per block pair of round r: kJacInner sweeps of cyclic
// Jacobi on the 64 x 64 subproblem in LDS (one sweep per call is enough for
// the outer iteration to converge, and costs a quarter of solving each
// subproblem exactly); writes the rotation V (64 x 64, row-major) to vb[p].
// A subproblem that is already diagonal is left alone (V = I).  Within an
// inner round the 32 rotations touch disjoint index pairs, so S <- J^T S J
// splits into independent 2 x 2 blocks.
constexpr int kJacInner = 1;

__global__ __launch_bounds__(256) void k_jac_solve(const double *__restrict__ G, int L, int r,
                                                   const double *__restrict__ aux,
                                                   double *__restrict__ vb) {
  __shared__ double S[kJP][kJLd];
  __shared__ double V[kJP][kJLd];
  __shared__ double cs[kJB], sn[kJB];
  __shared__ int px[kJB], py[kJB];
  __shared__ int busy, nrot;
  const int p = blockIdx.x;
  int u, v;
  rr_pair(L / kJB, r, p, u, v);
  const double fl = aux[0];
  if (threadIdx.x == 0) busy = 0;
  for (int e = threadIdx.x; e < kJP * kJP; e += 256) {
    const int i = e / kJP, j = e % kJP;
    S[i][j] = G[(int64_t)pair_index(u, v, i) * L + pair_index(u, v, j)];
    V[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  {
    int mine = 0;
    for (int e = threadIdx.x; e < kJP * kJP; e += 256) {
      const int i = e / kJP, j = e % kJP;
      if (i < j && !negligible(S[i][j], S[i][i], S[j][j], fl)) mine = 1;
    }
    if (mine) busy = 1;  // benign race: every writer stores 1
  }
  __syncthreads();
  for (int sweep = 0; busy && sweep < kJacInner; ++sweep) {
    if (threadIdx.x == 0) nrot = 0;
    for (int rr = 0; rr < kJP - 1; ++rr) {
      if (threadIdx.x < kJB) {
        int x, y;
        rr_pair(kJP, rr, threadIdx.x, x, y);
        const double gxx = S[x][x], gyy = S[y][y], gxy = S[x][y];
        double c = 1.0, sv = 0.0;
        if (!negligible(gxy, gxx, gyy, fl)) {
          const double tau = (gyy - gxx) / (2.0 * gxy);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sv = t * c;
          nrot = 1;  // benign race
        }
        cs[threadIdx.x] = c;
        sn[threadIdx.x] = sv;
        px[threadIdx.x] = x;
        py[threadIdx.x] = y;
      }
      __syncthreads();
      // S <- J^T S J by 2 x 2 blocks (row pair P, column pair Q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int blk = e * 256 + threadIdx.x;
        const int P = blk >> 5, Q = blk & 31;
        const int x0 = px[P], y0 = py[P], x1 = px[Q], y1 = py[Q];
        const double cp = cs[P], sp = sn[P], cq = cs[Q], sq = sn[Q];
        const double a00 = S[x0][x1], a01 = S[x0][y1], a10 = S[y0][x1], a11 = S[y0][y1];
        const double r00 = cp * a00 - sp * a10, r01 = cp * a01 - sp * a11;
        const double r10 = sp * a00 + cp * a10, r11 = sp * a01 + cp * a11;
        double b00 = cq * r00 - sq * r01, b01 = sq * r00 + cq * r01;
        double b10 = cq * r10 - sq * r11, b11 = sq * r10 + cq * r11;
        if (P == Q && sp != 0.0) {  // the rotated pair's entry is zero
          b01 = 0.0;
          b10 = 0.0;
        }
        S[x0][x1] = b00;
        S[x0][y1] = b01;
        S[y0][x1] = b10;
        S[y0][y1] = b11;
      }
      // V <- V J: row i, column pair Q
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int t = e * 256 + threadIdx.x;
        const int Q = t >> 6, i = t & 63;
        const int x = px[Q], y = py[Q];
        const double c = cs[Q], sv = sn[Q];
        const double va = V[i][x], vbv = V[i][y];
        V[i][x] = c * va - sv * vbv;
        V[i][y] = sv * va + c * vbv;
      }
      __syncthreads();
    }
    if (nrot == 0) break;
    __syncthreads();
  }
  double *o = vb + (int64_t)p * kJP * kJP;
  for (int e = threadIdx.x; e < kJP * kJP; e += 256) o[e] = V[e / kJP][e % kJP];
}

// G <- V^T G V and U <- U V for the block-diagonal V of round r.  The first
// b(b+1)/2 workgroups take the block-pair regions (p, q), p <= q, of G (and
// write the mirror); the rest take 64-row slabs of U times a pair's columns.
__global__ __launch_bounds__(256) void k_jac_apply(double *__restrict__ G, double *__restrict__ U,
                                                   int L, int r, const double *__restrict__ vb) {
  __shared__ double X[kJP][kJLd];
  __shared__ double Vp[kJP][kJLd];
  __shared__ double Vq[kJP][kJLd];
  const int nb = L / kJP;  // pairs
  const int ngg = nb * (nb + 1) / 2;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int n2 = L / kJB;
  if ((int)blockIdx.x < ngg) {
    int p = 0, rem = blockIdx.x;
    while (rem >= nb - p) {
      rem -= nb - p;
      ++p;
    }
    const int q = p + rem;
    int up, vp, uq, vq;
    rr_pair(n2, r, p, up, vp);
    rr_pair(n2, r, q, uq, vq);
    for (int e = threadIdx.x; e < kJP * kJP; e += 256) {
      const int i = e / kJP, j = e % kJP;
      X[i][j] = G[(int64_t)pair_index(up, vp, i) * L + pair_index(uq, vq, j)];
      Vp[i][j] = vb[(int64_t)p * kJP * kJP + e];
      Vq[i][j] = vb[(int64_t)q * kJP * kJP + e];
    }
    __syncthreads();
    // T = X Vq (rows 4ty.., columns tx + 16 j)
    double t[4][4] = {};
    for (int x = 0; x < kJP; ++x) {
      double xa[4], vv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xa[i] = X[ty * 4 + i][x];
#pragma unroll
      for (int j = 0; j < 4; ++j) vv[j] = Vq[x][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) t[i][j] = fma(xa[i], vv[j], t[i][j]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) X[ty * 4 + i][tx + 16 * j] = t[i][j];
    __syncthreads();
    // Y = Vp^T T
    double y[4][4] = {};
    for (int x = 0; x < kJP; ++x) {
      double va[4], tv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) va[i] = Vp[x][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) tv[j] = X[x][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) y[i][j] = fma(va[i], tv[j], y[i][j]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) X[ty * 4 + i][tx + 16 * j] = y[i][j];
    __syncthreads();
    for (int e = threadIdx.x; e < kJP * kJP; e += 256) {
      const int i = e / kJP, j = e % kJP;
      const int gi = pair_index(up, vp, i), gj = pair_index(uq, vq, j);
      // the diagonal region is kept exactly symmetric
      const double val = p == q ? 0.5 * (X[i][j] + X[j][i]) : X[i][j];
      G[(int64_t)gi * L + gj] = val;
      if (p != q) G[(int64_t)gj * L + gi] = val;
    }
  } else {
    const int blk = blockIdx.x - ngg;
    const int rb = blk / nb, p = blk % nb;
    int up, vp;
    rr_pair(n2, r, p, up, vp);
    for (int e = threadIdx.x; e < kJP * kJP; e += 256) {
      const int i = e / kJP, j = e % kJP;
      X[i][j] = U[(int64_t)(rb * kJP + i) * L + pair_index(up, vp, j)];
      Vp[i][j] = vb[(int64_t)p * kJP * kJP + e];
    }
    __syncthreads();
    double t[4][4] = {};
    for (int x = 0; x < kJP; ++x) {
      double xa[4], vv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xa[i] = X[ty * 4 + i][x];
#pragma unroll
      for (int j = 0; j < 4; ++j) vv[j] = Vp[x][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) t[i][j] = fma(xa[i], vv[j], t[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        U[(int64_t)(rb * kJP + ty * 4 + i) * L + pair_index(up, vp, tx + 16 * j)] = t[i][j];
  }
}

// flag[b] = 1 if row slab b (64 rows) of G holds an off-diagonal entry
// that is not negligible, else 0.
__global__ __launch_bounds__(256) void k_jac_check(const double *__restrict__ G, int L,
                                                   const double *__restrict__ aux,
                                                   int *__restrict__ flag) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const double fl = aux[0];
  int mine = 0;
  const int x0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * L; e += 256) {
    const int x = x0 + e / L, y = e % L;
    if (y == x) continue;
    const double gxy = G[(int64_t)x * L + y];
    if (!negligible(gxy, G[(int64_t)x * L + x], G[(int64_t)y * L + y], fl)) mine = 1;
  }
  if (mine) any = 1;  // benign race: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0) flag[blockIdx.x] = any;
}

// Order of the eigenvalues (descending; ties by index), sigma of the k
// largest, and the sums the error needs: res[0] = sum of all l eigenvalues
// (= ||W||_F^2), res[1] = sum of the l - k smallest (clamped at 0).
__global__ __launch_bounds__(1024) void k_eig_order(const double *__restrict__ G, int L, int l,
                                                    int k, int *__restrict__ perm,
                                                    double *__restrict__ sigma,
                                                    double *__restrict__ res) {
  __shared__ double r0[16], r1[16];
  double s_all = 0.0, s_tail = 0.0;
  // NaN sorts last, so the ranks are a permutation of 0 .. l-1
  auto ev = [&](int x) {
    const double v = G[(int64_t)x * L + x];
    return isnan(v) ? -INFINITY : v;
  };
  for (int x = threadIdx.x; x < l; x += 1024) {
    const double lx = ev(x);
    int rank = 0;
    for (int y = 0; y < l; ++y) {
      const double ly = ev(y);
      rank += (ly > lx || (ly == lx && y < x)) ? 1 : 0;
    }
    if (rank < k) {
      perm[rank] = x;
      sigma[rank] = sqrt(fmax(lx, 0.0));
    } else {
      s_tail += fmax(lx, 0.0);
    }
    s_all += lx;
  }
  for (int o = 32; o > 0; o >>= 1) {
    s_all += __shfl_xor(s_all, o, 64);
    s_tail += __shfl_xor(s_tail, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    r0[threadIdx.x >> 6] = s_all;
    r1[threadIdx.x >> 6] = s_tail;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int x = 0; x < 16; ++x) {
      a += r0[x];
      b += r1[x];
    }
    res[0] = a;
    res[1] = b;
  }
}

// U_A = Q U[:, perm] (m x k, column-major ldu): 64 x 64 tiles, FP64.
__global__ __launch_bounds__(256) void k_rank_u(const double *__restrict__ Q, int64_t ldq,
                                                int64_t m, int l, const double *__restrict__ Ue,
                                                int L, const int *__restrict__ perm, int k,
                                                double *__restrict__ out, int64_t ldu) {
  __shared__ double qa[16][65];
  __shared__ double ub[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 64;
  double acc[4][4] = {};
  for (int s0 = 0; s0 < l; s0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int s = e >> 6, c = e & 63;
      const int sg = s0 + s;
      const int64_t i = i0 + c;
      const int j = j0 + c;
      qa[s][c] = (sg < l && i < m) ? Q[(int64_t)sg * ldq + i] : 0.0;
      ub[s][c] = (sg < l && j < k) ? Ue[(int64_t)sg * L + clamp_idx(perm[j], l)] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = qa[s][tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = ub[s][ty * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int jj = j0 + ty * 4 + j;
    if (jj >= k) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t ii = i0 + tx + 16 * i;
      if (ii < m) out[(int64_t)jj * ldu + ii] = acc[i][j];
    }
  }
}

// Sign convention: the largest-magnitude entry (first on ties) of column j of
// U_A is made positive; mcoef[s][j] = sign_j U[s][perm j] / sigma_j (binary32,
// row-major l x k; 0 where sigma_j = 0), the coefficients of V_A (FP64).
__global__ __launch_bounds__(256) void k_rank_sign(double *__restrict__ ua, int64_t ldu, int64_t m,
                                                   const double *__restrict__ Ue, int L, int l,
                                                   const int *__restrict__ perm,
                                                   const double *__restrict__ sigma, int k,
                                                   double *__restrict__ mcoef) {
  __shared__ double bv[4];
  __shared__ int64_t bi[4];
  __shared__ double sgn_s;
  const int j = blockIdx.x;
  double* col = ua + (int64_t)j * ldu;
  double best = -1.0;
  int64_t besti = INT64_MAX;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const double a = fabs(col[i]);
    if (a > best || (a == best && i < besti)) {
      best = a;
      besti = i;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int64_t oi = __shfl_xor((long long)besti, o, 64);
    if (ob > best || (ob == best && oi < besti)) {
      best = ob;
      besti = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    bv[threadIdx.x >> 6] = best;
    bi[threadIdx.x >> 6] = besti;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = bv[0];
    int64_t i = bi[0];
    for (int x = 1; x < 4; ++x)
      if (bv[x] > b || (bv[x] == b && bi[x] < i)) {
        b = bv[x];
        i = bi[x];
      }
    sgn_s = (i < m && col[i] < 0.0) ? -1.0 : 1.0;
  }
  __syncthreads();
  const double sg = sgn_s;
  if (sg < 0.0)
    for (int64_t i = threadIdx.x; i < m; i += 256) col[i] = -col[i];
  const double sj = sigma[j];
  const double f = sj > 0.0 ? sg / sj : 0.0;
  const int pj = clamp_idx(perm[j], l);
  for (int s = threadIdx.x; s < l; s += 256) mcoef[(int64_t)s * k + j] = f * Ue[(int64_t)s * L + pj];
}

// V_A = W^T mcoef (n x k, column-major ldv): 64 x 64 tiles; FP64 sums
// (the coefficients of small sigma_j are large and their terms cancel),
// stored as binary32.
__global__ __launch_bounds__(256) void k_rank_v(const float *__restrict__ w, int64_t ldw, int64_t n,
                                                int l, const double *__restrict__ mcoef, int k,
                                                float *__restrict__ out, int64_t ldv) {
  __shared__ float wa[16][65];
  __shared__ double mb[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 64;
  double acc[4][4] = {};
  for (int s0 = 0; s0 < l; s0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int s = e >> 6, c = e & 63;
      const int sg = s0 + s;
      const int64_t i = i0 + c;
      const int j = j0 + c;
      wa[s][c] = (sg < l && i < n) ? w[(int64_t)sg * ldw + i] : 0.f;
      mb[s][c] = (sg < l && j < k) ? mcoef[(int64_t)sg * k + j] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (double)wa[s][tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = mb[s][ty * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int jj = j0 + ty * 4 + j;
    if (jj >= k) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t ii = i0 + tx + 16 * i;
      if (ii < n) out[(int64_t)jj * ldv + ii] = (float)acc[i][j];
    }
  }
}

// Orthonormalising coefficients: mcoef[s][j] = U[s][perm j] / sigma_j for
// the k leading eigenpairs of Y^T Y, 0 where sigma_j <= 1e-6 sigma_0 (those
// directions are rounding noise of the binary32 Y); row-major l x k, FP64.
__global__ __launch_bounds__(256) void k_ortho_coef(const double *__restrict__ Ue, int L, int l,
                                                    const int *__restrict__ perm,
                                                    const double *__restrict__ sigma, int k,
                                                    double *__restrict__ mcoef) {
  const int j = blockIdx.x;
  const double sj = sigma[j], s0 = sigma[0];
  const double f = (sj > 1e-6 * s0 && sj > 0.0) ? 1.0 / sj : 0.0;
  const int pj = clamp_idx(perm[j], l);
  for (int s = threadIdx.x; s < l; s += 256) mcoef[(int64_t)s * k + j] = f * Ue[(int64_t)s * L + pj];
}

// out[i * c + j] = in[j * ldi + i] (binary32, m x c column-major to row-major)
__global__ __launch_bounds__(256) void k_to_rowmajor(const float *__restrict__ in, int64_t ldi,
                                                     int64_t m, int c, float *__restrict__ out) {
  __shared__ float t[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int j0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int64_t i = i0 + tx;
    const int j = j0 + y;
    t[y][tx] = (i < m && j < c) ? in[(int64_t)j * ldi + i] : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t i = i0 + y;
    const int j = j0 + tx;
    if (i < m && j < c) out[i * c + j] = t[tx][y];
  }
}

// out[j * ldo + i] = (double) in[j * ldi + i]
__global__ __launch_bounds__(256) void k_cols_to_f64(const float *__restrict__ in, int64_t ldi,
                                                     int64_t m, int c, double *__restrict__ out,
                                                     int64_t ldo) {
  const int j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
    out[(int64_t)j * ldo + i] = (double)in[(int64_t)j * ldi + i];
}

// Cholesky factor R (upper, R^T R = G) of the l x l Gram matrix in G (row
// stride L) and its inverse, by one workgroup: R row-major in rbuf (row
// stride L), mcoef[p][c] = (R^-1)[p][c] (row-major l x l).  Each dot
// product is split over a group of 8 lanes (lane g sums the terms p = g
// mod 8) and reduced by shuffles, so a step's latency is about an eighth of
// its length.  A pivot that falls to 1e-13 of its diagonal entry marks a
// dependent column: its row and column of R^-1 are zero, so the
// orthonormalised block loses it.
__global__ __launch_bounds__(1024) void k_chol_inv(const double *__restrict__ G, int L, int l,
                                                   double *__restrict__ rbuf,
                                                   double *__restrict__ mcoef) {
  __shared__ double invd[kRankMaxL];
  __shared__ double vec[kRankMaxL];  // column j of R (factorisation) or row p (inverse)
  const int g8 = threadIdx.x & 7, grp = threadIdx.x >> 3;  // 128 groups of 8 lanes
  auto group_sum = [](double a) {
    a += __shfl_xor(a, 1, 64);
    a += __shfl_xor(a, 2, 64);
    a += __shfl_xor(a, 4, 64);
    return a;
  };
  for (int j = 0; j < l; ++j) {
    for (int p = threadIdx.x; p < j; p += 1024) vec[p] = rbuf[(int64_t)p * L + j];
    __syncthreads();
    if (threadIdx.x < 64) {  // pivot: G[j][j] - |R[:j, j]|^2 by one wave
      double a = 0.0;
      for (int p = threadIdx.x; p < j; p += 64) a += vec[p] * vec[p];
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
      if (threadIdx.x == 0) {
        const double g = G[(int64_t)j * L + j];
        const double r = g - a;
        const double d = (r > 1e-13 * g && r > 0.0) ? sqrt(r) : 0.0;
        rbuf[(int64_t)j * L + j] = d;
        invd[j] = d > 0.0 ? 1.0 / d : 0.0;
      }
    }
    __syncthreads();
    const double inv = invd[j];
    // row j: R[j][c] = (G[j][c] - R[:j, j] . R[:j, c]) / R[j][j]
    for (int c0 = j + 1; c0 < l; c0 += 128) {
      const int c = c0 + grp;
      double a = 0.0;
      if (c < l)
        for (int p = g8; p < j; p += 8) a += vec[p] * rbuf[(int64_t)p * L + c];
      a = group_sum(a);
      if (c < l && g8 == 0) rbuf[(int64_t)j * L + c] = (G[(int64_t)j * L + c] - a) * inv;
    }
    __syncthreads();
  }
  // R^-1 by rows from the last: X[p][c] = -(R[p][p+1..c] . X[p+1..c][c]) / R[p][p]
  for (int p = l - 1; p >= 0; --p) {
    for (int q = threadIdx.x; q < l; q += 1024) vec[q] = q > p ? rbuf[(int64_t)p * L + q] : 0.0;
    __syncthreads();
    for (int c0 = 0; c0 < l; c0 += 128) {
      const int c = c0 + grp;
      double a = 0.0;
      if (c < l && c > p)
        for (int q = p + 1 + g8; q <= c; q += 8) a += vec[q] * mcoef[(int64_t)q * l + c];
      a = group_sum(a);
      if (c < l && g8 == 0) mcoef[(int64_t)p * l + c] = c == p ? invd[p] : (c > p ? -a * invd[p] : 0.0);
    }
    __syncthreads();
  }
}

// b[j * ldb + i] = (float)(u[j * ldu + i] * sigma[j]): the target U_k Sigma_k
__global__ __launch_bounds__(256) void k_scale_cols(const double *__restrict__ u, int64_t ldu,
                                                    int64_t m, const double *__restrict__ sigma,
                                                    float *__restrict__ b, int64_t ldb) {
  const int j = blockIdx.y;
  const double sj = sigma[j];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
    b[(int64_t)j * ldb + i] = (float)(u[(int64_t)j * ldu + i] * sj);
}

}  // namespace

hipError_t launch_scale_cols(const RankPlan &P, char *scr, const double *u, int64_t ldu, int64_t m,
                             int k, float *b, int64_t ldb, hipStream_t s) {
  const unsigned gx = (unsigned)((m + 255) / 256 < 64 ? (m + 255) / 256 : 64);
  hipLaunchKernelGGL(k_scale_cols, dim3(gx, (unsigned)k), dim3(256), 0, s, u, ldu, m,
                     (const double *)(scr + P.sigma), b, ldb);
  return hipGetLastError();
}

hipError_t launch_cholqr_apply(const RankPlan &P, char *scr, int l, const float *y, int64_t ldy,
                               int64_t m, float *out, int64_t ldo, hipStream_t s) {
  double *mc = (double *)(scr + P.mcoef);
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(1024), 0, s, (const double *)(scr + P.G), P.L, l,
                     (double *)(scr + P.U), mc);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_rank_v, dim3((unsigned)((m + 63) / 64), (unsigned)((l + 63) / 64)), dim3(256),
                     0, s, y, ldy, m, l, (const double *)mc, l, out, ldo);
  return hipGetLastError();
}

hipError_t launch_eig_order(const RankPlan &P, char *scr, int l, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_eig_order, dim3(1), dim3(1024), 0, s, (const double *)(scr + P.G), P.L, l,
                     k, (int *)(scr + P.perm), (double *)(scr + P.sigma),
                     (double *)(scr + P.aux) + 1);
  return hipGetLastError();
}

hipError_t launch_orth_apply(const RankPlan &P, char *scr, int l, const float *y, int64_t ldy,
                             int64_t m, float *out, int64_t ldo, hipStream_t s) {
  double *mc = (double *)(scr + P.mcoef);
  hipLaunchKernelGGL(k_ortho_coef, dim3((unsigned)l), dim3(256), 0, s,
                     (const double *)(scr + P.U), P.L, l, (const int *)(scr + P.perm),
                     (const double *)(scr + P.sigma), l, mc);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_rank_v, dim3((unsigned)((m + 63) / 64), (unsigned)((l + 63) / 64)), dim3(256),
                     0, s, y, ldy, m, l, (const double *)mc, l, out, ldo);
  return hipGetLastError();
}

hipError_t launch_ritz_vectors(const RankPlan &P, char *scr, int l, int k, const double *Q,
                               int64_t ldq, int64_t m, double *ua, int64_t ldu, hipStream_t s) {
  const double *U = (const double *)(scr + P.U);
  const int *perm = (const int *)(scr + P.perm);
  hipLaunchKernelGGL(k_rank_u, dim3((unsigned)((m + 63) / 64), (unsigned)((k + 63) / 64)), dim3(256),
                     0, s, Q, ldq, m, l, U, P.L, perm, k, ua, ldu);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_rank_sign, dim3((unsigned)k), dim3(256), 0, s, ua, ldu, m, U, P.L, l, perm,
                     (const double *)(scr + P.sigma), k, (double *)(scr + P.mcoef));
  return hipGetLastError();
}

hipError_t launch_to_rowmajor(const float *in, int64_t ldi, int64_t m, int c, float *out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_to_rowmajor, dim3((unsigned)((m + 31) / 32), (unsigned)((c + 31) / 32)),
                     dim3(256), 0, s, in, ldi, m, c, out);
  return hipGetLastError();
}

hipError_t launch_cols_to_f64(const float *in, int64_t ldi, int64_t m, int c, double *out,
                              int64_t ldo, hipStream_t s) {
  const unsigned gx = (unsigned)((m + 255) / 256 < 64 ? (m + 255) / 256 : 64);
  hipLaunchKernelGGL(k_cols_to_f64, dim3(gx, (unsigned)c), dim3(256), 0, s, in, ldi, m, c, out, ldo);
  return hipGetLastError();
}

// Workspace of rank_k for l <= lmax picks over n columns.
RankPlan rank_plan(int lmax, int64_t n) {
  RankPlan P{};
  const int L = ((lmax < 1 ? 1 : lmax) + 63) / 64 * 64;
  P.L = L;
  P.nt = L / 64;
  const int ntiles = P.nt * (P.nt + 1) / 2;
  const int64_t maxsplit = (n + 63) / 64;
  int64_t ns = (1024 + ntiles - 1) / ntiles;
  if (ns > maxsplit) ns = maxsplit;
  const int64_t cap = (int64_t)32 << 20;  // partial tiles at most 32 MiB
  if (ns * ntiles * 4096 * 8 > cap) ns = cap / ((int64_t)ntiles * 4096 * 8);
  if (ns < 1) ns = 1;
  P.chunk = ((n + ns - 1) / ns + 63) / 64 * 64;
  P.nsplit = (int)((n + P.chunk - 1) / P.chunk);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  P.G = take((size_t)L * L * 8);
  P.U = take((size_t)L * L * 8);
  P.vb = take((size_t)(L / kJP) * kJP * kJP * 8);
  P.part = take((size_t)P.nsplit * ntiles * 4096 * 8);
  P.mcoef = take((size_t)L * L * 8);
  P.perm = take((size_t)L * 4);
  P.sigma = take((size_t)L * 8);
  P.aux = take(64);
  P.flag = take((size_t)(L / 64) * 4);
  P.bytes = off;
  return P;
}

hipError_t launch_wgram(const RankPlan &P, const float *w, int64_t ldw, int l, int64_t n,
                        char *scr, hipStream_t s) {
  return launch_wgram2(P, w, w, ldw, l, n, scr, s);
}

hipError_t launch_wgram2(const RankPlan &P, const float *w, const float *v, int64_t ldw, int l,
                         int64_t n, char *scr, hipStream_t s) {
  const int ntiles = P.nt * (P.nt + 1) / 2;
  double *part = (double *)(scr + P.part);
  hipLaunchKernelGGL(k_wgram_part, dim3((unsigned)(ntiles * P.nsplit)), dim3(256), 0, s, w, v, ldw,
                     l, n, P.nt, P.chunk, part);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_wgram_reduce, dim3((unsigned)ntiles), dim3(256), 0, s, part, P.nsplit, P.nt,
                     l, (double *)(scr + P.G), (double *)(scr + P.U));
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL(k_jac_floor, dim3(1), dim3(256), 0, s, (const double *)(scr + P.G), P.L,
                     (double *)(scr + P.aux));
  return hipGetLastError();
}

hipError_t launch_jacobi_sweep(const RankPlan &P, char *scr, hipStream_t s) {
  const int L = P.L;
  const int n2 = L / kJB, nb = L / kJP;
  double *G = (double *)(scr + P.G), *U = (double *)(scr + P.U), *vb = (double *)(scr + P.vb);
  const double *aux = (const double *)(scr + P.aux);
  const unsigned napply = (unsigned)(nb * (nb + 1) / 2 + (L / kJP) * nb);
  for (int r = 0; r < n2 - 1; ++r) {
    hipLaunchKernelGGL(k_jac_solve, dim3((unsigned)nb), dim3(256), 0, s, G, L, r, aux, vb);
    hipError_t e = hipGetLastError();
    if (e) return e;
    hipLaunchKernelGGL(k_jac_apply, dim3(napply), dim3(256), 0, s, G, U, L, r, vb);
    if ((e = hipGetLastError())) return e;
  }
  hipLaunchKernelGGL(k_jac_check, dim3((unsigned)(L / 64)), dim3(256), 0, s, (const double *)G, L,
                     aux, (int *)(scr + P.flag));
  return hipGetLastError();
}

hipError_t launch_rank_outputs(const RankPlan &P, char *scr, int l, int k, const double *Q,
                               int64_t ldq, int64_t m, double *ua, int64_t ldu, const float *w,
                               int64_t ldw, int64_t n, float *va, int64_t ldv, hipStream_t s) {
  const int L = P.L;
  const double *G = (const double *)(scr + P.G), *U = (const double *)(scr + P.U);
  int *perm = (int *)(scr + P.perm);
  double *sigma = (double *)(scr + P.sigma);
  hipLaunchKernelGGL(k_eig_order, dim3(1), dim3(1024), 0, s, G, L, l, k, perm, sigma,
                     (double *)(scr + P.aux) + 1);
  hipError_t e = hipGetLastError();
  if (e || !ua) return e;
  hipLaunchKernelGGL(k_rank_u, dim3((unsigned)((m + 63) / 64), (unsigned)((k + 63) / 64)), dim3(256),
                     0, s, Q, ldq, m, l, U, L, (const int *)perm, k, ua, ldu);
  if ((e = hipGetLastError())) return e;
  double *mc = (double *)(scr + P.mcoef);
  hipLaunchKernelGGL(k_rank_sign, dim3((unsigned)k), dim3(256), 0, s, ua, ldu, m, U, L, l,
                     (const int *)perm, (const double *)sigma, k, mc);
  if ((e = hipGetLastError()) || !va) return e;
  hipLaunchKernelGGL(k_rank_v, dim3((unsigned)((n + 63) / 64), (unsigned)((k + 63) / 64)), dim3(256),
                     0, s, w, ldw, n, l, (const double *)mc, k, va, ldv);
  return hipGetLastError();
}

}  // namespace gcss
