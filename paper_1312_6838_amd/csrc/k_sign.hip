// Concise target B = A Omega with a random sign Omega drawn on the fly
// (Section 5.1: one row Omega_i: per column of A, never stored; Algorithm 2's
// map step sums A_i Omega_i: over the columns).  Omega_ij comes from
// Philox4x32-10 (sign_words / sign_entry in gcss_device.h).
//
// Sparse Omega (density d, d * r small): column j of B is the signed sum of
// the d * n columns of A whose entry in Omega's column j is non-zero, so a
// pass reads only those columns.  One workgroup per (four target columns,
// column range): it tests its range in blocks of 256 * kSpT columns,
// compacts the hits in column order through LDS, and accumulates them in
// that order (binary32, fixed order, so the result is reproducible); the
// ranges' partial columns are summed in order.  Dense Omega (d * r large) runs the MFMA projection
// with the Omega tiles generated in the kernel.
#include "gcss_device.h"

namespace gcss {
namespace {

constexpr int kSpThreads = 256;
constexpr int kSpT = 8;     // columns tested per thread per block
constexpr int kSpUnr = 4;   // hit columns loaded before any is added

// NCH: 16-byte chunks of a column per thread (the column is split over the
// workgroup's threads).  NJ: target columns per workgroup (1, 2 or 4; one
// Philox call yields the entries of four consecutive target columns), as
// many as the accumulators allow.
template <int DT, int NCH, int NJ>
__global__ __launch_bounds__(kSpThreads) void k_proj_sparse(AView A, uint32_t k0, uint32_t k1,
                                                            uint32_t thr, int64_t r,
                                                            int64_t cchunk, float *__restrict__ P,
                                                            int64_t ldp) {
  constexpr int EPC = Elem<DT>::epc, ES = Elem<DT>::esize;
  // hit: column offset in the block (bits 0..10), target column in the
  // group (bits 11..12), sign (bit 31)
  __shared__ int32_t hits[kSpThreads * kSpT * NJ];
  __shared__ int wcnt[kSpThreads / 64];
  const int64_t j0 = (int64_t)blockIdx.x * NJ;
  const int64_t split = blockIdx.y;
  const int64_t m = A.m, n = A.n;
  const int64_t c0 = split * cchunk;
  const int64_t c1 = c0 + cchunk < n ? c0 + cchunk : n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t nchunk = (m * ES + 15) / 16;
  const char *abase = (const char *)A.a;
  const int64_t colb = A.lda * ES;

  float acc[NJ][NCH][EPC];
#pragma unroll
  for (int q = 0; q < NJ; ++q)
#pragma unroll
    for (int x = 0; x < NCH; ++x)
#pragma unroll
      for (int e = 0; e < EPC; ++e) acc[q][x][e] = 0.f;

  for (int64_t base = c0; base < c1; base += kSpThreads * kSpT) {
    // test this thread's kSpT consecutive columns against the NJ targets
    uint32_t hm[NJ], sm[NJ];
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < NJ; ++q) hm[q] = sm[q] = 0u;
#pragma unroll
    for (int t = 0; t < kSpT; ++t) {
      const int64_t i = base + tid * kSpT + t;
      if (i < c1) {
        const uint4 w4 = sign_words(i, (uint32_t)(j0 >> 2), k0, k1);
#pragma unroll
        for (int q = 0; q < NJ; ++q) {
          const int wi = (int)(j0 & 3) + q;  // NJ divides 4, so wi < 4
          const uint32_t w = wi == 0 ? w4.x : (wi == 1 ? w4.y : (wi == 2 ? w4.z : w4.w));
          if ((w >> 1) < thr && j0 + q < r) {
            hm[q] |= 1u << t;
            sm[q] |= (w & 1u) << t;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NJ; ++q) cnt += __popc(hm[q]);
    // compact the hits in column order
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wcnt[wave] = incl;
    __syncthreads();
    int pos = incl - cnt, total = 0;
#pragma unroll
    for (int w = 0; w < kSpThreads / 64; ++w) {
      if (w < wave) pos += wcnt[w];
      total += wcnt[w];
    }
#pragma unroll
    for (int t = 0; t < kSpT; ++t)
#pragma unroll
      for (int q = 0; q < NJ; ++q)
        if ((hm[q] >> t) & 1u)
          hits[pos++] = (int32_t)((uint32_t)(tid * kSpT + t) | ((uint32_t)q << 11) |
                                  (((sm[q] >> t) & 1u) << 31));
    __syncthreads();
    // B[:, j] += sign * A_i for the hits, in order, kSpUnr columns in flight
    for (int h0 = 0; h0 < total; h0 += kSpUnr) {
      uint4 raw[kSpUnr][NCH];
      float sg[kSpUnr];
      int tq[kSpUnr];
#pragma unroll
      for (int u = 0; u < kSpUnr; ++u) {
        const bool live = h0 + u < total;
        const int32_t e = hits[live ? h0 + u : h0];
        const int64_t i = base + (e & 0x7ff);
        float sc = live ? (e < 0 ? -1.f : 1.f) : 0.f;
        if constexpr (DT == DT_FP8) sc *= A.scale[i];
        sg[u] = sc;
        tq[u] = (e >> 11) & 3;
        const char *col = abase + i * colb;
#pragma unroll
        for (int x = 0; x < NCH; ++x) {
          const int64_t ch = tid + kSpThreads * x;
          raw[u][x] = *(const uint4 *)(col + (ch < nchunk ? ch : nchunk - 1) * 16);
        }
      }
#pragma unroll
      for (int u = 0; u < kSpUnr; ++u)
#pragma unroll
        for (int x = 0; x < NCH; ++x) {
          float v[EPC];
          decode_chunk<DT>(raw[u][x], v);
#pragma unroll
          for (int q = 0; q < NJ; ++q) {
            const float sq = (NJ == 1 || tq[u] == q) ? sg[u] : 0.f;
#pragma unroll
            for (int e = 0; e < EPC; ++e) acc[q][x][e] = fmaf(sq, v[e], acc[q][x][e]);
          }
        }
    }
    __syncthreads();  // hits and wcnt are rewritten by the next block
  }
#pragma unroll
  for (int q = 0; q < NJ; ++q) {
    if (j0 + q >= r) continue;
    float *out = P + (split * r + j0 + q) * ldp;
#pragma unroll
    for (int x = 0; x < NCH; ++x) {
      const int64_t ch = tid + kSpThreads * x;
#pragma unroll
      for (int e = 0; e < EPC; ++e) {
        const int64_t row = ch * EPC + e;
        if (ch < nchunk && row < m) out[row] = acc[q][x][e];
      }
    }
  }
}

}  // namespace

uint32_t sign_threshold(double density) {
  const double t = density * 2147483648.0 + 0.5;
  if (!(t >= 1.0)) return 1u;
  if (t >= 2147483648.0) return 0x80000000u;
  return (uint32_t)t;
}

bool sign_uses_sparse(int64_t r, double density) { return density * (double)r <= 4.0; }

size_t sign_sparse_splits(int64_t m, int64_t n, int64_t r, size_t scratch_bytes) {
  const int64_t ldp = ((m + 3) / 4) * 4;
  const size_t per = (size_t)ldp * r * sizeof(float);
  int64_t sp = (4 * 4096 + r - 1) / r;  // about 4096 workgroups of four target columns
  const int64_t maxsp = (n + kSpThreads * kSpT - 1) / (kSpThreads * kSpT);
  if (sp > maxsp) sp = maxsp;
  if ((size_t)sp * per > scratch_bytes) sp = (int64_t)(scratch_bytes / per);
  return sp < 1 ? 1 : (size_t)sp;
}

hipError_t launch_project_sign(const AView &A, uint64_t seed, double density, int64_t r, float *B,
                               int64_t ldb, void *scratch, size_t scratch_bytes, hipStream_t s) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint32_t thr = sign_threshold(density);
  if (!sign_uses_sparse(r, density))
    return launch_project_sign_dense(A, k0, k1, thr, r, B, ldb, scratch, s);
  const int64_t ldp = ((A.m + 3) / 4) * 4;
  const int64_t sp = (int64_t)sign_sparse_splits(A.m, A.n, r, scratch_bytes);
  if ((size_t)sp * ldp * r * sizeof(float) > scratch_bytes) return hipErrorInvalidValue;
  int64_t cchunk = (A.n + sp - 1) / sp;
  cchunk = (cchunk + kSpThreads * kSpT - 1) / (kSpThreads * kSpT) * (kSpThreads * kSpT);
  const int64_t nsp = (A.n + cchunk - 1) / cchunk;
  float *P = (float *)scratch;
  const int64_t nchunk = (A.m * dtype_bytes(A.dtype) + 15) / 16;
  const int64_t per = (nchunk + kSpThreads - 1) / kSpThreads;  // <= 8 for m <= 8192
  const int nch = per <= 1 ? 1 : per <= 2 ? 2 : per <= 4 ? 4 : 8;
  // up to four target columns per workgroup while their accumulators fit
  const int acc_per_col = nch * (16 / dtype_bytes(A.dtype));
  const int nj = acc_per_col <= 16 ? 4 : (acc_per_col <= 32 ? 2 : 1);
  const dim3 grid((unsigned)((r + nj - 1) / nj), (unsigned)nsp);
#define GCSS_SPARSE(DTV, N)                                                                      \
  do {                                                                                           \
    if (nj == 4)                                                                                 \
      hipLaunchKernelGGL((k_proj_sparse<DTV, N, 4>), grid, dim3(kSpThreads), 0, s, A, k0, k1, thr, \
                         r, cchunk, P, ldp);                                                     \
    else if (nj == 2)                                                                            \
      hipLaunchKernelGGL((k_proj_sparse<DTV, N, 2>), grid, dim3(kSpThreads), 0, s, A, k0, k1, thr, \
                         r, cchunk, P, ldp);                                                     \
    else                                                                                         \
      hipLaunchKernelGGL((k_proj_sparse<DTV, N, 1>), grid, dim3(kSpThreads), 0, s, A, k0, k1, thr, \
                         r, cchunk, P, ldp);                                                     \
  } while (0)
  switch (A.dtype) {
    case DT_F32:
      if (nch == 1) GCSS_SPARSE(DT_F32, 1);
      else if (nch == 2) GCSS_SPARSE(DT_F32, 2);
      else if (nch == 4) GCSS_SPARSE(DT_F32, 4);
      else GCSS_SPARSE(DT_F32, 8);
      break;
    case DT_BF16:
      if (nch == 1) GCSS_SPARSE(DT_BF16, 1);
      else if (nch == 2) GCSS_SPARSE(DT_BF16, 2);
      else GCSS_SPARSE(DT_BF16, 4);
      break;
    case DT_FP8:
      if (nch == 1) GCSS_SPARSE(DT_FP8, 1);
      else GCSS_SPARSE(DT_FP8, 2);
      break;
    default: return hipErrorInvalidValue;
  }
#undef GCSS_SPARSE
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_proj_reduce(P, ldp, A.m, r, (int)nsp, B, ldb, s);
}

}  // namespace gcss
