// Achievable HBM read bandwidth: one read-only pass over a caller buffer
// with 16-byte non-temporal loads, consecutive lanes on consecutive chunks,
// eight loads in flight per lane, and each workgroup on one contiguous range
// of the buffer (as the streaming pass's workgroups take consecutive work
// units).  Measured on MI355X, contiguous ranges at two 4-wave workgroups per
// CU read 7.0-7.2 TB/s where a grid-stride walk over the same buffer reads
// 5.6-6.8 TB/s, so the contiguous form is the ceiling the streaming pass is
// compared with, beside the published peak.
//
// The loads feed an XOR fold so they cannot be removed: workgroup b writes
// the XOR of the 32-bit words it read to sink[b], and the XOR of all sink
// entries equals the XOR of every word of the buffer (each word is read
// exactly once), which a caller can check.
#include "gcss_internal.h"

namespace gcss {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 8;

typedef uint32_t pv4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kProbeThreads) void k_hbm_read(const pv4 *__restrict__ p, int64_t nvec,
                                                            float *__restrict__ sink) {
  __shared__ uint32_t wred[kProbeThreads / 64];
  const int64_t per = (nvec + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < nvec ? b0 + per : nvec;
  int64_t i = b0 + threadIdx.x;
  uint32_t acc = 0u;
  for (; i + (int64_t)(kProbeUnroll - 1) * kProbeThreads < b1; i += (int64_t)kProbeUnroll * kProbeThreads) {
    pv4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(p + i + u * kProbeThreads);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc ^= v[u][0] ^ v[u][1] ^ v[u][2] ^ v[u][3];
  }
  for (; i < b1; i += kProbeThreads) {
    const pv4 v = __builtin_nontemporal_load(p + i);
    acc ^= v[0] ^ v[1] ^ v[2] ^ v[3];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, o, 64);
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0u;
#pragma unroll
    for (int w = 0; w < kProbeThreads / 64; ++w) a ^= wred[w];
    sink[blockIdx.x] = __uint_as_float(a);
  }
}

}  // namespace

int hbm_probe_grid(int64_t bytes, int num_cu) {
  const int64_t nvec = bytes / 16;
  // at least one full step of loads per workgroup, at most two workgroups per CU
  int64_t want = (nvec + kProbeThreads * kProbeUnroll - 1) / (kProbeThreads * kProbeUnroll);
  const int64_t cap = 2LL * num_cu;
  if (want > cap) want = cap;
  if (want > kProbeSinkFloats) want = kProbeSinkFloats;
  return (int)(want < 1 ? 1 : want);
}

hipError_t launch_hbm_probe(const void *buf, int64_t bytes, float *sink, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_hbm_read, dim3(grid), dim3(kProbeThreads), 0, s, (const pv4 *)buf,
                     bytes / 16, sink);
  return hipGetLastError();
}

}  // namespace gcss
