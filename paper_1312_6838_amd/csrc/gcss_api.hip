// Host engine behind the C ABI of include/gcss.h: argument checks, the
// workspace carve, the order of kernel launches of one greedy step, graph
// capture of the k-step loop, and read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gcss.h"
#include "gcss_internal.h"

using namespace gcss;

namespace {

thread_local std::string g_err;

gcss_status fail(gcss_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(GCSS_ERR_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                             \
  } while (0)

constexpr int kPlanCU = 256;       // CU count used to size the workspace (MI355X)
constexpr int kSpareSlots = GCSS_ASYNC_SPARE_STEPS;  // extra steps of a captured loop (rejected picks)
constexpr double kBasisTau = 1e-13;  // dependence threshold of the basis-only mode
constexpr size_t kChainLdsMax = 44 * 1024;  // dynamic LDS the chain's row kernels may take

inline size_t up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t ld_for(int64_t m) { return (int64_t)up((size_t)m, 64); }

struct Carve {
  size_t off = 0;
  template <typename T>
  size_t take(size_t count) {
    size_t o = up(off, 256);
    off = o + up(count * sizeof(T), 256);
    return o;
  }
};

// Offsets of every workspace region for a description (sizes only).
struct Layout {
  size_t f0, g0, f, g, mask0, mask, part, qpart, npart, Q, e1, e2, w, q64, q32, z32, c1, c2, c3, ups,
      st, idx, obj, scal, pick, quad, ap64, gram, bexp, V, P, Pn, Pu, scratch, total;
  int64_t lp;      // row stride of the dot partials of the per-step chain
  bool chain;      // the per-step chain kernels fit (their LDS holds r_max + k_max + 1 doubles)
  size_t scratch_bytes;
  size_t qbuf;  // padded stream length of q32 / z32 / q64
  StreamGeo geo;
  int64_t ldq;
};

// Scratch of gcss_top_eig for a block of width s: the projection's
// partial sums, Y, Q (column-major) and Q (row-major), then the eigensolver's
// buffers.
struct EigLayout {
  size_t y, qf, qr, rank, bytes;
  RankPlan P;
};
EigLayout eig_layout(int64_t m, int64_t ldq, int s, int num_cu) {
  EigLayout E{};
  size_t off = up(proj_scratch_bytes(m, m, s, num_cu), 256);
  E.y = off;
  off += up((size_t)ldq * s * 4, 256);
  E.qf = off;
  off += up((size_t)ldq * s * 4, 256);
  E.qr = off;
  off += up((size_t)m * s * 4, 256);
  E.rank = off;
  E.P = rank_plan(s, m);
  E.bytes = off + E.P.bytes;
  return E;
}

bool make_layout(const gcss_desc *d, int num_cu, Layout *L) {
  const int64_t m = d->m, n = d->n, k = d->k_max, r = d->r_max;
  L->ldq = ld_for(m);
  L->geo = stream_geometry(m, n, d->a_dtype, num_cu);
  if (L->geo.nj == 0) return false;
  L->qbuf = (size_t)L->geo.qlen;
  Carve c;
  L->f0 = c.take<double>(n);
  L->g0 = c.take<double>(n);
  L->f = c.take<double>(n);
  L->g = c.take<double>(n);
  L->mask0 = c.take<uint8_t>(n);
  L->mask = c.take<uint8_t>(n);
  L->part = c.take<ArgPart>(std::max(L->geo.grid, 1));
  L->qpart = c.take<double>(std::max(L->geo.grid, 1));
  L->npart = c.take<double>(1024);
  L->Q = c.take<double>((size_t)L->ldq * (k + 1));
  L->e1 = c.take<double>(L->ldq);
  L->e2 = c.take<double>(L->ldq);
  L->w = c.take<double>(L->ldq);
  const size_t qlen = std::max<size_t>(L->qbuf, L->ldq);
  L->q64 = c.take<double>(qlen);
  L->q32 = c.take<float>(qlen);
  L->z32 = c.take<float>(qlen);
  L->c1 = c.take<double>(k + 8);
  L->c2 = c.take<double>(k + 8);
  L->c3 = c.take<double>(k + 8);
  L->ups = c.take<double>(std::max<int64_t>(r, 1) + 8);
  L->st = c.take<DevState>(1);
  L->idx = c.take<int64_t>(k + 8);
  L->obj = c.take<double>(k + 8);
  L->scal = c.take<double>(64);
  L->pick = c.take<int64_t>(k + 8);
  L->quad = c.take<double>(k + 8);
  L->ap64 = c.take<double>(L->ldq);
  L->gram = d->self_target ? c.take<float>((size_t)L->ldq * m) : 0;
  // binary32 copy of a bfloat16 target (the values every B-reading kernel
  // takes), leading dimension ldq
  L->bexp = r > 0 ? c.take<float>((size_t)L->ldq * r) : 0;
  // the per-step chain: w history V (as Q), dot partials per row block of
  // 1024 rows (B = A: also C e2, m entries), and one norm and one q . w
  // partial per 32-row workgroup
  L->chain = chain_fits(m, r, (int)k, kChainLdsMax);
  L->lp = (int64_t)up((size_t)(std::max<int64_t>(r, d->self_target ? m : 0) + k + 1), 4);
  L->V = c.take<double>((size_t)L->ldq * (k + 1));
  L->P = c.take<double>((size_t)chain_row_blocks(m) * L->lp);
  L->Pn = c.take<double>(chain_row_groups(m));
  L->Pu = c.take<double>(chain_row_groups(m));
  // transient scratch: split-K partials, or the reconstruction-error buffers
  size_t s = 0;
  if (d->self_target) s = std::max(s, gram_scratch_bytes(m, n, L->ldq, num_cu));
  if (r > 0) s = std::max(s, proj_scratch_bytes(m, n, r, num_cu));
  const size_t err_bytes = up((size_t)std::max<int64_t>(r, 1) * 8, 256) +
                           up((size_t)L->ldq * k * 4, 256) + 3 * up((size_t)(k + 8) * 8, 256);
  s = std::max(s, err_bytes);
  if (r > 0) s = std::max(s, err_scratch_bytes(m, (int)k, r, num_cu));
  if (d->self_target) s = std::max(s, qta_scratch_bytes(n, (int)k));
  if (k <= kRankMaxL) s = std::max(s, rank_plan((int)k, n).bytes);
  if (d->self_target) {
    const int64_t smax = std::min<int64_t>(std::min<int64_t>(k, m), kRankMaxL);
    s = std::max(s, eig_layout(m, L->ldq, (int)smax, num_cu).bytes);
  }
  L->scratch_bytes = s;
  L->scratch = c.take<uint8_t>(s);
  L->total = up(c.off, 256);
  return true;
}

gcss_status check_desc(const gcss_desc *d) {
  if (!d) return fail(GCSS_ERR_ARG, "null descriptor");
  if (d->m < 1 || d->n < 1) return fail(GCSS_ERR_ARG, "m and n must be >= 1");
  if (d->a_dtype < GCSS_F32 || d->a_dtype > GCSS_FP8_E4M3)
    return fail(GCSS_ERR_ARG, "unknown a_dtype %d", d->a_dtype);
  const int es = dtype_bytes(d->a_dtype);
  if (d->lda < d->m) return fail(GCSS_ERR_ARG, "lda (%lld) < m (%lld)", (long long)d->lda, (long long)d->m);
  if ((d->lda * es) % 16 != 0) return fail(GCSS_ERR_ARG, "lda * element size must be a multiple of 16 bytes");
  if (d->k_max < 1 || d->k_max > d->n) return fail(GCSS_ERR_ARG, "k_max must be in [1, n]");
  if (d->r_max < 0) return fail(GCSS_ERR_ARG, "r_max must be >= 0");
  if (d->reserved != 0) return fail(GCSS_ERR_ARG, "reserved must be 0");
  if (d->m > 8192) return fail(GCSS_ERR_UNSUPPORTED, "m = %lld exceeds 8192", (long long)d->m);
  if (!d->self_target && d->r_max == 0)
    return fail(GCSS_ERR_ARG, "neither an explicit target (r_max) nor the self target reserved");
  return GCSS_OK;
}

}  // namespace

struct gcss_ctx {
  int device = 0;
  int num_cu = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  AView A{};
  gcss_desc d{};
  Layout L{};
  char *ws = nullptr;
  size_t ws_bytes = 0;
  int target = 0;  // 0 none, 1 explicit B, 2 Gram (B = A)
  // batched selection (Algorithm 4): cached group table and captured loop
  std::vector<GroupEnt> bgroups;
  std::vector<int64_t> bgfirst;
  std::vector<int64_t> bcol_off;
  std::vector<int32_t> bkb;  // per-block budgets of the captured graph
  int bkm = -1;              // its k_merge
  hipGraphExec_t bgraph = nullptr;
  // the merge selection's context (over the pooled columns, in the batched
  // region of the workspace), kept with the captured graph
  gcss_ctx *msub = nullptr;
  const float *B = nullptr;  // the target as binary32 (the caller's, or the copy of a BF16 one)
  int64_t r = 0, ldb = 0;
  const void *Braw = nullptr;  // the caller's target as given
  int b_dtype = GCSS_F32;
  int64_t ldb_raw = 0;
  // caller's embedding W = Q^T A (row-major k_max x ldw), or none
  float *emb = nullptr;
  int64_t ldw = 0;
  // Q (and obj) hold the basis (objective) of the last gcss_select(_async)
  // under the current target
  bool q_from_select = false;
  // last completed selection (host copy), for reuse of its basis
  std::vector<int64_t> last_idx;
  bool basis_valid = false;
  // event timing of the fused stream (gcss_select only)
  bool profiling = false;
  std::vector<hipEvent_t> ev;  // pairs around stream launches, then the loop pair
  size_t ev_used = 0;
  gcss_profile prof{};
  // launch settings of the streaming passes
  gcss_tuning tune{};
  // per-step work by the six-kernel chain (else the general cols / rows kernels)
  bool use_chain = false;
  bool chain_ok = true;  // the chain is allowed (GCSS_CHAIN=0 turns it off)
  // per-step kernels of the batched block phase: 0 the fastest that fits,
  // 1 one workgroup per block, 2 the six chain kernels, 3 the general
  // kernels (GCSS_BATCH_STEP=block / chain / general, for comparisons)
  int batch_step = 0;
  // merge of Algorithm 4 over its sub-context even where the pool's Gram
  // form fits (GCSS_MERGE=sub, for comparisons)
  bool merge_sub = false;
  // captured loops: select_async's (with its output copy) and select's
  hipGraphExec_t graph = nullptr;
  int graph_k = -1;
  hipGraphExec_t sgraph = nullptr;
  int sgraph_k = -1;
  void *graph_out[3] = {nullptr, nullptr, nullptr};

  template <typename T>
  T *at(size_t off) const { return (T *)(ws + off); }
  StepBufs bufs(const int64_t *pick_list = nullptr, int advance = 0) const {
    StepBufs sb{};
    sb.st = at<DevState>(L.st);
    sb.Q = at<double>(L.Q);
    sb.ldq = L.ldq;
    sb.q32 = at<float>(L.q32);
    sb.z32 = at<float>(L.z32);
    sb.q64 = at<double>(L.q64);
    sb.g0 = at<double>(L.g0);
    sb.mask = at<uint8_t>(L.mask);
    sb.idx = at<int64_t>(L.idx);
    sb.obj = at<double>(L.obj);
    sb.part = at<double>(L.npart);
    sb.pick_list = pick_list;
    sb.advance = advance;
    return sb;
  }
  double *F0() const { return at<double>(L.scal); }
  double *err_dev() const { return at<double>(L.scal) + 1; }
};

namespace {

void drop_graph(gcss_ctx *h) {
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  h->graph = nullptr;
  h->graph_k = -1;
  if (h->sgraph) (void)hipGraphExecDestroy(h->sgraph);
  h->sgraph = nullptr;
  h->sgraph_k = -1;
}


const char *tuning_error(const gcss_tuning &t) {
  if (t.stream_pd != 1 && t.stream_pd != 2) return "stream_pd must be 1 or 2";
  if (t.stream_upw < 1 || t.stream_upw > 64) return "stream_upw must be in 1..64";
  if (t.batch_group != 16 && t.batch_group != 32 && t.batch_group != 64)
    return "batch_group must be 16, 32 or 64";
  if (t.batch_wg_per_cu < 0 || t.batch_wg_per_cu > 64) return "batch_wg_per_cu must be in 0..64";
  return nullptr;
}

// Streaming-pass geometry under a launch setting: the shape follows from m
// and the storage type, the grid and the unit size from the setting and the
// kernel's occupancy.
hipError_t tuned_geometry(const gcss_desc *d, int num_cu, const gcss_tuning &t, StreamGeo *out) {
  StreamGeo geo = stream_geometry(d->m, d->n, d->a_dtype, num_cu);
  if (geo.nj == 0) return hipErrorInvalidValue;
  geo.pd = t.stream_pd;
  geo.upw = t.stream_upw;
  geo.g = t.batch_group;
  hipError_t e = stream_finalize(geo, d->n, d->a_dtype, num_cu);
  if (e == hipSuccess) *out = geo;
  return e;
}

// Gram-Schmidt of column p (state) against the basis, with one re-orthogonalisation.
hipError_t enqueue_basis_step(gcss_ctx *h, const StepBufs &sb) {
  const int64_t m = h->d.m, ldq = h->L.ldq;
  const int kmax = h->d.k_max;
  double *Q = h->at<double>(h->L.Q);
  double *e1 = h->at<double>(h->L.e1), *e2 = h->at<double>(h->L.e2);
  double *c1 = h->at<double>(h->L.c1), *c2 = h->at<double>(h->L.c2);
  hipStream_t s = h->stream;
  hipError_t e;
  // first projection of the pick's column: decoded to FP64 by the previous
  // stream pass, or (caller's pick list) decoded here
  const double *ap = h->at<double>(h->L.ap64);
  const int vs = sb.pick_list ? VEC_ACOL : VEC_F64;
  if ((e = launch_cols(Q, nullptr, ldq, m, 1, 0, kmax, vs, ap, h->A, c1, CF_NONE, sb, s))) return e;
  if ((e = launch_rows(Q, nullptr, ldq, m, 1, 0, vs, ap, h->A, c1, e1, nullptr, RF_NONE, sb, s))) return e;
  if ((e = launch_cols(Q, nullptr, ldq, m, 1, 0, kmax, VEC_F64, e1, h->A, c2, CF_NONE, sb, s))) return e;
  return launch_rows(Q, nullptr, ldq, m, 1, 0, VEC_F64, e1, h->A, c2, e2, nullptr, RF_GS2, sb, s);
}

hipEvent_t next_event(gcss_ctx *h) {
  if (h->ev_used == h->ev.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev.push_back(e);
  }
  return h->ev[h->ev_used++];
}

hipError_t record(gcss_ctx *h) {
  hipEvent_t e = next_event(h);
  if (!e) return hipErrorOutOfMemory;
  return hipEventRecord(e, h->stream);
}

// The per-step chain of six kernels (k_chain.hip): basis update, target ops.
hipError_t enqueue_chain(gcss_ctx *h) {
  ChainArgs ca{};
  ca.st = h->at<DevState>(h->L.st);
  ca.Q = h->at<double>(h->L.Q);
  ca.ldq = h->L.ldq;
  ca.V = h->at<double>(h->L.V);
  ca.a = h->at<double>(h->L.ap64);
  ca.e1 = h->at<double>(h->L.e1);
  ca.e2 = h->at<double>(h->L.e2);
  ca.P = h->at<double>(h->L.P);
  ca.lp = h->L.lp;
  ca.Pn = h->at<double>(h->L.Pn);
  ca.Pu = h->at<double>(h->L.Pu);
  if (h->target == 2) {
    ca.B = h->at<float>(h->L.gram);
    ca.ldb = h->L.ldq;
    ca.r = 0;
    ca.gram = 1;
  } else {
    ca.B = h->Braw;
    ca.ldb = h->ldb_raw;
    ca.r = h->r;
    ca.b_bf16 = h->b_dtype == GCSS_BF16;
  }
  ca.q64 = h->at<double>(h->L.q64);
  ca.q32 = h->at<float>(h->L.q32);
  ca.z32 = h->at<float>(h->L.z32);
  ca.g0 = h->at<double>(h->L.g0);
  ca.mask = h->at<uint8_t>(h->L.mask);
  ca.idx = h->at<int64_t>(h->L.idx);
  ca.obj = h->at<double>(h->L.obj);
  ca.m = h->d.m;
  ca.kmax = h->d.k_max;
  return launch_chain(ca, h->stream);
}

// Basis update and target ops of one step with the general column-dot and
// row-update kernels (k_gemv.hip): eight launches.
hipError_t enqueue_general(gcss_ctx *h) {
  const StepBufs sb = h->bufs();
  const int64_t m = h->d.m, ldq = h->L.ldq;
  const int kmax = h->d.k_max;
  double *Q = h->at<double>(h->L.Q);
  double *w = h->at<double>(h->L.w), *q64 = h->at<double>(h->L.q64);
  double *c3 = h->at<double>(h->L.c3), *ups = h->at<double>(h->L.ups);
  hipStream_t s = h->stream;
  hipError_t e;
  if ((e = enqueue_basis_step(h, sb))) return e;
  if (h->target == 1) {
    // upsilon = B^T q, ||upsilon||^2 ; w = B upsilon
    if ((e = launch_cols(nullptr, h->B, h->ldb, m, 0, (int)h->r, (int)h->r, VEC_F64, q64, h->A, ups, CF_UPS, sb, s))) return e;
    if ((e = launch_rows(nullptr, h->B, h->ldb, m, 0, (int)h->r, -1, nullptr, h->A, ups, w, nullptr, RF_NONE, sb, s))) return e;
    // c3 = Q_{t-1}^T w
    if ((e = launch_cols(Q, nullptr, ldq, m, 1, 0, kmax, VEC_F64, w, h->A, c3, CF_NONE, sb, s))) return e;
  } else {
    // w = (A A^T) q ; c3 = [Q_{t-1} q]^T w, ||upsilon||^2 = q . w
    const float *C = h->at<float>(h->L.gram);
    if ((e = launch_cols(nullptr, C, ldq, m, 0, (int)m, (int)m, VEC_F64, q64, h->A, w, CF_NONE, sb, s))) return e;
    if ((e = launch_cols(Q, nullptr, ldq, m, 1, 1, kmax + 1, VEC_F64, w, h->A, c3, CF_GRAM_U2, sb, s))) return e;
  }
  // z = w - Q_{t-1} c3 ; record the pick
  return launch_rows(Q, nullptr, ldq, m, 1, 0, VEC_F64, w, h->A, c3, nullptr, h->at<float>(h->L.z32), RF_Z, sb, s);
}

// Adds the timed streaming passes (event pairs from index x0 on) to the
// profile.  Passes that read no column -- the one after a selection's last
// pick (explicit targets), a rescore after a rejected pick, or a batched
// pass after every block has finished -- take a few microseconds against the
// full pass's hundreds; those under a quarter of the longest are left out,
// so the average is that of passes over A.
hipError_t add_stream_times(gcss_ctx *h, size_t x0) {
  std::vector<float> d;
  for (size_t x = x0; x + 1 < h->ev_used; x += 2) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, h->ev[x], h->ev[x + 1]);
    if (e) return e;
    d.push_back(ms);
  }
  float mx = 0.f;
  for (float v : d) mx = std::max(mx, v);
  for (float v : d)
    if (v >= 0.25f * mx) {
      h->prof.stream_ms += v;
      h->prof.stream_launches += 1;
    }
  return hipSuccess;
}

// One greedy step: basis update and target ops, then the fused stream
// (with profiling on and timed, between two events).
hipError_t enqueue_step(gcss_ctx *h, bool timed = true) {
  hipError_t e = h->use_chain ? enqueue_chain(h) : enqueue_general(h);
  if (e) return e;
  timed = timed && h->profiling;
  if (timed && (e = record(h))) return e;
  // Gram target: the pass also returns the exact decrease ||A^T q||^2
  const bool ex = h->target == 2;
  if ((e = launch_stream(h->L.geo, h->A, h->at<float>(h->L.q32), h->at<double>(h->L.q64),
                         h->at<float>(h->L.z32), h->at<double>(h->L.f), h->at<double>(h->L.g),
                         h->at<double>(h->L.g0), h->at<uint8_t>(h->L.mask),
                         h->at<ArgPart>(h->L.part), h->at<DevState>(h->L.st),
                         h->at<double>(h->L.ap64), 0, ex ? h->at<double>(h->L.qpart) : nullptr,
                         ex ? h->at<double>(h->L.quad) : nullptr, h->emb, h->ldw, h->stream)))
    return e;
  if (timed && (e = record(h))) return e;
  return hipSuccess;
}

// Gram target: the objective from the exact decrements ||A^T q_s||^2 that
// the streaming passes returned (the per-step decrements use the binary32
// Gram matrix).
hipError_t enqueue_exact_objective(gcss_ctx *h) {
  if (h->target != 2) return hipSuccess;
  const StepBufs sb = h->bufs();
  return launch_obj_from_quad(h->F0(), h->at<double>(h->L.quad), sb.st, sb.obj, h->stream);
}

hipError_t enqueue_begin(gcss_ctx *h, int k) {
  const StepBufs sb = h->bufs();
  hipError_t e = launch_select_begin(h->at<double>(h->L.f0), h->at<double>(h->L.g0),
                                     h->at<uint8_t>(h->L.mask0), h->at<double>(h->L.f),
                                     h->at<double>(h->L.g), h->at<uint8_t>(h->L.mask), h->d.n, sb,
                                     k, h->d.k_max, h->F0(), h->d.tau, h->stream);
  if (e) return e;
  // first argmax over the initial scores
  return launch_stream(h->L.geo, h->A, h->at<float>(h->L.q32), h->at<double>(h->L.q64),
                       h->at<float>(h->L.z32), h->at<double>(h->L.f), h->at<double>(h->L.g),
                       h->at<double>(h->L.g0), h->at<uint8_t>(h->L.mask),
                       h->at<ArgPart>(h->L.part), sb.st, h->at<double>(h->L.ap64), 1, nullptr,
                       nullptr, nullptr, 0, h->stream);
}

// Begin + k + kSpareSlots steps + the exact objective (and, with finish, the
// copy to the outputs) on the context's stream.
hipError_t enqueue_loop(gcss_ctx *h, int k, int64_t *d_idx, double *d_obj, int32_t *d_nsel,
                        bool finish) {
  hipError_t e = enqueue_begin(h, k);
  for (int i = 0; !e && i < k + kSpareSlots; ++i) e = enqueue_step(h);
  if (!e) e = enqueue_exact_objective(h);
  if (!e && finish) e = launch_finish(h->bufs(), k, d_idx, d_obj, d_nsel, h->stream);
  return e;
}

// Capture begin + k + kSpareSlots steps + the exact objective (and, with
// outputs given, the copy to them) on the capture stream and instantiate it.
hipError_t capture_loop(gcss_ctx *h, int k, int64_t *d_idx, double *d_obj, int32_t *d_nsel,
                        bool finish, hipGraphExec_t *out) {
  if (!h->cap_stream) {
    hipError_t e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e) return e;
  }
  hipStream_t user = h->stream;
  const bool prof = h->profiling;
  h->profiling = false;
  h->stream = h->cap_stream;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed);
  if (!e) e = enqueue_loop(h, k, d_idx, d_obj, d_nsel, finish);
  hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
  h->stream = user;
  h->profiling = prof;
  if (e || e2) {
    if (g) (void)hipGraphDestroy(g);
    return e ? e : e2;
  }
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e) *out = nullptr;
  return e;
}

gcss_status check_ctx(gcss_ctx *h) {
  if (!h) return fail(GCSS_ERR_ARG, "null context");
  return GCSS_OK;
}

}  // namespace

extern "C" {

const char *gcss_last_error(void) { return g_err.c_str(); }

const char *gcss_version(void) { return "gcss-mi355x 0.1 (gfx950)"; }

gcss_status gcss_workspace_size(const gcss_desc *d, size_t *bytes) {
  gcss_status s = check_desc(d);
  if (s != GCSS_OK) return s;
  if (!bytes) return fail(GCSS_ERR_ARG, "null bytes");
  Layout L;
  if (!make_layout(d, kPlanCU, &L)) return fail(GCSS_ERR_UNSUPPORTED, "m too large for the stream kernel");
  *bytes = L.total;
  return GCSS_OK;
}

}  // extern "C"

namespace {

// Everything gcss_create does, on a caller-provided context object (the
// no-allocation entry point keeps its context on the stack).
gcss_status init_ctx(gcss_ctx *h, const gcss_desc *d, void *workspace, size_t ws_bytes) {
  gcss_status st = check_desc(d);
  if (st != GCSS_OK) return st;
  if (!d->a) return fail(GCSS_ERR_ARG, "null A");
  if (((uintptr_t)d->a) % 16) return fail(GCSS_ERR_ARG, "A must be 16-byte aligned");
  if (d->a_dtype == GCSS_FP8_E4M3 && !d->a_scale) return fail(GCSS_ERR_ARG, "FP8 A needs a_scale");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(GCSS_ERR_DEVICE, "no HIP device");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GCSS_ERR_DEVICE, "device %d is %s, not gfx950", dev, prop.gcnArchName);
  const int num_cu = std::min(prop.multiProcessorCount, kPlanCU);
  Layout L;
  if (!make_layout(d, num_cu, &L)) return fail(GCSS_ERR_UNSUPPORTED, "m too large for the stream kernel");
  if (!workspace) return fail(GCSS_ERR_WORKSPACE, "null workspace");
  if (((uintptr_t)workspace) % 256) return fail(GCSS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(GCSS_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

  // launch settings of the streaming passes: defaults, which the environment
  // (GCSS_STREAM_PD, GCSS_STREAM_UPW, GCSS_STREAM_G) may override, then the
  // grid and the unit from the kernel's occupancy
  gcss_tuning tune{1, 4, 64, 0};
  if (const char *v = getenv("GCSS_STREAM_G")) {
    const int gsz = atoi(v);
    if (gsz == 16 || gsz == 32 || gsz == 64) tune.batch_group = gsz;
  }
  if (const char *v = getenv("GCSS_STREAM_PD")) tune.stream_pd = atoi(v) >= 2 ? 2 : 1;
  if (const char *v = getenv("GCSS_STREAM_UPW")) tune.stream_upw = std::min(64, std::max(1, atoi(v)));
  {
    hipError_t fe = tuned_geometry(d, num_cu, tune, &L.geo);
    if (fe != hipSuccess) return fail(GCSS_ERR_DEVICE, "stream kernel occupancy: %s", hipGetErrorString(fe));
  }

  h->device = dev;
  h->num_cu = num_cu;
  h->stream = (hipStream_t)d->stream;
  h->d = *d;
  if (!(h->d.tau > 0.0)) h->d.tau = 1e-4;
  h->L = L;
  h->tune = tune;
  // per-step work: the six-kernel chain where it fits, else the general
  // column-dot / row-update kernels (GCSS_CHAIN=0 in the environment keeps
  // the general kernels, for comparisons)
  {
    const char *v = getenv("GCSS_CHAIN");
    h->chain_ok = !(v && atoi(v) == 0);
    h->use_chain = L.chain && h->chain_ok;
    const char *bs = getenv("GCSS_BATCH_STEP");
    h->batch_step = !bs ? 0 : !strcmp(bs, "block") ? 1 : !strcmp(bs, "chain") ? 2 : !strcmp(bs, "general") ? 3 : 0;
    const char *ms = getenv("GCSS_MERGE");
    h->merge_sub = ms && !strcmp(ms, "sub");
  }
  h->ws = (char *)workspace;
  h->ws_bytes = ws_bytes;
  h->A.a = d->a;
  h->A.scale = d->a_scale;
  h->A.m = d->m;
  h->A.n = d->n;
  h->A.lda = d->lda;
  h->A.dtype = d->a_dtype;
  // the stream kernels read q and z up to their padded length: zero the
  // padding once (kernels, not memsets, so the calls stay capturable)
  const size_t qlen = std::max<size_t>(L.qbuf, L.ldq);
  hipError_t e = launch_zero_f32(h->at<float>(L.q32), (int64_t)qlen, h->stream);
  if (!e) e = launch_zero_f32(h->at<float>(L.z32), (int64_t)qlen, h->stream);
  if (!e) e = launch_zero_f32(h->at<float>(L.q64), 2 * (int64_t)qlen, h->stream);
  if (e) return fail(GCSS_ERR_DEVICE, "init: %s", hipGetErrorString(e));
  return GCSS_OK;
}

}  // namespace

extern "C" {

gcss_status gcss_create(const gcss_desc *d, void *workspace, size_t ws_bytes, gcss_ctx **out) {
  if (!out) return fail(GCSS_ERR_ARG, "null out");
  *out = nullptr;
  gcss_ctx *h = new gcss_ctx();
  gcss_status st = init_ctx(h, d, workspace, ws_bytes);
  if (st != GCSS_OK) {
    delete h;
    return st;
  }
  *out = h;
  return GCSS_OK;
}

void gcss_destroy(gcss_ctx *h) {
  if (!h) return;
  drop_graph(h);
  if (h->bgraph) (void)hipGraphExecDestroy(h->bgraph);
  if (h->msub) gcss_destroy(h->msub);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  delete h;
}

gcss_status gcss_set_target(gcss_ctx *h, const void *b, int32_t b_dtype, int64_t r,
                            int64_t ldb) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  const int64_t m = h->d.m;
  if (b == nullptr && r == 0) {
    if (!h->d.self_target) return fail(GCSS_ERR_STATE, "self target not reserved at creation");
    h->q_from_select = false;
    float *C = h->at<float>(h->L.gram);
    HIPCHK(launch_gram(h->A, C, h->L.ldq, h->at<void>(h->L.scratch), h->num_cu, h->stream));
    HIPCHK(launch_init_gram(C, h->L.ldq, h->A, h->at<double>(h->L.f0), h->at<double>(h->L.g0),
                            h->at<uint8_t>(h->L.mask0), h->stream));
    HIPCHK(launch_sum_f64(h->at<double>(h->L.g0), h->d.n, h->F0(), h->at<double>(h->L.npart), 1024, h->stream));
    h->target = 2;
    h->B = nullptr;
    h->r = 0;
    h->ldb = 0;
    h->Braw = nullptr;
    h->b_dtype = GCSS_F32;
    h->ldb_raw = 0;
  } else {
    if (!b) return fail(GCSS_ERR_ARG, "null B with r = %lld", (long long)r);
    if (b_dtype != GCSS_F32 && b_dtype != GCSS_BF16)
      return fail(GCSS_ERR_ARG, "b_dtype must be GCSS_F32 or GCSS_BF16");
    if (r < 1 || r > h->d.r_max) return fail(GCSS_ERR_ARG, "r = %lld outside [1, r_max = %lld]", (long long)r, (long long)h->d.r_max);
    const int64_t es = b_dtype == GCSS_F32 ? 4 : 2;
    if (ldb < m || (ldb * es) % 16) return fail(GCSS_ERR_ARG, "ldb must be >= m and ldb * element size a multiple of 16 bytes");
    if (((uintptr_t)b) % 16) return fail(GCSS_ERR_ARG, "B must be 16-byte aligned");
    h->q_from_select = false;
    const float *bf = (const float *)b;
    int64_t ldbf = ldb;
    if (b_dtype == GCSS_BF16) {
      // the bfloat16 values, exactly, as binary32 for the kernels that read B
      float *x = h->at<float>(h->L.bexp);
      HIPCHK(launch_bf16_to_f32(b, m, r, ldb, x, h->L.ldq, h->stream));
      bf = x;
      ldbf = h->L.ldq;
    }
    HIPCHK(launch_init_factor(bf, ldbf, r, h->A, h->at<double>(h->L.f0), h->at<double>(h->L.g0),
                              h->at<uint8_t>(h->L.mask0), h->stream));
    // (the step buffer for upsilon, r_max + 8 doubles, is free here)
    HIPCHK(launch_sumsq_f32(bf, m, r, ldbf, h->F0(), h->at<double>(h->L.ups), h->stream));
    h->target = 1;
    h->B = bf;
    h->r = r;
    h->ldb = ldbf;
    h->Braw = b;
    h->b_dtype = b_dtype;
    h->ldb_raw = ldb;
  }
  h->basis_valid = false;
  drop_graph(h);
  if (h->bgraph) (void)hipGraphExecDestroy(h->bgraph);
  h->bgraph = nullptr;
  return GCSS_OK;
}

gcss_status gcss_project_target(gcss_ctx *h, const float *omega, int64_t r, void *b_out,
                                int32_t b_dtype, int64_t ldb) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (!omega || !b_out) return fail(GCSS_ERR_ARG, "null omega or b_out");
  if (r < 1 || r > h->d.r_max) return fail(GCSS_ERR_ARG, "r outside [1, r_max]");
  if (b_dtype != GCSS_F32 && b_dtype != GCSS_BF16)
    return fail(GCSS_ERR_ARG, "b_dtype must be GCSS_F32 or GCSS_BF16");
  const int64_t es = b_dtype == GCSS_F32 ? 4 : 2;
  if (ldb < h->d.m || (ldb * es) % 16) return fail(GCSS_ERR_ARG, "ldb must be >= m and ldb * element size a multiple of 16 bytes");
  if (((uintptr_t)omega) % 16 || ((uintptr_t)b_out) % 16) return fail(GCSS_ERR_ARG, "omega and b_out must be 16-byte aligned");
  if (b_dtype == GCSS_F32) {
    HIPCHK(launch_project(h->A, omega, r, (float *)b_out, ldb, h->at<void>(h->L.scratch), h->num_cu, h->stream));
  } else {
    // binary32 product into the target copy, rounded once (nearest, ties
    // to even) into the caller's bfloat16 buffer, which becomes the target
    float *x = h->at<float>(h->L.bexp);
    HIPCHK(launch_project(h->A, omega, r, x, h->L.ldq, h->at<void>(h->L.scratch), h->num_cu, h->stream));
    HIPCHK(launch_quantize(x, h->d.m, r, h->L.ldq, GCSS_BF16, b_out, ldb, nullptr, h->stream));
  }
  return gcss_set_target(h, b_out, b_dtype, r, ldb);
}

gcss_status gcss_project_sign(gcss_ctx *h, uint64_t seed, double density, int64_t r,
                             float *b_out, int64_t ldb) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (!b_out) return fail(GCSS_ERR_ARG, "null b_out");
  if (r < 1 || r > h->d.r_max) return fail(GCSS_ERR_ARG, "r outside [1, r_max]");
  if (!(density > 0.0 && density <= 1.0)) return fail(GCSS_ERR_ARG, "density must be in (0, 1]");
  if (ldb < h->d.m || (ldb * 4) % 16) return fail(GCSS_ERR_ARG, "ldb must be >= m and a multiple of 4");
  if (((uintptr_t)b_out) % 16) return fail(GCSS_ERR_ARG, "b_out must be 16-byte aligned");
  HIPCHK(launch_project_sign(h->A, seed, density, r, b_out, ldb, h->at<void>(h->L.scratch),
                             h->L.scratch_bytes, h->stream));
  return gcss_set_target(h, b_out, GCSS_F32, r, ldb);
}

gcss_status gcss_select(gcss_ctx *h, int32_t k, int64_t *idx, double *objective,
                        int32_t *n_selected) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (!idx) return fail(GCSS_ERR_ARG, "null idx");
  if (k < 1 || k > h->d.k_max) return fail(GCSS_ERR_ARG, "k = %d outside [1, k_max = %d]", k, h->d.k_max);
  if (!h->target) return fail(GCSS_ERR_STATE, "no target set");
  hipEvent_t loop0 = nullptr, loop1 = nullptr;
  if (h->profiling) {
    h->ev_used = 0;
    loop0 = next_event(h);
    loop1 = next_event(h);
    if (!loop0 || !loop1) return fail(GCSS_ERR_DEVICE, "event create failed");
    HIPCHK(hipEventRecord(loop0, h->stream));
  }
  // The loop is replayed from a captured graph (begin, k + spare steps, the
  // exact objective); with profiling on it is enqueued directly, with events.
  int64_t ran = 0;
  if (h->profiling) {
    HIPCHK(enqueue_begin(h, k));
    // the pass after the k-th pick reads A only for the Gram target's exact
    // decrease or an embedding row; otherwise it is left untimed
    const bool last_reads = h->target == 2 || h->emb != nullptr;
    for (int i = 0; i < k; ++i) HIPCHK(enqueue_step(h, i + 1 < k || last_reads));
    ran = k;
  } else {
    if (!h->sgraph || h->sgraph_k != k) {
      if (h->sgraph) (void)hipGraphExecDestroy(h->sgraph);
      h->sgraph = nullptr;
      hipError_t e = capture_loop(h, k, nullptr, nullptr, nullptr, false, &h->sgraph);
      if (e) return fail(GCSS_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
      h->sgraph_k = k;
    }
    HIPCHK(hipGraphLaunch(h->sgraph, h->stream));
    ran = k + kSpareSlots;
  }
  DevState hs;
  // Every step either adds a pick or drops its candidate for good (a pick
  // the basis check rejects), so at most k + n steps end any selection.
  bool extra = false;
  for (;;) {
    HIPCHK(hipMemcpyAsync(&hs, h->at<DevState>(h->L.st), sizeof hs, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (hs.done) break;
    if (ran > (int64_t)k + h->d.n)
      return fail(GCSS_ERR_DEVICE, "selection did not finish after %lld steps", (long long)ran);
    int slots = k - hs.t;  // picks were rejected: run the missing steps
    if (slots < 1) slots = 1;
    for (int i = 0; i < slots; ++i) HIPCHK(enqueue_step(h));
    ran += slots;
    extra = true;
  }
  if (h->profiling || extra) HIPCHK(enqueue_exact_objective(h));
  if (h->profiling) {
    HIPCHK(hipEventRecord(loop1, h->stream));
    HIPCHK(hipEventSynchronize(loop1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, loop0, loop1));
    h->prof.loop_ms += ms;
    h->prof.selects += 1;
    HIPCHK(add_stream_times(h, 2));
  }
  std::vector<int64_t> hidx(k);
  std::vector<double> hobj(k + 1);
  HIPCHK(hipMemcpyAsync(hidx.data(), h->at<int64_t>(h->L.idx), sizeof(int64_t) * k, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(hobj.data(), h->at<double>(h->L.obj), sizeof(double) * (k + 1), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const int t = hs.t;
  for (int s = 0; s < k; ++s) idx[s] = s < t ? hidx[s] : -1;
  if (objective) {
    objective[0] = hobj[0];
    for (int s = 0; s < k; ++s) objective[s + 1] = s < t ? hobj[s + 1] : hobj[t];
  }
  if (n_selected) *n_selected = t;
  h->last_idx.assign(hidx.begin(), hidx.begin() + t);
  h->basis_valid = true;
  h->q_from_select = true;
  return hs.exhausted ? GCSS_WARN_EXHAUSTED : GCSS_OK;
}

gcss_status gcss_select_async(gcss_ctx *h, int32_t k, int64_t *d_idx, double *d_obj,
                              int32_t *d_nsel) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (!d_idx) return fail(GCSS_ERR_ARG, "null d_idx");
  if (k < 1 || k > h->d.k_max) return fail(GCSS_ERR_ARG, "k = %d outside [1, k_max = %d]", k, h->d.k_max);
  if (!h->target) return fail(GCSS_ERR_STATE, "no target set");
  const bool reuse = h->graph && h->graph_k == k && h->graph_out[0] == (void *)d_idx &&
                     h->graph_out[1] == (void *)d_obj && h->graph_out[2] == (void *)d_nsel;
  if (!reuse) {
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    h->graph_k = -1;
    hipError_t e = capture_loop(h, k, d_idx, d_obj, d_nsel, true, &h->graph);
    if (e) return fail(GCSS_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    h->graph_k = k;
    h->graph_out[0] = d_idx;
    h->graph_out[1] = d_obj;
    h->graph_out[2] = d_nsel;
  }
  HIPCHK(hipGraphLaunch(h->graph, h->stream));
  h->basis_valid = false;  // the host does not know the picks
  h->q_from_select = true;
  return GCSS_OK;
}

gcss_status gcss_reconstruction_error(gcss_ctx *h, const int64_t *idx, int32_t k, double *err) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (!err) return fail(GCSS_ERR_ARG, "null err");
  if (!h->target) return fail(GCSS_ERR_STATE, "no target set");
  if (k < 0 || k > h->d.k_max) return fail(GCSS_ERR_ARG, "k = %d outside [0, k_max]", k);
  if (k > 0 && !idx) return fail(GCSS_ERR_ARG, "null idx");
  std::vector<int64_t> v(idx, idx + k);
  for (int s = 0; s < k; ++s)
    if (v[s] < 0 || v[s] >= h->d.n) return fail(GCSS_ERR_ARG, "idx[%d] = %lld out of range", s, (long long)v[s]);
  {
    std::vector<int64_t> sorted(v);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(GCSS_ERR_ARG, "idx has repeated columns");
  }
  const int64_t m = h->d.m, ldq = h->L.ldq;
  hipStream_t s = h->stream;
  int kb = k;  // basis size
  const bool reuse = h->basis_valid && k <= (int)h->last_idx.size() &&
                     std::equal(v.begin(), v.end(), h->last_idx.begin());
  if (!reuse && k > 0) {
    int64_t *pick = h->at<int64_t>(h->L.pick);
    HIPCHK(hipMemcpyAsync(pick, v.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
    const StepBufs sb = h->bufs(pick, 1);
    // fresh state in basis-only mode
    HIPCHK(launch_select_begin(h->at<double>(h->L.f0), h->at<double>(h->L.g0), h->at<uint8_t>(h->L.mask0),
                               h->at<double>(h->L.f), h->at<double>(h->L.g), h->at<uint8_t>(h->L.mask),
                               h->d.n, sb, k, h->d.k_max, h->F0(), kBasisTau, s));
    for (int i = 0; i < k; ++i) HIPCHK(enqueue_basis_step(h, sb));
    DevState hs;
    HIPCHK(hipMemcpyAsync(&hs, sb.st, sizeof hs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    kb = hs.t;
    h->basis_valid = false;
    h->q_from_select = false;
  }
  const double *Q = h->at<double>(h->L.Q);
  char *scr = h->at<char>(h->L.scratch);
  if (h->target == 1) {
    HIPCHK(launch_err_tiled(Q, ldq, m, kb, h->B, h->ldb, h->r, scr, h->L.scratch_bytes, h->num_cu,
                            h->err_dev(), s));
  } else if (kb == 0) {
    HIPCHK(launch_sum_f64(h->F0(), 1, h->err_dev(), nullptr, 0, s));
  } else {
    // ||A||^2 - sum_s ||A^T q_s||^2; the selection that built this basis
    // already computed the terms exactly (quad), so only a fresh basis needs them
    double *quad = h->at<double>(h->L.quad);
    if (!reuse) HIPCHK(launch_qta(Q, ldq, kb, nullptr, h->A, (double *)scr, quad, s));
    HIPCHK(launch_gram_err(h->F0(), quad, kb, h->err_dev(), s));
  }
  HIPCHK(hipMemcpyAsync(err, h->err_dev(), sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return GCSS_OK;
}

gcss_status gcss_set_embedding(gcss_ctx *h, float *w, int64_t ldw) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (w && ldw < h->d.n) return fail(GCSS_ERR_ARG, "ldw (%lld) < n (%lld)", (long long)ldw, (long long)h->d.n);
  if (((uintptr_t)w) % 4) return fail(GCSS_ERR_ARG, "w must be 4-byte aligned");
  if (w != h->emb) drop_graph(h);
  h->emb = w;
  h->ldw = w ? ldw : 0;
  return GCSS_OK;
}

// Block Jacobi sweeps on the prepared G until it is diagonal (at most 30).
constexpr int kEigCheck = 4;  // subspace iterations between Rayleigh-Ritz checks

static gcss_status run_jacobi(gcss_ctx *h, const RankPlan &P, char *scr) {
  hipStream_t s = h->stream;
  int conv = 1;
  std::vector<int> flags((size_t)(P.L / 64));
  for (int sweep = 0; sweep < 30 && conv; ++sweep) {
    HIPCHK(launch_jacobi_sweep(P, scr, s));
    HIPCHK(hipMemcpyAsync(flags.data(), scr + P.flag, sizeof(int) * flags.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    conv = 0;
    for (int f : flags) conv |= f;
  }
  if (conv) return fail(GCSS_ERR_DEVICE, "eigen-decomposition did not converge in 30 sweeps");
  return GCSS_OK;
}

gcss_status gcss_top_eig(gcss_ctx *h, int32_t s_block, int32_t max_iters, double tol, uint64_t seed,
                         int32_t k, double *lambda, double *u, int64_t ldu, float *b_out,
                         int64_t ldb, int32_t *iters, double *change) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  const int64_t m = h->d.m, ldq = h->L.ldq;
  if (!lambda) return fail(GCSS_ERR_ARG, "null lambda");
  if (h->target != 2) return fail(GCSS_ERR_STATE, "needs the Gram matrix of A (set_target(NULL) first)");
  const int64_t smax = std::min<int64_t>(std::min<int64_t>(h->d.k_max, m), kRankMaxL);
  if (s_block < 1 || s_block > smax) return fail(GCSS_ERR_ARG, "block width s = %d outside [1, %lld]", s_block, (long long)smax);
  if (k < 1 || k > s_block) return fail(GCSS_ERR_ARG, "need 1 <= k <= s");
  if (max_iters < 1 || max_iters > 100) return fail(GCSS_ERR_ARG, "max_iters outside [1, 100]");
  if (!(tol >= 0.0)) return fail(GCSS_ERR_ARG, "tol must be >= 0");
  if (u && (ldu < m || ((uintptr_t)u) % 8)) return fail(GCSS_ERR_ARG, "ldu < m or misaligned u");
  if (b_out && (!u || ldb < m || ((uintptr_t)b_out) % 16 || (ldb * 4) % 16))
    return fail(GCSS_ERR_ARG, "b_out needs u, ldb >= m (multiple of 4) and 16-byte alignment");
  const int sb = s_block;
  const EigLayout E = eig_layout(m, ldq, sb, h->num_cu);
  if (E.bytes > h->L.scratch_bytes) return fail(GCSS_ERR_UNSUPPORTED, "workspace too small for s = %d", sb);
  hipStream_t st = h->stream;
  char *scr = h->at<char>(h->L.scratch);
  float *Y = (float *)(scr + E.y), *Qf = (float *)(scr + E.qf), *Qr = (float *)(scr + E.qr);
  char *rs = scr + E.rank;
  const AView C{h->at<float>(h->L.gram), nullptr, m, m, ldq, GCSS_F32};
  // Y = C Omega with a dense random sign Omega (m x s, drawn in the kernel)
  HIPCHK(launch_project_sign_dense(C, (uint32_t)seed, (uint32_t)(seed >> 32), sign_threshold(1.0), sb,
                                   Y, ldq, scr, st));
  std::vector<double> sig((size_t)sb);
  double prev = -1.0, last_change = 0.0;
  int it = 0;
  for (it = 1; it <= max_iters; ++it) {
    // Q = orth(Y): Cholesky QR (Y <- Y R^-1, R^T R = Y^T Y); a second pass
    // before each Rayleigh-Ritz check, where Q must be orthonormal to
    // rounding (the power steps in between tolerate the first pass's error)
    const bool check = it % kEigCheck == 0 || it == max_iters;
    const int passes = check ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
      const float *src = pass == 0 ? Y : Qf;
      float *dst = pass == 0 ? Qf : Y;
      HIPCHK(launch_wgram(E.P, src, ldq, sb, m, rs, st));
      HIPCHK(launch_cholqr_apply(E.P, rs, sb, src, ldq, m, dst, ldq, st));
    }
    // the orthonormal block is in Qf after one pass, in Y after two; Y <- C Q
    if (passes == 2) HIPCHK(hipMemcpyAsync(Qf, Y, (size_t)ldq * sb * 4, hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_to_rowmajor(Qf, ldq, m, sb, Qr, st));
    HIPCHK(launch_project(C, Qr, sb, Y, ldq, scr, h->num_cu, st));
    // Rayleigh-Ritz every kCheck iterations and at the last: T = Q^T C Q,
    // whose eigenvalues approximate C's leading ones
    if (!check) continue;
    HIPCHK(launch_wgram2(E.P, Qf, Y, ldq, sb, m, rs, st));
    gcss_status g = run_jacobi(h, E.P, rs);
    if (g) return g;
    HIPCHK(launch_eig_order(E.P, rs, sb, k, st));
    HIPCHK(hipMemcpyAsync(sig.data(), rs + E.P.sigma, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double sum = 0.0;
    for (int j = 0; j < k; ++j) sum += sig[j] * sig[j];
    last_change = prev < 0.0 ? 1.0 : std::fabs(sum - prev) / std::max(sum, 1e-300);
    prev = sum;
    if (last_change <= tol) break;
  }
  if (it > max_iters) it = max_iters;
  for (int j = 0; j < k; ++j) lambda[j] = sig[j] * sig[j];
  if (u) {
    // u = Q U_T[:, :k] with Q in FP64 (the selection basis is overwritten)
    double *Q64 = h->at<double>(h->L.Q);
    HIPCHK(launch_cols_to_f64(Qf, ldq, m, sb, Q64, ldq, st));
    h->q_from_select = false;
    h->basis_valid = false;
    HIPCHK(launch_ritz_vectors(E.P, rs, sb, k, Q64, ldq, m, u, ldu, st));
    if (b_out) HIPCHK(launch_scale_cols(E.P, rs, u, ldu, m, k, b_out, ldb, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (iters) *iters = it;
  if (change) *change = last_change;
  return GCSS_OK;
}

gcss_status gcss_rank_k(gcss_ctx *h, const float *w, int64_t ldw, int32_t l, int32_t k, double *u,
                        int64_t ldu, float *v, int64_t ldv, double *sigma, double *err) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  const int64_t m = h->d.m, n = h->d.n;
  if (!w || !sigma) return fail(GCSS_ERR_ARG, "null w or sigma");
  if (ldw < n) return fail(GCSS_ERR_ARG, "ldw (%lld) < n (%lld)", (long long)ldw, (long long)n);
  if (k < 1 || k > l) return fail(GCSS_ERR_ARG, "need 1 <= k <= l (k = %d, l = %d)", k, l);
  if (u && ldu < m) return fail(GCSS_ERR_ARG, "ldu < m");
  if (v && ldv < n) return fail(GCSS_ERR_ARG, "ldv < n");
  if (((uintptr_t)w) % 4 || ((uintptr_t)u) % 8 || ((uintptr_t)v) % 4)
    return fail(GCSS_ERR_ARG, "misaligned w, u or v");
  if (!h->q_from_select) return fail(GCSS_ERR_STATE, "no selection basis (select first, under the current target)");
  if (l > kRankMaxL || l > h->d.k_max) return fail(GCSS_ERR_UNSUPPORTED, "l = %d exceeds %d", l, kRankMaxL);
  const RankPlan P = rank_plan(l, n);
  if (P.bytes > h->L.scratch_bytes) return fail(GCSS_ERR_UNSUPPORTED, "workspace too small for l = %d", l);
  hipStream_t s = h->stream;
  DevState hs;
  HIPCHK(hipMemcpyAsync(&hs, h->at<DevState>(h->L.st), sizeof hs, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (l < 1 || l > hs.t) return fail(GCSS_ERR_ARG, "l = %d outside [1, picks of the last selection = %d]", l, hs.t);
  char *scr = h->at<char>(h->L.scratch);
  HIPCHK(launch_wgram(P, w, ldw, l, n, scr, s));
  {
    gcss_status g = run_jacobi(h, P, scr);
    if (g) return g;
  }
  HIPCHK(launch_rank_outputs(P, scr, l, k, h->at<double>(h->L.Q), h->L.ldq, m, u, ldu, w, ldw, n, v,
                             ldv, s));
  // ||A - Q W||^2: the selection's own objective for B = A, else
  // ||A||^2 - ||W||_F^2 (sum of g0 minus the sum of the eigenvalues)
  double sums[3] = {0.0, 0.0, 0.0};  // [unused floor, sum of eigenvalues, tail]
  double fres = 0.0;
  if (h->target == 2) {
    HIPCHK(hipMemcpyAsync(&fres, h->at<double>(h->L.obj) + l, sizeof(double), hipMemcpyDeviceToHost, s));
  } else {
    HIPCHK(launch_sum_f64(h->at<double>(h->L.g0), n, h->err_dev(), h->at<double>(h->L.npart), 1024, s));
    HIPCHK(hipMemcpyAsync(&fres, h->err_dev(), sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipMemcpyAsync(sums, scr + P.aux, sizeof sums, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(sigma, scr + P.sigma, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (h->target != 2) fres -= sums[1];
  if (err) *err = fres + sums[2];
  return GCSS_OK;
}

gcss_status gcss_qless_r(const float *w, int64_t n, int64_t ldw, const int64_t *idx, int32_t k,
                         float *r, int64_t ldr, void *stream) {
  if (!w || !idx || !r) return fail(GCSS_ERR_ARG, "null w, idx or r");
  if (n < 1 || ldw < n) return fail(GCSS_ERR_ARG, "need n >= 1 and ldw >= n");
  if (k < 1 || ldr < k) return fail(GCSS_ERR_ARG, "need k >= 1 and ldr >= k");
  if (k > 65535) return fail(GCSS_ERR_UNSUPPORTED, "k = %d exceeds 65535", k);
  if (((uintptr_t)w) % 4 || ((uintptr_t)r) % 4 || ((uintptr_t)idx) % 8)
    return fail(GCSS_ERR_ARG, "misaligned w, r or idx");
  HIPCHK(launch_qless_r(w, n, ldw, idx, k, r, ldr, (hipStream_t)stream));
  return GCSS_OK;
}

gcss_status gcss_set_profiling(gcss_ctx *h, int32_t enable) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  h->profiling = enable != 0;
  h->prof = gcss_profile{};
  return GCSS_OK;
}

gcss_status gcss_get_profile(gcss_ctx *h, gcss_profile *out) {
  if (check_ctx(h) || !out) return fail(GCSS_ERR_ARG, "null argument");
  *out = h->prof;
  return GCSS_OK;
}

namespace {

// Per-block buffers of the batched selection, carved after the context's own.
struct BLayout {
  size_t st, Q, ap64, e1, e2, w, q64, q32, z32, c1, c2, c3, ups, idx, obj, npart, groups, gfirst,
      gpart, bcnt, kb, V, P, Pn, Pu, pick, a0, sc0, mloc, mobj, mns, mglob, sub, total;
  int64_t sQ, sQ32, sIO, sC, sUps, ngroups_max;
  int64_t lp, sP, sPn;  // the per-step chain's partials per block
  bool chain;           // per-step work by the chain kernels, all blocks at once
  // the merge over the pool's Gram form (pools of at most kGramMergeMax slots)
  bool gm;
  size_t mst, GH, mf, mg, mg0, mex, mW, mU, mpart;
  int64_t ldgh;
};

constexpr int64_t kGramMergeMax = 2048;

gcss_desc sub_desc(const gcss_desc *d, int64_t npool, int32_t k_merge) {
  gcss_desc s = *d;
  s.n = npool;
  s.a = nullptr;
  s.a_scale = nullptr;
  s.k_max = k_merge;
  s.self_target = 0;
  return s;
}

bool make_blayout(const gcss_desc *d, const Layout &L, int nblocks, int kb, int km, BLayout *B) {
  const int64_t m = d->m, n = d->n, r = std::max<int64_t>(d->r_max, 1), ldq = L.ldq;
  B->sQ = ldq * (kb + 1);
  B->sQ32 = (int64_t)up(std::max<size_t>(L.qbuf, (size_t)ldq), 64);
  B->sIO = kb + 8;
  B->sC = kb + 8;
  B->sUps = r + 8;
  B->ngroups_max = n / 16 + nblocks + 1;
  Carve c;
  B->st = c.take<DevState>(nblocks);
  B->Q = c.take<double>((size_t)nblocks * B->sQ);
  B->ap64 = c.take<double>((size_t)nblocks * ldq);
  B->e1 = c.take<double>((size_t)nblocks * ldq);
  B->e2 = c.take<double>((size_t)nblocks * ldq);
  B->w = c.take<double>((size_t)nblocks * ldq);
  B->q64 = c.take<double>((size_t)nblocks * ldq);
  B->q32 = c.take<float>((size_t)nblocks * B->sQ32);
  B->z32 = c.take<float>((size_t)nblocks * B->sQ32);
  B->c1 = c.take<double>((size_t)nblocks * B->sC);
  B->c2 = c.take<double>((size_t)nblocks * B->sC);
  B->c3 = c.take<double>((size_t)nblocks * B->sC);
  B->ups = c.take<double>((size_t)nblocks * B->sUps);
  B->idx = c.take<int64_t>((size_t)nblocks * B->sIO);
  B->obj = c.take<double>((size_t)nblocks * B->sIO);
  B->npart = c.take<double>((size_t)nblocks * 128);
  B->groups = c.take<GroupEnt>(B->ngroups_max);
  B->gfirst = c.take<int64_t>(nblocks + 1);
  B->gpart = c.take<ArgPart>(B->ngroups_max);
  B->bcnt = c.take<uint32_t>(64);
  B->kb = c.take<int32_t>(nblocks);
  // the chain's w history (as Q), dot partials and per-workgroup partials
  B->chain = chain_fits(m, r, kb, kChainLdsMax);
  B->lp = (int64_t)up((size_t)(r + kb + 1), 4);
  B->sP = (int64_t)chain_row_blocks(m) * B->lp;
  B->sPn = chain_row_groups(m);
  B->V = B->chain ? c.take<double>((size_t)nblocks * B->sQ) : 0;
  B->P = B->chain ? c.take<double>((size_t)nblocks * B->sP) : 0;
  B->Pn = B->chain ? c.take<double>((size_t)nblocks * B->sPn) : 0;
  B->Pu = B->chain ? c.take<double>((size_t)nblocks * B->sPn) : 0;
  // the pool: nblocks * kb slots (block-major), gathered into a0
  const int64_t P = (int64_t)nblocks * kb;
  B->pick = c.take<int64_t>(P);
  B->a0 = c.take<uint8_t>((size_t)P * d->lda * dtype_bytes(d->a_dtype));
  B->sc0 = c.take<float>(P);
  // the merge's outputs: local picks, objective, count, global picks
  B->mloc = c.take<int64_t>(km + 8);
  B->mobj = c.take<double>(km + 8);
  B->mns = c.take<int32_t>(64);
  B->mglob = c.take<int64_t>(km + 8);
  // the Gram form of the merge: G and H (P x (P + r)), scores, histories
  B->gm = P <= kGramMergeMax;
  B->ldgh = (int64_t)up((size_t)(P + r), 4);
  if (B->gm) {
    B->mst = c.take<DevState>(1);
    B->GH = c.take<double>((size_t)P * B->ldgh);
    B->mf = c.take<double>(P);
    B->mg = c.take<double>(P);
    B->mg0 = c.take<double>(P);
    B->mex = c.take<uint8_t>(P);
    B->mW = c.take<double>((size_t)(km + 1) * P);
    B->mU = c.take<double>((size_t)(km + 1) * r);
    B->mpart = c.take<ArgPart>(merge_step_groups(P));
  }
  if (km > P) return false;
  gcss_desc sd = sub_desc(d, P, km);
  Layout SL;
  if (!make_layout(&sd, kPlanCU, &SL)) return false;
  B->sub = c.take<uint8_t>(SL.total);
  B->total = up(c.off, 256);
  return true;
}

// One lockstep step of all blocks (timed: event pairs around the batched
// stream pass, when profiling is on).
hipError_t enqueue_batched_step(gcss_ctx *h, const BLayout &B, char *base, int nb, int kb,
                                int grid, bool timed = false) {
  auto at = [&](size_t off) { return base + off; };
  const int64_t m = h->d.m, ldq = h->L.ldq, r = h->r;
  double *Q = (double *)at(B.Q), *ap = (double *)at(B.ap64), *e1 = (double *)at(B.e1),
         *e2 = (double *)at(B.e2), *w = (double *)at(B.w), *q64 = (double *)at(B.q64),
         *c1 = (double *)at(B.c1), *c2 = (double *)at(B.c2), *c3 = (double *)at(B.c3),
         *ups = (double *)at(B.ups);
  float *q32 = (float *)at(B.q32), *z32 = (float *)at(B.z32);
  StepBufs sb{};
  sb.st = (DevState *)at(B.st);
  sb.Q = Q;
  sb.ldq = ldq;
  sb.q32 = q32;
  sb.z32 = z32;
  sb.q64 = q64;
  sb.g0 = h->at<double>(h->L.g0);
  sb.mask = h->at<uint8_t>(h->L.mask);
  sb.idx = (int64_t *)at(B.idx);
  sb.obj = (double *)at(B.obj);
  sb.part = (double *)at(B.npart);
  BatchStride bs{1, B.sQ, ldq, B.sQ32, B.sIO, 128};
  hipStream_t s = h->stream;
  hipError_t e;
  const AView &A = h->A;
  // one workgroup per block while a block's step is small (and there are
  // blocks enough to spread over the chip), else the six chain kernels with
  // every block along gridDim.z, else the general kernels
  const bool fits_block = B.chain && chain_block_fits(m, r, kb, kChainLdsMax);
  int mode = h->batch_step;
  if (mode == 0) mode = !h->chain_ok ? 3 : (fits_block && nb >= 16 && kb <= 64) ? 1 : B.chain ? 2 : 3;
  if (mode == 1 && !fits_block) mode = B.chain ? 2 : 3;
  if (mode == 2 && !B.chain) mode = 3;
  if (mode != 3) {
    ChainArgs ca{};
    ca.st = sb.st;
    ca.Q = Q;
    ca.ldq = ldq;
    ca.V = (double *)at(B.V);
    ca.a = ap;
    ca.e1 = e1;
    ca.e2 = e2;
    ca.P = (double *)at(B.P);
    ca.lp = B.lp;
    ca.Pn = (double *)at(B.Pn);
    ca.Pu = (double *)at(B.Pu);
    ca.B = h->Braw;
    ca.ldb = h->ldb_raw;
    ca.r = r;
    ca.b_bf16 = h->b_dtype == GCSS_BF16;
    ca.q64 = q64;
    ca.q32 = q32;
    ca.z32 = z32;
    ca.g0 = sb.g0;
    ca.mask = sb.mask;
    ca.idx = sb.idx;
    ca.obj = sb.obj;
    ca.m = m;
    ca.kmax = kb;
    ca.nprob = nb;
    ca.s_q = B.sQ;
    ca.s_vec = ldq;
    ca.s_p = B.sP;
    ca.s_pn = B.sPn;
    ca.s_q32 = B.sQ32;
    ca.s_io = B.sIO;
    if ((e = mode == 1 ? launch_chain_block(ca, s) : launch_chain(ca, s))) return e;
  } else {
  if ((e = launch_cols(Q, nullptr, ldq, m, 1, 0, kb, VEC_F64, ap, A, c1, CF_NONE, sb, s, nb, bs, ArgStride{B.sQ, ldq, B.sC, 0}))) return e;
  if ((e = launch_rows(Q, nullptr, ldq, m, 1, 0, VEC_F64, ap, A, c1, e1, nullptr, RF_NONE, sb, s, nb, bs, ArgStride{B.sQ, ldq, ldq, B.sC}))) return e;
  if ((e = launch_cols(Q, nullptr, ldq, m, 1, 0, kb, VEC_F64, e1, A, c2, CF_NONE, sb, s, nb, bs, ArgStride{B.sQ, ldq, B.sC, 0}))) return e;
  if ((e = launch_rows(Q, nullptr, ldq, m, 1, 0, VEC_F64, e1, A, c2, e2, nullptr, RF_GS2, sb, s, nb, bs, ArgStride{B.sQ, ldq, ldq, B.sC}))) return e;
  if ((e = launch_cols(nullptr, h->B, h->ldb, m, 0, (int)r, (int)r, VEC_F64, q64, A, ups, CF_UPS, sb, s, nb, bs, ArgStride{0, ldq, B.sUps, 0}))) return e;
  if ((e = launch_rows(nullptr, h->B, h->ldb, m, 0, (int)r, -1, nullptr, A, ups, w, nullptr, RF_NONE, sb, s, nb, bs, ArgStride{0, 0, ldq, B.sUps}))) return e;
  if ((e = launch_cols(Q, nullptr, ldq, m, 1, 0, kb, VEC_F64, w, A, c3, CF_NONE, sb, s, nb, bs, ArgStride{B.sQ, ldq, B.sC, 0}))) return e;
  if ((e = launch_rows(Q, nullptr, ldq, m, 1, 0, VEC_F64, w, A, c3, nullptr, z32, RF_Z, sb, s, nb, bs, ArgStride{B.sQ, ldq, 0, B.sC}))) return e;
  }
  if (timed && h->profiling && (e = record(h))) return e;
  if ((e = launch_stream_batched(h->L.geo, grid, A, (const GroupEnt *)at(B.groups), (int64_t)h->bgroups.size(), q32, z32, B.sQ32,
                                 h->at<double>(h->L.f), h->at<double>(h->L.g), h->at<double>(h->L.g0), h->at<uint8_t>(h->L.mask),
                                 (ArgPart *)at(B.gpart), (const DevState *)at(B.st), (uint32_t *)at(B.bcnt), 0, s))) return e;
  if (timed && h->profiling && (e = record(h))) return e;
  return launch_block_argmax(A, (const ArgPart *)at(B.gpart), (const int64_t *)at(B.gfirst), nb, (DevState *)at(B.st), ap, ldq, s);
}

}  // namespace

namespace {

// Tail of Algorithm 4 after the block phase, on the context's stream: the
// pool slots, the pooled columns gathered, the merge context's target and
// initial scores, its selection loop (outputs into the batched region) and
// the global indices of its picks.  No host involvement: it is captured with
// the block phase.
// The merge's arguments for the Gram form (k_merge.hip).
MergeArgs merge_args(gcss_ctx *h, const BLayout &B, char *base, int64_t P, int km) {
  MergeArgs a{};
  a.a0 = base + B.a0;
  a.sc0 = (const float *)(base + B.sc0);
  a.lda = h->d.lda;
  a.m = h->d.m;
  a.P = P;
  a.B = h->B;
  a.ldb = h->ldb;
  a.r = (int)h->r;
  a.GH = (double *)(base + B.GH);
  a.ldgh = B.ldgh;
  a.f = (double *)(base + B.mf);
  a.g = (double *)(base + B.mg);
  a.g0 = (double *)(base + B.mg0);
  a.excl = (uint8_t *)(base + B.mex);
  a.W = (double *)(base + B.mW);
  a.U = (double *)(base + B.mU);
  a.part = (ArgPart *)(base + B.mpart);
  a.st = (DevState *)(base + B.mst);
  a.loc = (int64_t *)(base + B.mloc);
  a.obj = (double *)(base + B.mobj);
  a.ns = (int32_t *)(base + B.mns);
  a.F0 = h->F0();
  a.tau = h->d.tau;
  a.k = km;
  return a;
}

bool use_gram_merge(const gcss_ctx *h, const BLayout &B, int km) {
  return B.gm && !h->merge_sub &&
         merge_gram_lds_bytes(km, (int)h->r) <= 48 * 1024;
}

hipError_t enqueue_merge(gcss_ctx *h, const BLayout &B, char *base, int nb, int kbm, int km) {
  hipStream_t s = h->stream;
  gcss_ctx *sub = h->msub;
  const int64_t P = (int64_t)nb * kbm;
  hipError_t e = launch_pool((const DevState *)(base + B.st), (const int64_t *)(base + B.idx), B.sIO,
                             kbm, nb, (int64_t *)(base + B.pick), s);
  if (!e) e = launch_gather_cols(h->A, (const int64_t *)(base + B.pick), P, base + B.a0,
                                 (float *)(base + B.sc0), s);
  if (e) return e;
  if (use_gram_merge(h, B, km)) {
    // the pool's Gram form: G and H once, then one launch per step (the
    // first only picks), spare steps for rejected picks
    const MergeArgs a = merge_args(h, B, base, P, km);
    e = launch_merge_gram(a, h->A.dtype, s);
    for (int i = 0; !e && i < km + 1 + kSpareSlots; ++i) e = launch_merge_step(a, s);
    if (!e) e = launch_merge_map((const int64_t *)(base + B.mloc), (const int64_t *)(base + B.pick), P,
                                 km, (int64_t *)(base + B.mglob), s);
    return e;
  }
  hipStream_t own = sub->stream;
  sub->stream = s;
  if (gcss_set_target(sub, h->B, GCSS_F32, h->r, h->ldb) != GCSS_OK) e = hipErrorInvalidValue;
  if (!e) e = enqueue_loop(sub, km, (int64_t *)(base + B.mloc), (double *)(base + B.mobj),
                           (int32_t *)(base + B.mns), true);
  sub->stream = own;
  if (!e) e = launch_merge_map((const int64_t *)(base + B.mloc), (const int64_t *)(base + B.pick), P,
                               km, (int64_t *)(base + B.mglob), s);
  return e;
}

// Block phase of Algorithm 4 on the context's stream: scores and states
// reset, the score-only pass, then kbm + kSpareSlots lockstep steps (timed:
// event pairs around the first kbm batched passes, when profiling is on).
hipError_t enqueue_blocks(gcss_ctx *h, const BLayout &B, char *base, int nb, int kbm, int grid,
                          bool timed) {
  hipStream_t s = h->stream;
  hipError_t e = launch_zero_f32((float *)(base + B.q32), (int64_t)nb * B.sQ32, s);
  // the stream kernel reads q and z up to the padded length: the padding
  // (never written by the step kernels) must hold zeros, whatever the
  // workspace held before
  if (!e) e = launch_zero_f32((float *)(base + B.z32), (int64_t)nb * B.sQ32, s);
  if (!e) e = launch_batch_begin(h->at<double>(h->L.f0), h->at<double>(h->L.g0), h->at<uint8_t>(h->L.mask0),
                                 h->at<double>(h->L.f), h->at<double>(h->L.g), h->at<uint8_t>(h->L.mask), h->d.n,
                                 (DevState *)(base + B.st), nb, (const int32_t *)(base + B.kb), kbm,
                                 (int64_t *)(base + B.idx), (double *)(base + B.obj), B.sIO, h->F0(), h->d.tau,
                                 (uint32_t *)(base + B.bcnt), s);
  if (!e) e = launch_stream_batched(h->L.geo, grid, h->A, (const GroupEnt *)(base + B.groups), (int64_t)h->bgroups.size(),
                                    (const float *)(base + B.q32), (const float *)(base + B.z32), B.sQ32,
                                    h->at<double>(h->L.f), h->at<double>(h->L.g), h->at<double>(h->L.g0),
                                    h->at<uint8_t>(h->L.mask), (ArgPart *)(base + B.gpart), (const DevState *)(base + B.st),
                                    (uint32_t *)(base + B.bcnt), 1, s);
  if (!e) e = launch_block_argmax(h->A, (const ArgPart *)(base + B.gpart), (const int64_t *)(base + B.gfirst), nb,
                                  (DevState *)(base + B.st), (double *)(base + B.ap64), h->L.ldq, s);
  // (the pass after the last pick of the largest budget, and the spare
  // steps, which return at once when every block is done, are not timed)
  for (int i = 0; !e && i < kbm + kSpareSlots; ++i)
    e = enqueue_batched_step(h, B, base, nb, kbm, grid, timed && i + 1 < kbm);
  return e;
}

// Budget rounding by largest remainders (the Algorithm 4 budgets other than
// floor(l / c)): floors of the shares capped at the widths, then the columns
// missing to min(l, n) one at a time to the block with the largest
// remainder among those with room, the lower block first on ties.  Every
// remainder of a block with room lies in [0, 1) after the floors, so this is
// a round robin over the blocks in that order, skipping full ones.
void round_budgets(const std::vector<double> &share, const std::vector<int64_t> &width, int64_t l,
                   int32_t *out) {
  const int c = (int)share.size();
  int64_t total = 0, cols = 0;
  for (int b = 0; b < c; ++b) {
    const int64_t f = std::min<int64_t>((int64_t)std::floor(share[b]), width[b]);
    out[b] = (int32_t)f;
    total += f;
    cols += width[b];
  }
  int64_t missing = std::min<int64_t>(l, cols) - total;
  std::vector<int> order(c);
  for (int b = 0; b < c; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (share[x] - out[x]) > (share[y] - out[y]);
  });
  while (missing > 0) {
    for (int x = 0; x < c && missing > 0; ++x) {
      const int b = order[x];
      if (out[b] < width[b]) {
        ++out[b];
        --missing;
      }
    }
  }
}

}  // namespace

gcss_status gcss_block_budgets(gcss_ctx *h, int32_t nblocks, const int64_t *col_off,
                               const double *norms2, int32_t l, int32_t policy,
                               int32_t *k_blocks) {
  if (!col_off || !k_blocks) return fail(GCSS_ERR_ARG, "null col_off or k_blocks");
  if (nblocks < 1 || l < 0) return fail(GCSS_ERR_ARG, "need nblocks >= 1 and l >= 0");
  if (policy != GCSS_BUDGET_UNIFORM && policy != GCSS_BUDGET_EVEN && policy != GCSS_BUDGET_NORM)
    return fail(GCSS_ERR_ARG, "unknown budget policy %d", policy);
  if (col_off[0] != 0) return fail(GCSS_ERR_ARG, "col_off must start at 0");
  std::vector<int64_t> width(nblocks);
  for (int b = 0; b < nblocks; ++b) {
    if (col_off[b + 1] <= col_off[b]) return fail(GCSS_ERR_ARG, "col_off must be strictly increasing");
    width[b] = col_off[b + 1] - col_off[b];
  }
  if (h && col_off[nblocks] != h->d.n) return fail(GCSS_ERR_ARG, "col_off must run from 0 to n");
  if (policy == GCSS_BUDGET_UNIFORM) {
    for (int b = 0; b < nblocks; ++b) k_blocks[b] = (int32_t)std::min<int64_t>(l / nblocks, width[b]);
    return GCSS_OK;
  }
  std::vector<double> share(nblocks, (double)l / nblocks);
  if (policy == GCSS_BUDGET_NORM) {
    std::vector<double> nrm(nblocks);
    if (norms2) {
      for (int b = 0; b < nblocks; ++b) nrm[b] = norms2[b];
    } else {
      // ||A_(b)||_F^2 from the context's FP64 column norms, summed per block
      // on the device in a fixed order
      if (check_ctx(h)) return fail(GCSS_ERR_ARG, "no context and no norms2");
      if (h->target == 0) return fail(GCSS_ERR_STATE, "column norms need a target (gcss_set_target)");
      const size_t need = up((size_t)(nblocks + 1) * 8, 256) + (size_t)nblocks * 8;
      if (need > h->L.scratch_bytes) return fail(GCSS_ERR_UNSUPPORTED, "too many blocks for the scratch");
      char *scr = h->at<char>(h->L.scratch);
      int64_t *off_d = (int64_t *)scr;
      double *out_d = (double *)(scr + up((size_t)(nblocks + 1) * 8, 256));
      HIPCHK(hipMemcpyAsync(off_d, col_off, (size_t)(nblocks + 1) * 8, hipMemcpyHostToDevice, h->stream));
      HIPCHK(launch_seg_sum(h->at<double>(h->L.g0), off_d, nblocks, out_d, h->stream));
      HIPCHK(hipMemcpyAsync(nrm.data(), out_d, (size_t)nblocks * 8, hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    double tot = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      if (!(nrm[b] >= 0.0) || !std::isfinite(nrm[b])) return fail(GCSS_ERR_ARG, "block norm %d not finite and >= 0", b);
      tot += nrm[b];
    }
    if (tot > 0.0)
      for (int b = 0; b < nblocks; ++b) share[b] = (double)l * nrm[b] / tot;
  }
  round_budgets(share, width, l, k_blocks);
  return GCSS_OK;
}

gcss_status gcss_batched_workspace_size(const gcss_desc *d, int32_t nblocks, int32_t k_block,
                                        int32_t k_merge, size_t *bytes) {
  gcss_status st = check_desc(d);
  if (st != GCSS_OK) return st;
  if (!bytes || nblocks < 1 || k_block < 1 || k_merge < 1) return fail(GCSS_ERR_ARG, "bad batched sizes");
  if ((int64_t)nblocks * k_block < k_merge) return fail(GCSS_ERR_ARG, "k_merge exceeds the pool (nblocks * k_block)");
  Layout L;
  if (!make_layout(d, kPlanCU, &L)) return fail(GCSS_ERR_UNSUPPORTED, "m too large for the stream kernel");
  BLayout B;
  if (!make_blayout(d, L, nblocks, k_block, k_merge, &B)) return fail(GCSS_ERR_UNSUPPORTED, "batched layout");
  *bytes = B.total + 256;
  return GCSS_OK;
}

gcss_status gcss_select_batched(gcss_ctx *h, int32_t nblocks, const int64_t *col_off,
                                int32_t k_block, int32_t k_merge, int64_t *idx_block,
                                int64_t *idx_merge, double *obj_merge, int32_t *n_merge) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (nblocks < 1 || k_block < 1) return fail(GCSS_ERR_ARG, "bad batched sizes");
  std::vector<int32_t> kb(nblocks, k_block);
  return gcss_select_batched_budgets(h, nblocks, col_off, kb.data(), k_merge, idx_block, idx_merge,
                                     obj_merge, n_merge);
}

gcss_status gcss_select_batched_budgets(gcss_ctx *h, int32_t nblocks, const int64_t *col_off,
                                        const int32_t *k_blocks, int32_t k_merge,
                                        int64_t *idx_block, int64_t *idx_merge, double *obj_merge,
                                        int32_t *n_merge) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (!col_off || !k_blocks || !idx_block || !idx_merge) return fail(GCSS_ERR_ARG, "null argument");
  if (nblocks < 1 || k_merge < 1) return fail(GCSS_ERR_ARG, "bad batched sizes");
  int kbm = 0;
  for (int b = 0; b < nblocks; ++b) {
    if (k_blocks[b] < 0) return fail(GCSS_ERR_ARG, "budget of block %d is negative", b);
    kbm = std::max(kbm, (int)k_blocks[b]);
  }
  if (kbm < 1) return fail(GCSS_ERR_ARG, "every block budget is zero");
  if ((int64_t)nblocks * kbm < k_merge) return fail(GCSS_ERR_ARG, "k_merge exceeds the pool (nblocks * max budget)");
  if (h->target != 1) return fail(GCSS_ERR_STATE, "batched selection needs an explicit target B");
  if (col_off[0] != 0 || col_off[nblocks] != h->d.n) return fail(GCSS_ERR_ARG, "col_off must run from 0 to n");
  for (int b = 0; b < nblocks; ++b) {
    if (col_off[b + 1] <= col_off[b]) return fail(GCSS_ERR_ARG, "col_off must be strictly increasing");
    if (k_blocks[b] > col_off[b + 1] - col_off[b]) return fail(GCSS_ERR_ARG, "budget of block %d exceeds its width", b);
  }
  BLayout B;
  if (!make_blayout(&h->d, h->L, nblocks, kbm, k_merge, &B)) return fail(GCSS_ERR_UNSUPPORTED, "batched layout");
  h->q_from_select = false;
  char *base = (char *)up((uintptr_t)(h->ws + h->L.total), 256);
  if ((size_t)(base - h->ws) + B.total > h->ws_bytes)
    return fail(GCSS_ERR_WORKSPACE, "workspace lacks the batched region (gcss_batched_workspace_size)");
  hipStream_t s = h->stream;
  const int64_t P = (int64_t)nblocks * kbm;

  // group table (groups of up to G consecutive columns, never across
  // blocks), budgets and the merge context: set up once per block layout
  std::vector<int64_t> off(col_off, col_off + nblocks + 1);
  std::vector<int32_t> kbv(k_blocks, k_blocks + nblocks);
  const bool same = h->bgraph && h->msub && h->bkb == kbv && h->bkm == k_merge && off == h->bcol_off;
  if (!same) {
    const int G = h->L.geo.g;
    h->bgroups.clear();
    h->bgfirst.assign(nblocks + 1, 0);
    for (int b = 0; b < nblocks; ++b) {
      h->bgfirst[b] = (int64_t)h->bgroups.size();
      for (int64_t c0 = off[b]; c0 < off[b + 1]; c0 += G)
        h->bgroups.push_back(GroupEnt{c0, (int32_t)std::min<int64_t>(G, off[b + 1] - c0), b});
    }
    h->bgfirst[nblocks] = (int64_t)h->bgroups.size();
    if ((int64_t)h->bgroups.size() > B.ngroups_max) return fail(GCSS_ERR_UNSUPPORTED, "too many column groups");
    HIPCHK(hipMemcpyAsync(base + B.groups, h->bgroups.data(), sizeof(GroupEnt) * h->bgroups.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(base + B.gfirst, h->bgfirst.data(), sizeof(int64_t) * h->bgfirst.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(base + B.kb, kbv.data(), sizeof(int32_t) * nblocks, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h->bgraph) (void)hipGraphExecDestroy(h->bgraph);
    h->bgraph = nullptr;
    if (h->msub) gcss_destroy(h->msub);
    h->msub = nullptr;
    h->bcol_off = off;
    h->bkb = kbv;
    h->bkm = k_merge;
    // the merge context over the pool slots (fixed addresses in the batched region)
    gcss_desc sd = sub_desc(&h->d, P, k_merge);
    sd.a = base + B.a0;
    sd.a_scale = h->d.a_dtype == GCSS_FP8_E4M3 ? (const float *)(base + B.sc0) : nullptr;
    sd.tau = h->d.tau;
    sd.stream = (void *)s;
    size_t sub_bytes = 0;
    gcss_status st = gcss_workspace_size(&sd, &sub_bytes);
    if (st != GCSS_OK) return st;
    st = gcss_create(&sd, base + B.sub, sub_bytes, &h->msub);
    if (st != GCSS_OK) {
      h->msub = nullptr;
      return st;
    }
  }
  int grid = 1;
  HIPCHK(batched_stream_grid(h->L.geo, h->d.a_dtype, h->num_cu, (int64_t)h->bgroups.size(),
                             h->tune.batch_wg_per_cu, &grid));

  // Block phase and merge: one captured graph, replayed; with profiling on
  // they are enqueued directly, with events around every batched pass
  if (h->profiling) {
    h->ev_used = 0;
    hipError_t e = enqueue_blocks(h, B, base, nblocks, kbm, grid, true);
    if (!e) e = enqueue_merge(h, B, base, nblocks, kbm, k_merge);
    if (e) return fail(GCSS_ERR_DEVICE, "batched selection: %s", hipGetErrorString(e));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(add_stream_times(h, 0));
    h->prof.selects += 1;
  } else {
    if (!h->bgraph) {
      if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
      drop_graph(h->msub);
      hipStream_t user = h->stream;
      h->stream = h->cap_stream;
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed);
      if (!e) e = enqueue_blocks(h, B, base, nblocks, kbm, grid, false);
      if (!e) e = enqueue_merge(h, B, base, nblocks, kbm, k_merge);
      hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
      h->stream = user;
      if (e || e2) {
        if (g) (void)hipGraphDestroy(g);
        return fail(GCSS_ERR_DEVICE, "batched capture failed: %s", hipGetErrorString(e ? e : e2));
      }
      e = hipGraphInstantiate(&h->bgraph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e) {
        h->bgraph = nullptr;
        return fail(GCSS_ERR_DEVICE, "batched graph instantiate: %s", hipGetErrorString(e));
      }
    }
    HIPCHK(hipGraphLaunch(h->bgraph, s));
  }

  // results: the pool slots (every block's picks), the block states, the
  // merge's picks, objective and state
  std::vector<int64_t> slots(P);
  std::vector<DevState> bst(nblocks);
  std::vector<int64_t> mg(k_merge);
  std::vector<double> mo(k_merge + 1);
  int32_t mns = 0;
  DevState mst;
  const bool gram = use_gram_merge(h, B, k_merge);
  auto fetch = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(slots.data(), base + B.pick, sizeof(int64_t) * P, hipMemcpyDeviceToHost, s);
    if (!e) e = hipMemcpyAsync(bst.data(), base + B.st, sizeof(DevState) * nblocks, hipMemcpyDeviceToHost, s);
    if (!e) e = hipMemcpyAsync(mg.data(), base + B.mglob, sizeof(int64_t) * k_merge, hipMemcpyDeviceToHost, s);
    if (!e) e = hipMemcpyAsync(mo.data(), base + B.mobj, sizeof(double) * (k_merge + 1), hipMemcpyDeviceToHost, s);
    if (!e) e = hipMemcpyAsync(&mns, base + B.mns, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    const DevState *mstp = gram ? (const DevState *)(base + B.mst) : h->msub->at<DevState>(h->msub->L.st);
    if (!e) e = hipMemcpyAsync(&mst, mstp, sizeof mst, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    return e;
  };
  HIPCHK(fetch());
  // Blocks whose basis check rejected more picks than the captured loop has
  // spare steps for: more lockstep steps (finished blocks skip them) until
  // every block has its budget or has run out of candidates (each step adds
  // a pick or drops a candidate, so this ends), then the merge again.
  bool redo = false;
  {
    int64_t wmax = 0;
    for (int b = 0; b < nblocks; ++b) wmax = std::max<int64_t>(wmax, off[b + 1] - off[b]);
    int64_t ran = 0;
    for (;;) {
      int need = 0;
      for (int b = 0; b < nblocks; ++b)
        if (!bst[b].done) need = std::max(need, std::max(1, k_blocks[b] - bst[b].t));
      if (need == 0) break;
      if (ran > (int64_t)kbm + wmax)
        return fail(GCSS_ERR_DEVICE, "batched selection did not finish after %lld extra steps", (long long)ran);
      for (int i = 0; i < need; ++i) HIPCHK(enqueue_batched_step(h, B, base, nblocks, kbm, grid));
      ran += need;
      HIPCHK(hipMemcpyAsync(bst.data(), base + B.st, sizeof(DevState) * nblocks, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      redo = true;
    }
  }
  if (redo) {
    hipError_t e = enqueue_merge(h, B, base, nblocks, kbm, k_merge);
    if (e) return fail(GCSS_ERR_DEVICE, "merge: %s", hipGetErrorString(e));
    HIPCHK(fetch());
  }
  // a merge whose basis check rejected more picks than its spare steps: the
  // missing steps, then its outputs again
  if (!mst.done && gram) {
    // the Gram form: more steps until done (each step adds a pick or drops
    // a candidate)
    const MergeArgs a = merge_args(h, B, base, P, k_merge);
    int64_t ran = 0;
    while (!mst.done) {
      if (ran > (int64_t)k_merge + P)
        return fail(GCSS_ERR_DEVICE, "merge selection did not finish after %lld extra steps", (long long)ran);
      const int need = std::max(1, k_merge - mst.t);
      for (int i = 0; i < need; ++i) HIPCHK(launch_merge_step(a, s));
      ran += need;
      HIPCHK(hipMemcpyAsync(&mst, base + B.mst, sizeof mst, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    HIPCHK(launch_merge_map((const int64_t *)(base + B.mloc), (const int64_t *)(base + B.pick), P, k_merge,
                            (int64_t *)(base + B.mglob), s));
    HIPCHK(fetch());
  } else if (!mst.done) {
    gcss_ctx *sub = h->msub;
    int64_t ran = 0;
    while (!mst.done) {
      if (ran > (int64_t)k_merge + P)
        return fail(GCSS_ERR_DEVICE, "merge selection did not finish after %lld extra steps", (long long)ran);
      const int need = std::max(1, k_merge - mst.t);
      for (int i = 0; i < need; ++i) HIPCHK(enqueue_step(sub));
      ran += need;
      HIPCHK(hipMemcpyAsync(&mst, sub->at<DevState>(sub->L.st), sizeof mst, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    HIPCHK(enqueue_exact_objective(sub));
    HIPCHK(launch_finish(sub->bufs(), k_merge, (int64_t *)(base + B.mloc), (double *)(base + B.mobj),
                         (int32_t *)(base + B.mns), s));
    HIPCHK(launch_merge_map((const int64_t *)(base + B.mloc), (const int64_t *)(base + B.pick), P, k_merge,
                            (int64_t *)(base + B.mglob), s));
    HIPCHK(fetch());
  }
  for (int64_t x = 0; x < P; ++x) idx_block[x] = slots[x];
  for (int j = 0; j < k_merge; ++j) idx_merge[j] = mg[j];
  if (obj_merge)
    for (int j = 0; j <= k_merge; ++j) obj_merge[j] = mo[j];
  if (n_merge) *n_merge = mns;
  h->basis_valid = false;
  return (mns < k_merge) ? GCSS_WARN_EXHAUSTED : GCSS_OK;
}

gcss_status gcss_gather_columns(gcss_ctx *h, const int64_t *idx, int64_t count, void *out,
                                float *out_scales) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (count < 0) return fail(GCSS_ERR_ARG, "count < 0");
  if (count == 0) return GCSS_OK;
  if (!idx || !out) return fail(GCSS_ERR_ARG, "null idx or out");
  if (h->d.a_dtype == GCSS_FP8_E4M3 && !out_scales) return fail(GCSS_ERR_ARG, "FP8 needs out_scales");
  if (((uintptr_t)out) % 16 || ((uintptr_t)idx) % 8) return fail(GCSS_ERR_ARG, "misaligned out or idx");
  HIPCHK(launch_gather_cols(h->A, idx, count, out, out_scales, h->stream));
  return GCSS_OK;
}

gcss_status gcss_quantize(const float *a, int64_t m, int64_t n, int64_t lda, int32_t dtype,
                          void *out, int64_t ldo, float *scales, void *stream) {
  if (!a || !out) return fail(GCSS_ERR_ARG, "null a or out");
  if (m < 1 || n < 1 || lda < m || ldo < m) return fail(GCSS_ERR_ARG, "bad sizes");
  if (dtype != GCSS_BF16 && dtype != GCSS_FP8_E4M3) return fail(GCSS_ERR_ARG, "dtype must be BF16 or FP8_E4M3");
  if (dtype == GCSS_FP8_E4M3 && !scales) return fail(GCSS_ERR_ARG, "FP8 needs scales");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(GCSS_ERR_DEVICE, "no HIP device");
  HIPCHK(launch_quantize(a, m, n, lda, dtype, out, ldo, scales, (hipStream_t)stream));
  return GCSS_OK;
}

gcss_status gcss_read_state(gcss_ctx *h, int32_t item, void *host, size_t bytes, size_t *copied) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (!host) return fail(GCSS_ERR_ARG, "null host");
  const int64_t n = h->d.n, m = h->d.m;
  const void *src = nullptr;
  size_t sz = 0, spitch = 0, width = 0, rows = 0;
  int32_t flags[4];
  DevState hs;
  HIPCHK(hipMemcpyAsync(&hs, h->at<DevState>(h->L.st), sizeof hs, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  switch (item) {
    case GCSS_STATE_F0: src = h->at<double>(h->L.f0); sz = 8 * n; break;
    case GCSS_STATE_G0: src = h->at<double>(h->L.g0); sz = 8 * n; break;
    case GCSS_STATE_F: src = h->at<double>(h->L.f); sz = 8 * n; break;
    case GCSS_STATE_G: src = h->at<double>(h->L.g); sz = 8 * n; break;
    case GCSS_STATE_Q:
      src = h->at<double>(h->L.Q); spitch = 8 * h->L.ldq; width = 8 * m; rows = hs.t; break;
    case GCSS_STATE_Z: src = h->at<float>(h->L.z32); sz = 4 * m; break;
    case GCSS_STATE_B:
      if (h->target != 1) return fail(GCSS_ERR_STATE, "no explicit target");
      src = h->B; spitch = 4 * h->ldb; width = 4 * m; rows = h->r; break;
    case GCSS_STATE_GRAM:
      if (h->target != 2) return fail(GCSS_ERR_STATE, "no Gram target");
      src = h->at<float>(h->L.gram); spitch = 4 * h->L.ldq; width = 4 * m; rows = m; break;
    case GCSS_STATE_NREJECT: src = &hs.n_reject; sz = 4; break;
    case GCSS_STATE_FLAGS: sz = sizeof flags; break;
    default: return fail(GCSS_ERR_ARG, "unknown item %d", item);
  }
  size_t done = 0;
  if (item == GCSS_STATE_FLAGS) {
    flags[0] = hs.t;
    flags[1] = hs.done;
    flags[2] = hs.exhausted;
    flags[3] = hs.n_reject;
    done = std::min(bytes, sz);
    memcpy(host, flags, done);
  } else if (item == GCSS_STATE_NREJECT) {
    done = std::min(bytes, sz);
    memcpy(host, src, done);
  } else if (width) {
    const size_t want = width * rows;
    const size_t nrows = std::min(rows, bytes / (width ? width : 1));
    if (nrows) HIPCHK(hipMemcpy2DAsync(host, width, src, spitch, width, nrows, hipMemcpyDeviceToHost, h->stream));
    done = nrows * width;
    (void)want;
  } else {
    done = std::min(bytes, sz);
    if (done) HIPCHK(hipMemcpyAsync(host, src, done, hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  if (copied) *copied = done;
  return GCSS_OK;
}

gcss_status gcss_get_tuning(gcss_ctx *h, gcss_tuning *out) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (!out) return fail(GCSS_ERR_ARG, "null tuning");
  *out = h->tune;
  return GCSS_OK;
}

gcss_status gcss_set_tuning(gcss_ctx *h, const gcss_tuning *t) {
  if (check_ctx(h)) return GCSS_ERR_ARG;
  if (!t) return fail(GCSS_ERR_ARG, "null tuning");
  if (const char *why = tuning_error(*t)) return fail(GCSS_ERR_ARG, "%s", why);
  StreamGeo geo{};
  hipError_t e = tuned_geometry(&h->d, h->num_cu, *t, &geo);
  if (e != hipSuccess) return fail(GCSS_ERR_DEVICE, "stream kernel occupancy: %s", hipGetErrorString(e));
  // captured loops hold the old grid and group table
  HIPCHK(hipStreamSynchronize(h->stream));
  drop_graph(h);
  if (h->bgraph) (void)hipGraphExecDestroy(h->bgraph);
  h->bgraph = nullptr;
  h->L.geo = geo;
  h->tune = *t;
  return GCSS_OK;
}

// ---- selection without device allocation -----------------------------------
// The workspace of gcss_select_static: one array per device, allocated when
// the library's code object is loaded and held until the process ends.  Its
// host-side name is a stand-in, not a device address: kernels and copies
// get the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[GCSS_STATIC_SCRATCH_BYTES];

}  // extern "C"

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch, looked up once per device.
gcss_status scratch_for_current_device(void **ptr) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GCSS_ERR_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GCSS_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return GCSS_OK;
}

}  // namespace

extern "C" {

gcss_status gcss_select_static(const gcss_desc *d, const void *b, int32_t b_dtype, int64_t r,
                               int64_t ldb, int32_t k, int64_t *d_idx, double *d_obj,
                               int32_t *d_nsel) {
  if (!d || !d_idx) return fail(GCSS_ERR_ARG, "null descriptor or d_idx");
  if (k < 1 || k > d->k_max) return fail(GCSS_ERR_ARG, "k = %d outside [1, k_max = %d]", k, d->k_max);
  size_t need = 0;
  gcss_status st = gcss_workspace_size(d, &need);
  if (st != GCSS_OK) return st;
  if (need > (size_t)GCSS_STATIC_SCRATCH_BYTES)
    return fail(GCSS_ERR_UNSUPPORTED,
                "problem needs %zu bytes of workspace; the static scratch holds %zu "
                "(use gcss_create with a caller workspace)",
                need, (size_t)GCSS_STATIC_SCRATCH_BYTES);
  void *ws = nullptr;
  if ((st = scratch_for_current_device(&ws)) != GCSS_OK) return st;
  gcss_ctx h;  // host state only, released on return; the device work keeps running
  if ((st = init_ctx(&h, d, ws, (size_t)GCSS_STATIC_SCRATCH_BYTES)) != GCSS_OK) return st;
  if ((st = gcss_set_target(&h, b, b_dtype, r, ldb)) != GCSS_OK) return st;
  // the loop of gcss_select_async, enqueued directly (no graph, no events)
  hipError_t e = enqueue_begin(&h, k);
  for (int i = 0; !e && i < k + kSpareSlots; ++i) e = enqueue_step(&h);
  if (!e) e = enqueue_exact_objective(&h);
  if (!e) e = launch_finish(h.bufs(), k, d_idx, d_obj, d_nsel, h.stream);
  if (e) return fail(GCSS_ERR_DEVICE, "static selection: %s", hipGetErrorString(e));
  return GCSS_OK;
}

static_assert(GCSS_PROBE_SINK_FLOATS == kProbeSinkFloats, "probe sink size");

gcss_status gcss_hbm_probe(const void *buf, size_t bytes, float *sink, int32_t reps, void *stream,
                           double *seconds) {
  if (!buf || !sink || !seconds) return fail(GCSS_ERR_ARG, "null argument");
  if (((uintptr_t)buf) % 16 || bytes < 16 || bytes % 16) return fail(GCSS_ERR_ARG, "buffer must be 16-byte aligned, a positive multiple of 16 bytes");
  if (reps < 1) return fail(GCSS_ERR_ARG, "reps must be positive");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GCSS_ERR_DEVICE, "device %d is %s, not gfx950", dev, prop.gcnArchName);
  hipStream_t s = (hipStream_t)stream;
  const int grid = hbm_probe_grid((int64_t)bytes, prop.multiProcessorCount);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (!e) e = launch_zero_f32(sink, kProbeSinkFloats, s);
  if (!e) e = launch_hbm_probe(buf, (int64_t)bytes, sink, grid, s);  // untimed first pass
  if (!e) e = hipEventRecord(e0, s);
  for (int i = 0; !e && i < reps; ++i) e = launch_hbm_probe(buf, (int64_t)bytes, sink, grid, s);
  if (!e) e = hipEventRecord(e1, s);
  if (!e) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (!e) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e) return fail(GCSS_ERR_DEVICE, "hbm probe: %s", hipGetErrorString(e));
  *seconds = (double)ms * 1e-3 / reps;
  return GCSS_OK;
}

}  // extern "C"

namespace gcss {

void set_error(const char *msg) { g_err = msg ? msg : ""; }

bool ctx_describe(gcss_ctx *h, CtxInfo *out) {
  if (!h || !out) return false;
  out->stream = h->stream;
  out->m = h->d.m;
  out->n = h->d.n;
  out->dtype = h->d.a_dtype;
  out->target = h->target;
  return true;
}

}  // namespace gcss
