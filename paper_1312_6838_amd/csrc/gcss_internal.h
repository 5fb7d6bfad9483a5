// Internal declarations shared by the HIP sources of the library.
// Nothing here is part of the public ABI (include/gcss.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

struct gcss_ctx;  // the C ABI's context (gcss_api.hip)

namespace gcss {

// Element codes of the stored source matrix (same values as gcss_dtype).
enum Dtype : int { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2 };

inline int dtype_bytes(int dt) { return dt == DT_F32 ? 4 : (dt == DT_BF16 ? 2 : 1); }

// Per-selection state kept in device memory so that a whole k-step loop can
// be enqueued (or replayed from a graph) without the host looking at it.
struct alignas(256) DevState {
  int32_t t;          // picks made so far
  int32_t k;          // picks wanted
  int32_t done;       // 1: no more work (t == k or no candidate left)
  int32_t exhausted;  // 1: ran out of candidates
  int32_t skip;       // 1: the current pick was rejected; the step only rescores
  int32_t n_reject;   // number of rejected picks
  int32_t pos;        // position in a caller's pick list (basis-only mode)
  int32_t dec_pending;  // 1: a pick was recorded whose exact decrease is not yet known
  int64_t p;          // current pick (-1 none)
  double F;           // objective after the last completed pick
  double u2;          // ||upsilon||^2 of the current step
  double enorm2;      // ||e||^2 of the current pick after re-orthogonalisation
  double tau;         // eligibility threshold
  uint32_t cnt[16];   // last-block-done counters (reset by their last block)
};

// Read-only view of the source matrix for kernels.
struct AView {
  const void *a;
  const float *scale;  // FP8 only
  int64_t m, n, lda;
  int dtype;
};

// Where the vector operand of a column-dot kernel comes from.
enum VecSrc : int { VEC_F64 = 0, VEC_ACOL = 1 };

// Last-block actions.
enum ColsFinal : int { CF_NONE = 0, CF_UPS = 1, CF_GRAM_U2 = 2 };
enum RowsFinal : int { RF_NONE = 0, RF_GS2 = 1, RF_Z = 2 };

// Argmax partial: best candidate of one workgroup.
struct alignas(16) ArgPart {
  double score;
  int64_t idx;
};

// Stream-kernel launch geometry (chosen once per context).
struct StreamGeo {
  int nj;        // 16-byte chunks per lane per wave slice
  int w;         // waves per team (column slice count)
  int g;         // columns per team group
  int grid;      // workgroups
  int grid_ex;   // workgroups of the exact-decrease variant (Gram target)
  int ucol_ex;   // its unit size
  int qlen;      // padded length of q32/z32
  int pd;        // load groups in flight ahead of the one being reduced (1, 2)
  int ucol;      // columns per team in one work unit of the queue
  int upw;       // work units per workgroup the unit size aims at
  int occ;       // resident workgroups per CU of the chosen kernel
};

// ---- launchers (k_stream.hip) ----
StreamGeo stream_geometry(int64_t m, int64_t n, int dtype, int num_cu);
// Sets the grid from the occupancy of the chosen kernel (needs the device).
hipError_t stream_finalize(StreamGeo &geo, int64_t n, int dtype, int num_cu);
// qpart/quad non-null: the exact-decrease variant (Gram target), which reads
// q64 and writes sum_i (A_i . q)^2 to quad[t - 1].  emb non-null: row t - 1
// of the row-major embedding W (leading dimension ldw) receives A_i . q.
hipError_t launch_stream(const StreamGeo &geo, const AView &A, const float *q32,
                         const double *q64, const float *z32, double *f, double *g,
                         const double *g0, uint8_t *mask, ArgPart *part, DevState *st,
                         double *ap64, int score_only, double *qpart, double *quad,
                         float *emb, int64_t ldw, hipStream_t s);

// ---- launchers (k_gemv.hip) ----
// Buffers of one selection problem that the per-step kernels touch.
struct StepBufs {
  DevState *st;
  double *Q;                   // basis, m x kcap FP64, column-major, ld ldq
  int64_t ldq;
  float *q32, *z32;            // stream operands (qlen floats, zero padded)
  double *q64;                 // q of the current step (m doubles)
  const double *g0;            // initial g (rejection threshold)
  uint8_t *mask;               // 0 candidate, 1 selected, 2 excluded
  int64_t *idx;                // picks (kcap)
  double *obj;                 // objective (kcap + 1)
  double *part;                // per-workgroup partial sums (>= 1024)
  const int64_t *pick_list;    // if set: the pick of step t is pick_list[t]
  int advance;                 // basis-only mode: the GS2 finish also advances t
};

// Several independent problems (the column blocks of Algorithm 4) run the
// same per-step kernels side by side: gridDim.y = number of problems, and
// problem b finds its buffers at the base pointers plus b times these
// strides (all zero for a single problem).
struct BatchStride {
  int64_t st;    // DevState entries
  int64_t Q;     // doubles between bases
  int64_t vec;   // doubles between the m-vectors (ap64, e1, e2, w, q64)
  int64_t q32;   // floats between q32 (and z32) vectors
  int64_t io;    // entries between idx / obj arrays
  int64_t part;  // doubles between norm-partial arrays
};

__device__ __forceinline__ StepBufs shift_bufs(StepBufs sb, const BatchStride &bs, int b) {
  sb.st += b * bs.st;
  sb.Q += b * bs.Q;
  sb.q32 += b * bs.q32;
  sb.z32 += b * bs.q32;
  sb.q64 += b * bs.vec;
  sb.idx += b * bs.io;
  sb.obj += b * bs.io;
  sb.part += b * bs.part;
  return sb;
}

// Strides of the vector arguments of one cols / rows launch (per problem).
struct ArgStride {
  int64_t m;    // matrix M (0: shared, e.g. the target B)
  int64_t vec;  // base vector
  int64_t out;  // output
  int64_t c;    // coefficients
};

// Column dots:  out[s] = sum_{j<m} M[j + s*ldm] * v[j],  s < ns,
//   ns = (ns_from_t ? st->t : 0) + ns_add; v = vec (VEC_F64) or column p of A
//   (VEC_ACOL).  M is FP64 (Mq) or FP32 (Mf).  final_mode: CF_*.
hipError_t launch_cols(const double *Mq, const float *Mf, int64_t ldm, int64_t m,
                       int ns_from_t, int ns_add, int max_ns, int vsrc, const double *vec,
                       const AView &A, double *out, int final_mode, const StepBufs &sb,
                       hipStream_t s, int nprob = 1, BatchStride bs = BatchStride{},
                       ArgStride as = ArgStride{});
// Row updates:  out[j] = v[j] - sum_{s<ns} M[j + s*ldm] * c[s]  (v given), or
//   out[j] = sum_{s<ns} M[j + s*ldm] * c[s]  (vsrc < 0: no v).  Writes out64
//   and/or out32.  final_mode: RF_*.
hipError_t launch_rows(const double *Mq, const float *Mf, int64_t ldm, int64_t m,
                       int ns_from_t, int ns_add, int vsrc, const double *vec, const AView &A,
                       const double *c, double *out64, float *out32, int final_mode,
                       const StepBufs &sb, hipStream_t s, int nprob = 1,
                       BatchStride bs = BatchStride{}, ArgStride as = ArgStride{});
// Start of a selection: f = f0, g = g0, mask = mask0, state reset, outputs cleared.
hipError_t launch_select_begin(const double *f0, const double *g0, const uint8_t *mask0,
                               double *f, double *g, uint8_t *mask, int64_t n,
                               const StepBufs &sb, int k, int kcap, const double *F0,
                               double tau, hipStream_t s);
// Copy picks/objective (filling past the last pick) to caller buffers.
hipError_t launch_finish(const StepBufs &sb, int k, int64_t *idx_out, double *obj_out,
                         int32_t *nsel_out, hipStream_t s);
// out[0] = sum of x[0..n) (fixed order), FP64
// Fixed-order FP64 sum; part (npart doubles of scratch) serves long inputs.
hipError_t launch_sum_f64(const double *x, int64_t n, double *out, double *part, int npart,
                          hipStream_t s);
// out[0] = sum of squares of an m x r FP32 column-major matrix (part: r doubles)
hipError_t launch_sumsq_f32(const float *B, int64_t m, int64_t r, int64_t ldb, double *out,
                            double *part, hipStream_t s);
// Residual of an explicit target on basis Q (k columns):
//   colerr[c] = || B_c - Q (Q^T B_c) ||^2, FP64
// err = || B - Q (Q^T B) ||_F^2 (Q: m x k FP64 basis, B: m x r binary32),
// tiled FP64 passes in the scratch (err_scratch_bytes); err on the device
size_t err_scratch_bytes(int64_t m, int k, int64_t r, int num_cu);
hipError_t launch_err_tiled(const double *Q, int64_t ldq, int64_t m, int k, const float *B,
                            int64_t ldb, int64_t r, void *scratch, size_t scratch_bytes,
                            int num_cu, double *err, hipStream_t s);
hipError_t launch_q_to_f32(const double *Q, int64_t ldq, int64_t m, int k, float *Q32,
                           int64_t ld32, hipStream_t s);
hipError_t launch_copy_i64(const int64_t *src, int64_t *dst, int64_t n, hipStream_t s);
// err = trace - sum_{s<k} quad[s]
hipError_t launch_gram_err(const double *trace, const double *quad, int k, double *err,
                           hipStream_t s);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t s);

// ---- the per-step chain of a single problem (k_chain.hip) ----
struct ChainArgs {
  DevState *st;
  double *Q;          // basis, ld ldq, columns < t read, column t written
  int64_t ldq;
  double *V;          // w history (m x (kmax + 1)), ld ldq
  const double *a;    // the pick's column in FP64
  double *e1, *e2;    // m each
  double *P;          // dot partials: row blocks x lp
  int64_t lp;         // >= r + kmax + 1 (B = A: m + kmax + 1)
  double *Pn, *Pu;    // one double per row workgroup each
  const void *B;      // explicit target (binary32 or bfloat16), or C = A A^T (binary32)
  int64_t ldb;
  int64_t r;          // target width (0 for B = A)
  int b_bf16;         // explicit target stored as bfloat16
  int gram;           // B = A through C
  double *q64;
  float *q32, *z32;
  const double *g0;
  uint8_t *mask;
  int64_t *idx;
  double *obj;
  int64_t m;
  int kmax;
  // several problems at once (Algorithm 4's blocks): problem b's state is
  // st + b and its buffers sit at these strides from problem 0's; B, g0 and
  // mask are shared (the blocks' columns are disjoint).  One problem: 1, 0s.
  int nprob;
  int64_t s_q;    // Q and V (doubles)
  int64_t s_vec;  // a, e1, e2, q64 (doubles)
  int64_t s_p;    // P (doubles)
  int64_t s_pn;   // Pn and Pu (doubles)
  int64_t s_q32;  // q32 and z32 (floats)
  int64_t s_io;   // idx and obj
};
int chain_row_blocks(int64_t m);
int chain_row_groups(int64_t m);
size_t chain_lds_bytes(int64_t r, int kmax);
// the chain serves the shape: m within its row blocks, r + kmax + 1 doubles of LDS
bool chain_fits(int64_t m, int64_t r, int kmax, size_t lds_max);
hipError_t launch_chain(const ChainArgs &ca, hipStream_t s);
// The same step with one workgroup per problem (small problems: m <= 2048,
// explicit target; ca.nprob problems at the strides of ChainArgs)
size_t chain_block_lds_bytes(int64_t m, int64_t r, int kmax);
bool chain_block_fits(int64_t m, int64_t r, int kmax, size_t lds_max);
hipError_t launch_chain_block(const ChainArgs &ca, hipStream_t s);

// ---- launchers (k_mfma.hip) ----
// f0_i = scale_i^2 * || X^T A_i ||^2 (X: m x R, K-contiguous, ldx), g0_i, mask0_i
hipError_t launch_init_factor(const float *X, int64_t ldx, int64_t R, const AView &A,
                              double *f0, double *g0, uint8_t *mask0, hipStream_t s);
// f0_i = scale_i^2 * A_i^T C A_i (C: m x m symmetric, ldc), g0_i, mask0_i
hipError_t launch_init_gram(const float *C, int64_t ldc, const AView &A, double *f0,
                            double *g0, uint8_t *mask0, hipStream_t s);
// C = A A^T (m x m, ldc) using split-K partials in scratch (bytes >= gram_scratch_bytes)
size_t gram_scratch_bytes(int64_t m, int64_t n, int64_t ldc, int num_cu);
hipError_t launch_gram(const AView &A, float *C, int64_t ldc, void *scratch, int num_cu,
                       hipStream_t s);
// B = A Omega (m x r, ldb); Omega n x r row-major
size_t proj_scratch_bytes(int64_t m, int64_t n, int64_t r, int num_cu);
hipError_t launch_project(const AView &A, const float *omega, int64_t r, float *B,
                          int64_t ldb, void *scratch, int num_cu, hipStream_t s);

// Exact decrements of the Gram target: quad[s] = ||A^T q_s||^2 for s < nrow,
// nrow = st->t (st given) or kmax.  scratch >= qta_scratch_bytes(n, kmax).
size_t qta_scratch_bytes(int64_t n, int kmax);
hipError_t launch_qta(const double *Q, int64_t ldq, int kmax, const DevState *st,
                      const AView &A, double *scratch, double *quad, hipStream_t s);
// obj[s+1] = F0 - sum_{x<=s} quad[x], s < st->t
hipError_t launch_obj_from_quad(const double *F0, const double *quad, const DevState *st,
                                double *obj, hipStream_t s);

// ---- launchers (k_quant.hip) ----
hipError_t launch_quantize(const float *a, int64_t m, int64_t n, int64_t lda, int dtype,
                           void *out, int64_t ldo, float *scales, hipStream_t s);
// out (m x n binary32, ldo) = the bfloat16 matrix in (ldi), exactly
hipError_t launch_bf16_to_f32(const void *in, int64_t m, int64_t n, int64_t ldi, float *out,
                              int64_t ldo, hipStream_t s);
// ---- launchers (k_sign.hip, k_mfma.hip): B = A Omega, random sign Omega ----
// threshold of sign_entry for a density in (0, 1] (round(d 2^31), >= 1)
uint32_t sign_threshold(double density);
// the sparse kernel (reads d r of A's columns per target column) or the MFMA one
bool sign_uses_sparse(int64_t r, double density);
hipError_t launch_project_sign(const AView &A, uint64_t seed, double density, int64_t r, float *B,
                               int64_t ldb, void *scratch, size_t scratch_bytes, hipStream_t s);
hipError_t launch_project_sign_dense(const AView &A, uint32_t k0, uint32_t k1, uint32_t thr,
                                     int64_t r, float *B, int64_t ldb, void *scratch,
                                     hipStream_t s);
hipError_t launch_proj_reduce(const float *P, int64_t ldp, int64_t m, int64_t r, int nsplit,
                              float *B, int64_t ldb, hipStream_t s);

// ---- launchers (k_embed.hip) ----
hipError_t launch_qless_r(const float *w, int64_t n, int64_t ldw, const int64_t *idx, int k,
                          float *r, int64_t ldr, hipStream_t s);
// Rank-k approximation from the embedding: byte offsets of its buffers in a
// scratch region, and the Gram matrix's tiling.
struct RankPlan {
  int L = 0, nt = 0, nsplit = 0;
  int64_t chunk = 0;
  size_t G = 0, U = 0, vb = 0, part = 0, mcoef = 0, perm = 0, sigma = 0, aux = 0, flag = 0, bytes = 0;
};
constexpr int kRankMaxL = 2048;  // largest number of picks the eigen-decomposition takes
RankPlan rank_plan(int lmax, int64_t n);
// G = W W^T (padded), U = I, and the sweeps' absolute threshold
hipError_t launch_wgram(const RankPlan &P, const float *w, int64_t ldw, int l, int64_t n,
                        char *scr, hipStream_t s);
// G = W V^T for a product known to be symmetric (upper tiles, mirrored)
hipError_t launch_wgram2(const RankPlan &P, const float *w, const float *v, int64_t ldw, int l,
                         int64_t n, char *scr, hipStream_t s);
// eigenvalue order of the diagonalised G (perm, sigma = sqrt(lambda), sums)
hipError_t launch_eig_order(const RankPlan &P, char *scr, int l, int k, hipStream_t s);
// out (m x l, column-major) = Y U Sigma^-1 from the eigenpairs of Y^T Y
hipError_t launch_orth_apply(const RankPlan &P, char *scr, int l, const float *y, int64_t ldy,
                             int64_t m, float *out, int64_t ldo, hipStream_t s);
// out (m x l, column-major) = Y R^-1 with R the Cholesky factor of Y^T Y
// (G prepared by launch_wgram; U is used as R's storage)
hipError_t launch_cholqr_apply(const RankPlan &P, char *scr, int l, const float *y, int64_t ldy,
                               int64_t m, float *out, int64_t ldo, hipStream_t s);
// ua = Q U[:, perm] (k columns, sign convention of rank_k)
hipError_t launch_ritz_vectors(const RankPlan &P, char *scr, int l, int k, const double *Q,
                               int64_t ldq, int64_t m, double *ua, int64_t ldu, hipStream_t s);
hipError_t launch_to_rowmajor(const float *in, int64_t ldi, int64_t m, int c, float *out,
                              hipStream_t s);
// b = u diag(sigma) in binary32 (sigma of the last eigenvalue order)
hipError_t launch_scale_cols(const RankPlan &P, char *scr, const double *u, int64_t ldu, int64_t m,
                             int k, float *b, int64_t ldb, hipStream_t s);
hipError_t launch_cols_to_f64(const float *in, int64_t ldi, int64_t m, int c, double *out,
                              int64_t ldo, hipStream_t s);
// one Jacobi sweep; the L / 64 ints at scr + P.flag are all 0 once G is diagonal
hipError_t launch_jacobi_sweep(const RankPlan &P, char *scr, hipStream_t s);
// eigenvalue order, sigma, error sums (scr + P.aux + 8: all, tail), then
// U_A (ua may be null) and V_A (va may be null)
hipError_t launch_rank_outputs(const RankPlan &P, char *scr, int l, int k, const double *Q,
                               int64_t ldq, int64_t m, double *ua, int64_t ldu, const float *w,
                               int64_t ldw, int64_t n, float *va, int64_t ldv, hipStream_t s);

// ---- batched (k_batched.hip) ----
// One group of consecutive columns inside one block of Algorithm 4.
struct GroupEnt {
  int64_t col0;
  int32_t ncol;
  int32_t blk;
};
// grid = resident workgroups per CU (at most wg_per_cu when > 0) x CUs, at
// most one per team of groups
hipError_t batched_stream_grid(const StreamGeo &geo, int dtype, int num_cu, int64_t ngroups,
                               int wg_per_cu, int *grid);
hipError_t launch_stream_batched(const StreamGeo &geo, int grid, const AView &A,
                                 const GroupEnt *groups, int64_t ngroups, const float *q32,
                                 const float *z32, int64_t qstride, double *f, double *g,
                                 const double *g0, const uint8_t *mask, ArgPart *gpart,
                                 const DevState *stb, uint32_t *bcnt, int score_only,
                                 hipStream_t s);
hipError_t launch_block_argmax(const AView &A, const ArgPart *gpart, const int64_t *gfirst,
                               int nprob, DevState *stb, double *ap64, int64_t apstride,
                               hipStream_t s);
// kb: device, the picks each problem wants (0: done from the start); kbm:
// entries of idx / obj per problem that are cleared
hipError_t launch_batch_begin(const double *f0, const double *g0, const uint8_t *mask0,
                              double *f, double *g, uint8_t *mask, int64_t n, DevState *stb,
                              int nprob, const int32_t *kb, int kbm, int64_t *idx, double *obj,
                              int64_t iostride, const double *F0, double tau, uint32_t *bcnt,
                              hipStream_t s);
// pick[b * kbm + j] = problem b's j-th pick, -1 past its last
hipError_t launch_pool(const DevState *stb, const int64_t *idx, int64_t iostride, int kbm,
                       int nprob, int64_t *pick, hipStream_t s);
// out[j] = pick[loc[j]] for j < km (-1 for a missing pick)
hipError_t launch_merge_map(const int64_t *loc, const int64_t *pick, int64_t npick, int km,
                            int64_t *out, hipStream_t s);
// out[b] = sum of x[off[b] .. off[b+1]) in a fixed order, b < nseg (off on the device)
hipError_t launch_seg_sum(const double *x, const int64_t *off, int nseg, double *out,
                          hipStream_t s);
hipError_t launch_gather_cols(const AView &A, const int64_t *pick, int64_t npick, void *a0,
                              float *scale0, hipStream_t s);

// ---- the merge selection of Algorithm 4 over a small pool (k_merge.hip) ----
struct MergeArgs {
  const void *a0;      // pooled columns (stored type, ld lda), P of them
  const float *sc0;    // their FP8 scales
  int64_t lda, m, P;
  const float *B;      // target, binary32, ld ldb, r columns
  int64_t ldb;
  int r;
  double *GH;          // row i: G_i. (P entries) then H_i. (r), ld ldgh
  int64_t ldgh;
  double *f, *g, *g0;  // P each
  uint8_t *excl;       // P: 1 picked, 2 dropped by the basis check
  double *W;           // k x P, row s = omega^(s)
  double *U;           // k x r, row s = upsilon^(s)
  ArgPart *part;       // one per step workgroup
  DevState *st;
  int64_t *loc;        // k picks (pool positions), -1 past the last
  double *obj;         // k + 1
  int32_t *ns;         // picks made
  const double *F0;    // ||B||_F^2
  double tau;
  int k;
};
size_t merge_gram_lds_bytes(int k, int r);
int merge_step_groups(int64_t P);
// G, H, the initial scores and the state (dtype: storage type of the pool)
hipError_t launch_merge_gram(const MergeArgs &a, int dtype, hipStream_t s);
// one step: the pick's update of every candidate and the next pick
hipError_t launch_merge_step(const MergeArgs &a, hipStream_t s);

// ---- context facts the autotuner keys its cache on (gcss_api.hip) ----
struct CtxInfo {
  hipStream_t stream;
  int64_t m, n;
  int dtype;
  int target;  // 0 none, 1 explicit B, 2 Gram (B = A)
};
bool ctx_describe(gcss_ctx *h, CtxInfo *out);
// Message gcss_last_error() returns on this thread.
void set_error(const char *msg);

// ---- HBM read probe (k_probe.hip) ----
constexpr int kProbeSinkFloats = 4096;  // largest grid, one sink entry per workgroup
int hbm_probe_grid(int64_t bytes, int num_cu);
hipError_t launch_hbm_probe(const void *buf, int64_t bytes, float *sink, int grid, hipStream_t s);

}  // namespace gcss
