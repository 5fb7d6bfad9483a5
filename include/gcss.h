/*
 * gcss.h -- C ABI of the MI355X (gfx950) library for greedy generalized
 * column subset selection (Farahat, Elgohary, Ghodsi, Kamel, "Greedy Column
 * Subset Selection for Large-scale Data Sets").
 *
 * Problem (Problems 1 and 5 of the paper): given a source matrix A (m x n)
 * and a target B (m x r), pick k columns S of A that greedily minimise
 *      F(S) = || B - P_S B ||_F^2 ,   P_S = projection onto span(A_S).
 * B = A is the centralized problem (Algorithm 1); B = A * Omega with a random
 * Omega is the paper's concise target (Section 5.1, Algorithm 2).
 *
 * Conventions
 *   - Matrices are column-major.  A's column i starts at element i*lda.
 *     lda >= m, and lda * sizeof(element) must be a multiple of 16 bytes;
 *     device pointers must be 16-byte aligned.  Pad entries are never read
 *     into results.
 *   - Pointers documented as "device" are HIP device memory owned by the
 *     caller; they must stay valid for the life of the context that borrows
 *     them.  Pointers documented as "host" are ordinary host memory.
 *   - Indices are 0-based (the paper's are 1-based).
 *   - Every call returns a gcss_status.  Nothing aborts or throws across the
 *     ABI.  On failure gcss_last_error() returns a message (per thread) and
 *     the context keeps its previous state.
 *   - All device work of a context is ordered on the stream given at
 *     creation (NULL = the device's default stream).  Calls that return host
 *     outputs synchronize that stream; the *_async calls do not.
 *   - The library allocates no device memory: the caller hands over one
 *     workspace sized by gcss_workspace_size().
 *   - Same inputs, same device -> bitwise identical outputs (no floating
 *     point atomics; every reduction has a fixed order).
 */
#ifndef GCSS_H
#define GCSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GCSS_OK = 0,
  GCSS_WARN_EXHAUSTED = 1,   /* fewer than k eligible columns; *n_selected < k   */
  GCSS_ERR_ARG = -1,         /* invalid argument (null pointer, size, alignment) */
  GCSS_ERR_STATE = -2,       /* call out of order (e.g. select before a target)  */
  GCSS_ERR_DEVICE = -3,      /* no usable gfx950 device, or a HIP runtime error  */
  GCSS_ERR_WORKSPACE = -4,   /* workspace missing or smaller than required       */
  GCSS_ERR_UNSUPPORTED = -5  /* shape or dtype outside what the kernels cover    */
} gcss_status;

/* Element type of the stored source matrix A. */
typedef enum {
  GCSS_F32 = 0,       /* IEEE binary32                                              */
  GCSS_BF16 = 1,      /* bfloat16 (upper half of binary32)                          */
  GCSS_FP8_E4M3 = 2   /* OCP FP8 E4M3 (e4m3fn); value = a_scale[i] * decode(code)   */
} gcss_dtype;

typedef struct gcss_ctx gcss_ctx;

/* Description of the source matrix and of the capacity a context reserves. */
typedef struct {
  int64_t m;               /* rows of A (and of B)                              >= 1 */
  int64_t n;               /* columns of A                                      >= 1 */
  int64_t lda;             /* leading dimension of A, in elements               >= m */
  int32_t a_dtype;         /* gcss_dtype                                             */
  const void *a;           /* device, borrowed: A, column-major                      */
  const float *a_scale;    /* device, borrowed: n per-column scales (FP8 only; NULL otherwise) */
  int32_t k_max;           /* largest k any later select may ask for        1..n     */
  int64_t r_max;           /* largest explicit target width (0 = none)               */
  int32_t self_target;     /* nonzero: reserve the m x m Gram target for B = A       */
  int32_t reserved;        /* must be 0                                              */
  double tau;              /* eligibility threshold: a column stays a candidate while
                              g_i > tau * g0_i (g = squared norm of its residual);
                              <= 0 selects 1e-4                                      */
  void *stream;            /* hipStream_t for all work of the context; NULL = default */
} gcss_desc;

/*
 * Bytes of device workspace a context for *d needs.  Host-only; does not
 * touch the device.  Errors: GCSS_ERR_ARG.
 */
gcss_status gcss_workspace_size(const gcss_desc *d, size_t *bytes);

/*
 * Create a context over the source matrix described by *d, on the current
 * HIP device.  workspace: device, >= gcss_workspace_size bytes, 256-byte
 * aligned, borrowed for the context's life.
 * Errors: GCSS_ERR_ARG, GCSS_ERR_WORKSPACE, GCSS_ERR_DEVICE (no gfx950),
 * GCSS_ERR_UNSUPPORTED (m > 8192, the most rows the streaming kernel keeps
 * in registers).
 */
gcss_status gcss_create(const gcss_desc *d, void *workspace, size_t ws_bytes, gcss_ctx **out);

/* Destroy a context (NULL is ignored).  Does not free borrowed memory. */
void gcss_destroy(gcss_ctx *h);

/*
 * Set the target and compute the initial scores of Algorithms 1/3:
 *     f_i = || B^T A_i ||^2 ,  g_i = || A_i ||^2 ,  F_0 = || B ||_F^2 .
 * b: device, borrowed, m x r column-major with leading dimension ldb >= m
 *    (ldb * element size a multiple of 16 bytes), 1 <= r <= r_max.
 * b_dtype: GCSS_F32 (binary32) or GCSS_BF16 (bfloat16).  A bfloat16 target
 *    is the matrix of its bfloat16 values: they are copied exactly into a
 *    binary32 copy in the workspace, which every kernel then reads.
 * b == NULL and r == 0: B = A (Algorithm 1; b_dtype is ignored).  The
 *    target then enters only through its Gram matrix A A^T (m x m), which is
 *    formed in the workspace; requires self_target at creation.
 * Errors: GCSS_ERR_ARG (also an unknown b_dtype), GCSS_ERR_STATE (self
 * target not reserved), GCSS_ERR_DEVICE.
 */
gcss_status gcss_set_target(gcss_ctx *h, const void *b, int32_t b_dtype, int64_t r, int64_t ldb);

/*
 * The paper's concise target (Section 5.1, Algorithm 2): B = A * Omega,
 * written to b_out, then set as the target as by gcss_set_target.
 * omega: device, n x r binary32 ROW-major (row i is the r-vector drawn for
 *        column i of A), borrowed only during the call.
 * b_out: device, m x r column-major, leading dimension ldb >= m (ldb *
 *        element size a multiple of 16 bytes), 16-byte aligned; borrowed for
 *        the context's life (it becomes the target).
 * b_dtype: GCSS_F32 stores the binary32 product; GCSS_BF16 rounds each
 *        binary32 entry once to the nearest bfloat16 (ties to even), and
 *        those values are the target.  Rows m..ldb-1 of a bfloat16 b_out are
 *        set to zero.
 * Errors: as gcss_set_target.
 */
gcss_status gcss_project_target(gcss_ctx *h, const float *omega, int64_t r, void *b_out,
                                int32_t b_dtype, int64_t ldb);

/*
 * Concise target from a random sign matrix drawn on the fly (Section 5.1:
 * Omega's entries are i.i.d. from a univariate distribution, one row per
 * column of A, never stored; the paper names uniform random sign and sparse
 * random sign matrices).  B = A Omega (m x r), then B becomes the target as
 * with gcss_set_target(h, b_out, r, ldb).
 * Omega_ij (i < n, j < r) for seed and density d in (0, 1]: let w be word
 * (j mod 4) of Philox4x32-10 (Salmon et al., SC 2011) applied to the counter
 * (i mod 2^32, i div 2^32, j div 4, 0) with the key (seed mod 2^32,
 * seed div 2^32), and t = round(d 2^31) (at least 1); then Omega_ij = 0 if
 * (w >> 1) >= t, else -1 if w is odd and +1 if it is even.  d = 1 is the
 * dense +-1 matrix; d = 1/sqrt(n) the sparse one of the paper.
 * When d r <= 4 a pass reads only the columns of A with a non-zero entry in
 * each column of Omega; otherwise the matrix-core projection runs with the
 * Omega tiles generated in the kernel.  Sums are binary32 in a fixed order.
 * b_out: device, ldb >= m, multiple of 4, 16-byte aligned, kept by the
 * context.  Errors: GCSS_ERR_ARG (r outside [1, r_max], d outside (0, 1],
 * ldb, alignment), GCSS_ERR_DEVICE.
 */
gcss_status gcss_project_sign(gcss_ctx *h, uint64_t seed, double density, int64_t r,
                              float *b_out, int64_t ldb);

/*
 * Greedy selection of k columns (Algorithm 3; Algorithm 1 for B = A) from the
 * initial scores of the current target.  Each call starts from those
 * scores, so repeated calls give identical results.
 * idx:        host, k entries: picks in order; -1 for picks not made.
 * objective:  host, k+1 entries (may be NULL): objective[0] = ||B||_F^2,
 *             objective[t] = F(first t picks) = objective[t-1] minus the
 *             decrease of Theorems 1 and 3, ||B^T q_t||^2 for the pick's unit
 *             residual direction q_t (FP64; for B = A it is recomputed after
 *             the loop as ||A^T q_t||^2 with FP64 products and sums);
 *             entries past *n_selected repeat the last value.
 * n_selected: host (may be NULL): number of picks made.
 * Returns GCSS_OK, or GCSS_WARN_EXHAUSTED when fewer than k columns stay
 * candidates (see gcss_desc.tau).  A column stops being a candidate when its
 * tracked residual g_i drops to tau * g0_i or below, when a pick of it is
 * rejected because its exact FP64 residual after re-orthogonalisation is at
 * most tau * g0_i, or when f_i or g_i is not finite (a column holding NaN or
 * infinity is never picked; no error is raised).  Errors: GCSS_ERR_ARG
 * (k < 1 or k > k_max), GCSS_ERR_STATE (no target), GCSS_ERR_DEVICE.
 * Synchronizes the stream.
 */
gcss_status gcss_select(gcss_ctx *h, int32_t k, int64_t *idx, double *objective,
                        int32_t *n_selected);

/*
 * As gcss_select, but the outputs stay on the device and the call does not
 * synchronize: d_idx (k int64), d_obj (k+1 double, may be NULL),
 * d_nsel (1 int32, may be NULL) are device pointers written on the stream.
 * The whole k-step loop is replayed from a HIP graph that is built on the
 * first call for a given k.  The graph holds k + GCSS_ASYNC_SPARE_STEPS
 * steps; a step whose pick the basis check rejects (a column that only
 * rounding kept a candidate: its exact FP64 residual is at most tau times
 * its squared norm) adds no pick, so after more rejections than that the
 * graph ends with *d_nsel < k although candidates remain.  gcss_read_state
 * (GCSS_STATE_FLAGS) then reports finished = 0; gcss_select, which loops
 * on the host, always finishes.
 */
#define GCSS_ASYNC_SPARE_STEPS 8
gcss_status gcss_select_async(gcss_ctx *h, int32_t k, int64_t *d_idx, double *d_obj,
                              int32_t *d_nsel);

/*
 * Reconstruction error || B - P_S B ||_F^2 of the current target for the
 * columns S = idx[0..k-1] (host, distinct, in [0, n)), written to *err
 * (host).  P_S comes from an FP64 Gram-Schmidt basis Q (with one
 * re-orthogonalisation) of A_S; a column numerically dependent on the
 * earlier ones adds no direction.  For an explicit B the residual
 * B - Q (Q^T B) is formed and summed in FP64.  For B = A the error is
 * ||A||_F^2 - sum_s ||A^T q_s||^2 with FP64 products and sums.
 * Errors: GCSS_ERR_ARG, GCSS_ERR_STATE, GCSS_ERR_DEVICE.
 */
gcss_status gcss_reconstruction_error(gcss_ctx *h, const int64_t *idx, int32_t k, double *err);

/*
 * Low-dimensional embedding of every column in the span of the picks
 * (Section 3, Eq. CSS_LowDim): W = Q^T A, with Q the orthonormal basis of
 * A_S in pick order.  Row t of W is omega = A^T q_{t+1}, the vector each
 * step's streaming pass already forms, so the embedding costs one extra
 * coalesced store of n floats per step (and, after the last pick, one more
 * pass over A for the last row).
 * w: device float, row-major k_max x ldw (row t starts at element t*ldw),
 * ldw >= n; owned by the caller, borrowed by the context until it is
 * replaced or turned off (w = NULL).  gcss_select and gcss_select_async
 * write rows 0 .. n_selected-1 (binary32; FP8 columns include their
 * scale); other rows are left as they were.  Batched selection does not
 * write it.  Changing the pointer rebuilds gcss_select_async's graph.
 * Errors: GCSS_ERR_ARG (ldw < n, misaligned w).
 */
gcss_status gcss_set_embedding(gcss_ctx *h, float *w, int64_t ldw);

/*
 * Q-less QR factor of the picks (Section 6): with Pi sorting the picked
 * columns first, A Pi = Q W Pi, and the first k columns of W Pi form the
 * upper triangular R (k x k) with A_S = Q R.
 * w: device, row-major embedding as written by a selection (ldw >= n);
 * idx: device, k int64 picks in pick order; r: device float, row-major
 * k x ldr (ldr >= k).  R[s][j] = W[s][idx[j]] for s <= j and 0 below the
 * diagonal (the entries W keeps there are rounding residue).  A column whose
 * idx entry is outside [0, n) is written as NaN.  Ordered on stream
 * (NULL = default stream).  Errors: GCSS_ERR_ARG, GCSS_ERR_DEVICE.
 */
gcss_status gcss_qless_r(const float *w, int64_t n, int64_t ldw, const int64_t *idx, int32_t k,
                         float *r, int64_t ldr, void *stream);

/*
 * Leading eigenpairs of C = A A^T (the squared singular values and left
 * singular vectors of A) by block subspace iteration with Rayleigh-Ritz,
 * for the quality metric of Section 7 (the best rank-l error
 * ||A||_F^2 - sum_{j<=l} lambda_j) and for the target B = U_k Sigma_k of the
 * paper's DistApproxSVD baseline.  Needs the Gram matrix (self target set).
 * Method: Y = C Omega (Omega an m x s dense random sign matrix from seed,
 * drawn in the kernel); then per iteration Q = orth(Y) (Cholesky QR in
 * FP64: Y <- Y R^-1 with R^T R = Y^T Y; twice before each check) and
 * Y = C Q (matrix cores, binary32); every 4 iterations and at the last, the
 * Ritz values of T = Q^T C Q (FP64 block Jacobi); it stops when the sum of
 * the k leading
 * Ritz values changed by at most tol (relative) since the previous check,
 * or after max_iters iterations.  Accuracy is limited by the binary32 C
 * (relative ~1e-7 of lambda_1) and by the convergence of the block
 * (clustered spectra converge slowly; the returned change says how far).
 * 1 <= k <= s <= min(k_max, m, 2048).  lambda: host, k doubles, descending.
 * u: device double, column-major m x k (ldu >= m), or NULL: Q times the
 * Ritz vectors, sign convention of gcss_rank_k; computing u overwrites the
 * selection basis, so gcss_rank_k needs a new selection afterwards.
 * b_out (device float, column-major m x k, ldb >= m, multiple of 4, or
 * NULL; needs u): the DistApproxSVD target U_k Sigma_k in binary32, ready
 * for gcss_set_target.
 * iters, change (host, may be NULL): iterations run, last relative change.
 * Uses the workspace's scratch; synchronizes.  Errors: GCSS_ERR_ARG,
 * GCSS_ERR_STATE (no Gram target), GCSS_ERR_UNSUPPORTED, GCSS_ERR_DEVICE.
 */
gcss_status gcss_top_eig(gcss_ctx *h, int32_t s, int32_t max_iters, double tol, uint64_t seed,
                         int32_t k, double *lambda, double *u, int64_t ldu, float *b_out,
                         int64_t ldb, int32_t *iters, double *change);

/*
 * Rank-k approximation of A inside the span of the first l picks (Section 3,
 * the procedure credited to Boutsidis et al.), and the approximate leading
 * singular triplets of A it gives (Eq. ApproxSVD):
 *   W = U_W Sigma V_W^T (SVD of the l x n embedding), A_{S,k} = Q W_k,
 *   u = Q U_W[:, :k]  (m x k),  sigma = Sigma[:k],  v = V_W[:, :k]  (n x k),
 * so that A_{S,k} = u diag(sigma) v^T is the best rank-k approximation of A
 * whose columns lie in span(A_S).
 * Uses the basis Q of the last gcss_select / gcss_select_async on this
 * context (under the current target) and its embedding w (as written with
 * gcss_set_embedding; device, row-major, ldw >= n, rows 0..l-1 read).
 * 1 <= k <= l <= min(picks of that selection, 2048).
 * Method: G = W W^T with FP64 sums of the binary32 products, eigenvalues and
 * vectors of G by block Jacobi in FP64 (sigma_j = sqrt(lambda_j)), then
 * u = Q U_k (FP64) and v = W^T U_k Sigma_k^-1 (binary32; a zero sigma_j
 * gives a zero column).  Sign: the largest-magnitude entry of each column of
 * u (the first on ties) is positive; v's column carries the same sign.
 * u: device double, column-major m x k, ldu >= m, or NULL; v: device float,
 * column-major n x k, ldv >= n, or NULL; sigma: host, k doubles (descending);
 * err (host, may be NULL): ||A - A_{S,k}||_F^2 = ||A - Q W||_F^2 + sum of
 * the l - k smallest lambda, with ||A - Q W||_F^2 the selection's objective
 * F(S) when B = A, else ||A||_F^2 - ||W||_F^2 (which loses the digits of
 * ||A||_F^2 that the binary32 W cannot hold).  Uses the workspace's
 * scratch; synchronizes the stream.
 * Errors: GCSS_ERR_ARG, GCSS_ERR_STATE (no selection basis),
 * GCSS_ERR_UNSUPPORTED (l > 2048), GCSS_ERR_DEVICE.
 */
gcss_status gcss_rank_k(gcss_ctx *h, const float *w, int64_t ldw, int32_t l, int32_t k, double *u,
                        int64_t ldu, float *v, int64_t ldv, double *sigma, double *err);

/*
 * Algorithm 4 on one GPU.  The columns of A are split into nblocks
 * consecutive blocks col_off[b] .. col_off[b+1]-1 (host, nblocks+1 entries,
 * col_off[0] = 0, col_off[nblocks] = n, strictly increasing).  Every block
 * selects k_block columns against the shared explicit target B (all blocks
 * advance together, one batched launch per phase of a step); the picks are
 * pooled in block order, then pick order, and k_merge columns are selected
 * from the pool against B.  Both phases run on the device as one captured
 * graph (replayed while the block layout and budgets stay the same); the
 * host only reads the results back, plus extra steps for a block or merge
 * whose basis check rejected more picks than the graph's spare steps.
 * idx_block: host, nblocks*k_block global indices (-1 for picks not made).
 * idx_merge: host, k_merge global indices.  obj_merge: host, k_merge+1 (may
 * be NULL).  n_merge: host (may be NULL).
 * Requires an explicit target (gcss_set_target / gcss_project_target) and
 * k_block*nblocks <= n.  Errors: GCSS_ERR_ARG, GCSS_ERR_STATE,
 * GCSS_ERR_UNSUPPORTED (pool larger than the context's k_max allows),
 * GCSS_ERR_DEVICE.  Synchronizes the stream.
 */
gcss_status gcss_select_batched(gcss_ctx *h, int32_t nblocks, const int64_t *col_off,
                                int32_t k_block, int32_t k_merge, int64_t *idx_block,
                                int64_t *idx_merge, double *obj_merge, int32_t *n_merge);

/* Rules for the per-block budgets l_(b) of Algorithm 4 (Section 5.2, the
 * paragraph after Algorithm 4, and the naive distributed selection). */
typedef enum {
  GCSS_BUDGET_UNIFORM = 0, /* floor(l / c) for each of the c blocks (the paper's)  */
  GCSS_BUDGET_EVEN = 1,    /* l / c, rounded by largest remainders                 */
  GCSS_BUDGET_NORM = 2     /* l ||A_(b)||_F^2 / ||A||_F^2, by largest remainders    */
} gcss_budget_policy;

/*
 * Per-block budgets for Algorithm 4 (Section 5.2, after Algorithm 4).
 * col_off: host, nblocks+1 entries as for gcss_select_batched.  l: the
 * total number of picks wanted (l >= 0).  Every budget is at most its
 * block's width.  UNIFORM: floor(l / c), the remainder unused.  EVEN and
 * NORM: the shares (l / c, or l ||A_(b)||^2 / ||A||^2, l / c for a zero A)
 * are rounded down and capped at the widths, then the columns missing to
 * min(l, n) go one at a time to the block with the largest share minus
 * budget among those with room, the lower block first on equal
 * remainders.  norms2: host, nblocks squared Frobenius norms of the blocks,
 * or NULL to take them from the context (the FP64 column norms of the
 * stored A, summed per block in a fixed order; needs a target, and h may
 * then not be NULL; synchronizes the context's stream).  h may be NULL when
 * norms2 is given or the policy is not NORM.  k_blocks: host, nblocks
 * outputs.  Errors: GCSS_ERR_ARG (policy, col_off, a negative or non-finite
 * norm), GCSS_ERR_STATE (norms from a context without a target),
 * GCSS_ERR_UNSUPPORTED (more blocks than the context's scratch holds),
 * GCSS_ERR_DEVICE.
 */
gcss_status gcss_block_budgets(gcss_ctx *h, int32_t nblocks, const int64_t *col_off,
                               const double *norms2, int32_t l, int32_t policy,
                               int32_t *k_blocks);

/*
 * Algorithm 4 with a budget per block: as gcss_select_batched, with block b
 * selecting k_blocks[b] columns (host, nblocks entries, 0 <= k_blocks[b] <=
 * the block's width, at least one positive).  The pool holds
 * nblocks * kmax slots, kmax the largest budget; idx_block is laid out the
 * same way (host, nblocks * kmax, block b's picks at b * kmax, -1 past its
 * last).  The pool is pooled in block order, then pick order, as in
 * gcss_select_batched; empty slots are zero columns, never picked.
 * Requires k_merge <= nblocks * kmax and a workspace sized by
 * gcss_batched_workspace_size with k_block = kmax.  Errors as for
 * gcss_select_batched.  Synchronizes the stream.
 */
gcss_status gcss_select_batched_budgets(gcss_ctx *h, int32_t nblocks, const int64_t *col_off,
                                        const int32_t *k_blocks, int32_t k_merge,
                                        int64_t *idx_block, int64_t *idx_merge, double *obj_merge,
                                        int32_t *n_merge);

/*
 * Bytes of workspace gcss_select_batched needs beyond gcss_workspace_size,
 * for the given block layout and budgets (k_block: the largest budget);
 * pass the total to gcss_create (the batched state is carved from the end
 * of the same workspace).
 */
gcss_status gcss_batched_workspace_size(const gcss_desc *d, int32_t nblocks, int32_t k_block,
                                        int32_t k_merge, size_t *bytes);

/*
 * Store a binary32 matrix in a reduced-precision format (the storage the
 * selection then streams).  a: device m x n, leading dimension lda.
 * out: device, leading dimension ldo (elements) >= m.  dtype GCSS_BF16:
 * round to nearest, ties to even.  dtype GCSS_FP8_E4M3: per column
 * scale_i = max_j |a_ji| / 448 (binary32 division; 1 for a zero column),
 * written to scales (device, n floats), and code = nearest E4M3 value of the
 * binary32 quotient a_ji / scale_i, ties to even, saturating at 448.
 * Pad entries m..ldo-1 of each column are set to zero.  Ordered on stream.
 * Errors: GCSS_ERR_ARG, GCSS_ERR_DEVICE.
 */
gcss_status gcss_quantize(const float *a, int64_t m, int64_t n, int64_t lda, int32_t dtype,
                          void *out, int64_t ldo, float *scales, void *stream);

/*
 * Copy columns of the context's A: column j of out = stored column idx[j]
 * (all lda elements, same storage type; FP8 also copies the scale into
 * out_scales[j]).  For the second selection of Algorithm 4 and of the
 * naive distributed selection (Section 5: a selection over the pooled
 * columns A_{:L}).  idx: device, count int64; an index outside [0, n)
 * gives a zero column (scale 1).  out: device, count * lda elements,
 * 16-byte aligned.  Ordered on the context's stream.
 * Errors: GCSS_ERR_ARG, GCSS_ERR_DEVICE.
 */
gcss_status gcss_gather_columns(gcss_ctx *h, const int64_t *idx, int64_t count, void *out,
                                float *out_scales);

/* What gcss_read_state copies back (for tests and diagnostics). */
typedef enum {
  GCSS_STATE_F0 = 0,    /* n doubles: initial f                                 */
  GCSS_STATE_G0 = 1,    /* n doubles: initial g                                 */
  GCSS_STATE_F = 2,     /* n doubles: f after the last select                   */
  GCSS_STATE_G = 3,     /* n doubles: g after the last select                   */
  GCSS_STATE_Q = 4,     /* m*t doubles: orthonormal basis of the picks (col-major, ld m) */
  GCSS_STATE_Z = 5,     /* m floats: z of the last completed step               */
  GCSS_STATE_B = 6,     /* m*r floats: the explicit target's values (col-major, ld m) */
  GCSS_STATE_GRAM = 7,  /* m*m floats: the Gram target A A^T (self target)      */
  GCSS_STATE_NREJECT = 8, /* 1 int32: picks rejected by the basis check          */
  GCSS_STATE_FLAGS = 9    /* 4 int32 of the last select / select_async: picks made,
                             finished (1: k picks or no candidate left; 0: a
                             select_async graph ran out of steps, see there),
                             exhausted (1: ran out of candidates), rejected picks */
} gcss_state_item;

/*
 * Copy an internal array of the context to host memory (synchronizes).
 * host: host buffer of `bytes` bytes; the copy is truncated to the item's
 * size, and *copied (may be NULL) receives the bytes written.
 */
gcss_status gcss_read_state(gcss_ctx *h, int32_t item, void *host, size_t bytes, size_t *copied);

/* Timings collected while profiling is on (HIP events on the context's
 * stream around every fused streaming pass), recorded by gcss_select and by
 * gcss_select_batched, which then enqueues its per-block loop directly
 * instead of replaying its graph; the graph-replayed gcss_select_async is not
 * instrumented. */
typedef struct {
  int64_t stream_launches;  /* fused streaming passes (step 4 of the loop) timed  */
  double stream_ms;         /* their summed duration, milliseconds.  Passes that
                               read no column are not counted: the pass after
                               the last pick (explicit target, no embedding;
                               the last block step of a batched call) is not
                               timed, and a pass under a quarter of the call's
                               longest (a rescore after a rejected pick) is
                               left out                                         */
  int64_t selects;          /* gcss_select calls timed                            */
  double loop_ms;           /* summed duration of their k-step loops, ms          */
} gcss_profile;

/* Turn event timing of gcss_select on (enable != 0) or off; always clears
 * the counters.  Errors: GCSS_ERR_ARG, GCSS_ERR_DEVICE. */
gcss_status gcss_set_profiling(gcss_ctx *h, int32_t enable);

/* Read the counters (host struct).  Errors: GCSS_ERR_ARG. */
gcss_status gcss_get_profile(gcss_ctx *h, gcss_profile *out);

/*
 * Launch settings of the streaming passes (the step that reads all of A once
 * per pick).  They set how the work is spread over the chip, never what is
 * computed: indices, scores and explicit-target objectives are bitwise the
 * same under every setting.  Under the Gram target (B = A) the objective's
 * decrements are FP64 sums of per-workgroup partials, whose grouping follows
 * the setting, so they can differ in the last bits.
 */
typedef struct {
  int32_t stream_pd;        /* column groups loaded ahead of the one being reduced: 1 or 2 (default 1) */
  int32_t stream_upw;       /* work units per workgroup that the unit size aims at: 1..64 (default 4) */
  int32_t batch_group;      /* columns per group of the batched pass: 16, 32 or 64 (default 64)     */
  int32_t batch_wg_per_cu;  /* resident workgroups per CU of the batched pass; 0 = all that fit     */
} gcss_tuning;

/* Current setting of a context (host struct).  Errors: GCSS_ERR_ARG. */
gcss_status gcss_get_tuning(gcss_ctx *h, gcss_tuning *out);

/* Apply a setting (host struct).  Synchronizes the stream and drops the
 * captured loops, which the next select_async / select_batched captures
 * again.  Errors: GCSS_ERR_ARG (a field out of range), GCSS_ERR_DEVICE. */
gcss_status gcss_set_tuning(gcss_ctx *h, const gcss_tuning *t);

/* Outcome of an autotuning call (host struct). */
typedef struct {
  gcss_tuning best;     /* the setting chosen, left applied to the context             */
  double best_ms;       /* its median time per timed call, milliseconds                */
  double initial_ms;    /* the same for the setting the context had on entry (0 when
                           the setting came from the cache)                             */
  int32_t candidates;   /* settings timed; 0 when the setting came from the cache       */
} gcss_tune_result;

/*
 * Autotuner for gcss_select: times gcss_select(h, k) under each candidate
 * setting (stream_pd in {1, 2} x stream_upw in {2, 4, 8, 16}, and the entry
 * setting), one untimed call then `reps` calls each bracketed by HIP events
 * on the context's stream, and applies the setting with the lowest median.
 * cache_path (host string, may be NULL): a JSON file of settings keyed by
 * device architecture, m, ceil(log2 n), storage type and target kind; a
 * cached setting is applied without timing, and a new result is added to the
 * file (written to a temporary file, then renamed over it).  Needs a target
 * (GCSS_ERR_STATE otherwise).  Leaves the context as after gcss_select(h, k).
 * Errors: GCSS_ERR_ARG (k, reps, an unreadable or malformed cache file, which
 * is left as it is; a cache file that cannot be written, in which case the
 * chosen setting is still applied), GCSS_ERR_STATE, GCSS_ERR_DEVICE (the
 * entry setting is restored).  Synchronizes the stream.  Not thread-safe
 * for one context, like every call on it; two processes that write the same
 * cache file at once keep one of their results.
 */
gcss_status gcss_autotune_select(gcss_ctx *h, int32_t k, int32_t reps, const char *cache_path,
                                 gcss_tune_result *out);

/*
 * Autotuner for gcss_select_batched (the one captured launch of Algorithm 4's
 * per-block selections): times that call with the given blocks and budgets
 * under batch_group in {16, 32, 64} x batch_wg_per_cu in {0, 2, 4} (and the
 * entry setting), as gcss_autotune_select does; the cache key adds the block
 * count.  Same arguments and errors as gcss_select_batched plus those of
 * gcss_autotune_select.
 */
gcss_status gcss_autotune_batched(gcss_ctx *h, int32_t nblocks, const int64_t *col_off,
                                  int32_t k_block, int32_t k_merge, int32_t reps,
                                  const char *cache_path, gcss_tune_result *out);

/*
 * Achievable HBM read bandwidth: times `reps` read-only passes over buf
 * (device, 16-byte aligned, bytes a positive multiple of 16; borrowed) with
 * the streaming pass's access pattern, after one untimed pass, between HIP
 * events on `stream` (hipStream_t, NULL = default), and returns the mean time
 * of one pass in *seconds (host).  bytes / *seconds is the practical ceiling
 * of a pass that reads each byte once.  sink: device, GCSS_PROBE_SINK_FLOATS
 * floats; the call zeroes it, then workgroup b stores the XOR of the 32-bit
 * words it read as the bit pattern of sink[b], so the XOR of all entries is
 * the XOR of every word of buf.  Errors: GCSS_ERR_ARG, GCSS_ERR_DEVICE.
 * Synchronizes the stream.
 */
#define GCSS_PROBE_SINK_FLOATS 4096
gcss_status gcss_hbm_probe(const void *buf, size_t bytes, float *sink, int32_t reps, void *stream,
                           double *seconds);

/*
 * Selection that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  One call does what gcss_create + gcss_set_target(b, r,
 * ldb) + gcss_select_async(k) do, with the workspace taken from a static
 * device array of GCSS_STATIC_SCRATCH_BYTES bytes that the library's code
 * object holds on every device it is loaded on until the process ends.
 * d: as for gcss_create (d->stream orders all work; host struct read during
 * the call only).  b, b_dtype, r, ldb: as for gcss_set_target (b == NULL,
 * r == 0: B = A, needs d->self_target).  d_idx (k int64), d_obj (k+1 double, may be NULL),
 * d_nsel (1 int32, may be NULL): device outputs as for gcss_select_async,
 * written on the stream; the call does not synchronize.  Picks and objective
 * are bitwise those of the context path with the default launch setting.
 * The array keeps the last call's contents; every call initialises what it
 * reads.  Calls that overlap on one device (other threads, or other streams
 * before the previous call's work has finished) share the array and race:
 * order them on one stream or wait for the previous one.
 * Errors: GCSS_ERR_ARG, GCSS_ERR_STATE (B = A without self_target),
 * GCSS_ERR_UNSUPPORTED (gcss_workspace_size(d) above the array's size; the
 * message gives both), GCSS_ERR_DEVICE.
 */
#define GCSS_STATIC_SCRATCH_BYTES (64u << 20)
gcss_status gcss_select_static(const gcss_desc *d, const void *b, int32_t b_dtype, int64_t r,
                               int64_t ldb, int32_t k, int64_t *d_idx, double *d_obj,
                               int32_t *d_nsel);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *gcss_last_error(void);

/* Library version string. */
const char *gcss_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GCSS_H */
