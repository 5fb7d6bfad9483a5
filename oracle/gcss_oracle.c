/*
 * gcss_oracle.c -- plain FP64 CPU oracle for greedy column subset selection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Farahat, Elgohary, Ghodsi, Kamel, "Greedy Column Subset
 * Selection for Large-scale Data Sets"):
 *
 *   orc_select            Algorithm 3 (greedy generalized CSS) in its
 *                         recursive form: the residual Gram and cross columns
 *                         of the pick, the history omega / upsilon and the
 *                         score update of Theorem 4.  With B == NULL it is
 *                         Algorithm 1 (B = A) with the update of Theorem 2.
 *   orc_error             the CSS objective ||B - P_S B||_F^2 of Problem 1 /
 *                         Problem 5, with P_S from a Householder QR of A_S
 *                         (the projection of Section 3.1 written without the
 *                         explicit inverse).
 *   orc_select_distributed  Algorithm 4: Algorithm 3 on every column block,
 *                         then Algorithm 3 on the pooled picks.
 *   orc_*bf16*, orc_*fp8* storage formats: bfloat16 and OCP FP8 E4M3 (e4m3fn)
 *                         written from their bit-level definitions; the
 *                         paper fixes no precision, these only define what a
 *                         reduced-precision copy of A holds.
 *
 * Everything is double precision.  Loops over columns run under OpenMP;
 * every reduction is done in a fixed order so results do not depend on the
 * thread count.
 *
 * Indices are 0-based (the paper's are 1-based).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EXHAUSTED 1
#define ORC_ERR_ARG (-1)
#define ORC_ERR_NOMEM (-2)

/* fixed column-chunk width for order-independent reductions over columns */
#define ORC_CHUNK 512

static double dotd(const double *x, const double *y, int64_t m) {
  double s = 0.0;
  for (int64_t j = 0; j < m; ++j) s += x[j] * y[j];
  return s;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* y = A w  (m-vector) summed over columns in fixed chunks, fixed order. */
static int matvec_cols(const double *A, int64_t m, int64_t n, int64_t lda,
                       const double *w, double *y) {
  int64_t nch = (n + ORC_CHUNK - 1) / ORC_CHUNK;
  double *part = (double *)calloc((size_t)(nch * m), sizeof(double));
  if (!part) return ORC_ERR_NOMEM;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    double *p = part + c * m;
    int64_t i1 = (c + 1) * ORC_CHUNK < n ? (c + 1) * ORC_CHUNK : n;
    for (int64_t i = c * ORC_CHUNK; i < i1; ++i) {
      const double *a = A + i * lda;
      double wi = w[i];
      if (wi == 0.0) continue;
      for (int64_t j = 0; j < m; ++j) p[j] += wi * a[j];
    }
  }
  for (int64_t j = 0; j < m; ++j) y[j] = 0.0;
  for (int64_t c = 0; c < nch; ++c)
    for (int64_t j = 0; j < m; ++j) y[j] += part[c * m + j];
  free(part);
  return ORC_OK;
}

/*
 * Initial scores of Algorithm 3 (and Algorithm 1):
 *   f_i = ||B^T A_i||^2,  g_i = A_i^T A_i.
 * With B == NULL (B = A): f_i = ||A^T A_i||^2, computed from its definition
 * (the n-vector A^T A_i, then its squared norm).
 */
int orc_init_scores(const double *A, int64_t m, int64_t n, int64_t lda,
                    const double *B, int64_t r, int64_t ldb, double *f, double *g) {
  if (!A || m < 1 || n < 1 || lda < m || !f || !g) return ORC_ERR_ARG;
  if (B && (r < 1 || ldb < m)) return ORC_ERR_ARG;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    const double *ai = A + i * lda;
    g[i] = dotd(ai, ai, m);
    double s = 0.0;
    if (B) {
      for (int64_t c = 0; c < r; ++c) {
        double h = dotd(B + c * ldb, ai, m);
        s += h * h;
      }
    } else {
      for (int64_t j = 0; j < n; ++j) {
        double h = dotd(A + j * lda, ai, m);
        s += h * h;
      }
    }
    f[i] = s;
  }
  return ORC_OK;
}

/*
 * Pieces of one greedy step.  Notation of Sections 4 and 5: after the picks
 * S so far, P projects onto span(A_S), E = (I - P) A and F = (I - P) B are the
 * residuals of the source and the target, G = E^T E and H = F^T E.  Column i
 * scores f_i / g_i with f_i = ||H_{:i}||^2 and g_i = G_ii (Lemma 1 and
 * Theorem 1 for B = A, Theorem 3 otherwise).  The history kept is, per pick
 * r, the n-vector W_r = G^{(r)}_{:p_r} / sqrt(G^{(r)}_{p_r p_r}) (omega) and
 * the target-side vector U_r = H^{(r)}_{:p_r} / sqrt(G^{(r)}_{p_r p_r})
 * (upsilon; for B = A it is W_r itself).
 */

/* Best candidate by f_i / g_i (the greedy criterion of Problems 3 and 6).
 * A candidate is unpicked, not dropped, has g0_i > 0, finite f_i and g_i and
 * g_i > tau * g0_i; on equal ratios the lower index wins.  *second receives
 * the runner-up ratio (-inf if none).  Returns -1 when there is no candidate. */
static int64_t best_candidate(const double *f, const double *g, const double *g0,
                              const unsigned char *excl, int64_t n, double tau,
                              double *first, double *second) {
  int64_t p = -1;
  double s1 = -INFINITY, s2 = -INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    if (excl[i]) continue;
    if (!(g0[i] > 0.0) || !isfinite(f[i]) || !isfinite(g[i])) continue;
    if (!(g[i] > tau * g0[i])) continue;
    double s = f[i] / g[i];
    if (s > s1) {
      s2 = s1;
      s1 = s;
      p = i;
    } else if (s > s2) {
      s2 = s;
    }
  }
  *first = s1;
  *second = s2;
  return p;
}

/* Column p of the residual Gram matrix, out = G_{:p} (Lemma 2 / Corollary 2:
 * each earlier pick r took W_r[p] W_r out of A^T A_p).  wp[r] = W_r[p]. */
static void residual_gram_column(const double *A, int64_t m, int64_t n, int64_t lda,
                                 const double *ap, const double *W, const double *wp, int32_t t,
                                 double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double d = dotd(A + i * lda, ap, m);
    for (int32_t s = 0; s < t; ++s) d -= wp[s] * W[(size_t)s * n + i];
    out[i] = d;
  }
}

/* Column p of the residual cross matrix, out = H_{:p} (r entries; the target
 * counterpart of residual_gram_column, Section 5.2). */
static void residual_cross_column(const double *B, int64_t m, int64_t r, int64_t ldb,
                                  const double *ap, const double *U, const double *wp, int32_t t,
                                  double *out) {
  for (int64_t c = 0; c < r; ++c) {
    double v = dotd(B + c * ldb, ap, m);
    for (int32_t s = 0; s < t; ++s) v -= wp[s] * U[(size_t)s * r + c];
    out[c] = v;
  }
}

/* The n-vector H^T upsilon that the update of f needs (Theorem 4; Theorem 2
 * for B = A, where it is G^T omega): A^T (B upsilon) with the earlier picks'
 * share removed, sum_r (U_r . upsilon) W_r.  y, coef: scratch (m, t). */
static int deflation_term(const double *A, int64_t m, int64_t n, int64_t lda, const double *B,
                          int64_t r, int64_t ldb, const double *W, const double *U,
                          const double *ups, int64_t rr, int32_t t, double *y, double *coef,
                          double *out) {
  if (!B) {
    int st = matvec_cols(A, m, n, lda, ups, y); /* A omega */
    if (st != ORC_OK) return st;
  } else {
    for (int64_t j = 0; j < m; ++j) y[j] = 0.0; /* B upsilon */
    for (int64_t c = 0; c < r; ++c) {
      const double *bc = B + c * ldb;
      for (int64_t j = 0; j < m; ++j) y[j] += ups[c] * bc[j];
    }
  }
  for (int32_t s = 0; s < t; ++s) {
    const double *us = B ? (U + (size_t)s * rr) : (W + (size_t)s * n);
    coef[s] = dotd(us, ups, rr);
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double v = dotd(A + i * lda, y, m);
    for (int32_t s = 0; s < t; ++s) v -= coef[s] * W[(size_t)s * n + i];
    out[i] = v;
  }
  return ORC_OK;
}

/* Rank-one deflation of G and H by the new pick, seen through the scores
 * (Theorem 4 / Theorem 2): ||H_{:i} - omega_i upsilon||^2 and
 * G_ii - omega_i^2, with hu = H^T upsilon and un = ||upsilon||^2. */
static void rank_one_update(double *f, double *g, const double *om, const double *hu, double un,
                            int64_t n) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double w = om[i];
    f[i] = f[i] - 2.0 * w * hu[i] + un * w * w;
    g[i] = g[i] - w * w;
  }
}

/*
 * Greedy generalized CSS, Algorithm 3 (B != NULL) / Algorithm 1 (B == NULL),
 * kept in the recursive form of Theorems 2 and 4: the scores are updated from
 * the history W, U, never recomputed from a projection.
 *
 * Inputs
 *   A      m x n column-major, leading dimension lda (source matrix)
 *   B      m x r column-major, leading dimension ldb (target), or NULL for B = A
 *   k      number of columns to select
 *   tau    eligibility threshold: column i is a candidate iff it is not
 *          selected, g0_i > 0, g_i > tau * g0_i and f_i, g_i are finite.
 *          (The paper leaves the degenerate 0/0 ratio undefined.)
 * Outputs (any optional pointer may be NULL)
 *   idx[k]        picks in order; -1 for picks not made
 *   obj[k+1]      obj[0] = ||B||_F^2, obj[t] = obj[t-1] - f_p/g_p  (Theorems 1/3)
 *   upsn[k]       ||upsilon^(t)||^2 per step (equal to f_p/g_p in exact arithmetic)
 *   score[k]      f_p/g_p at the pick
 *   gap[k]        (s1 - s2)/s1 for the two best candidate ratios (1 if only one)
 *   omega_out     k x n, row t = omega^(t)  (rows of W = Q^T A)
 *   fg_trace      k x 2n, row t = [f^(t), g^(t)] just before pick t
 *   g_final[n]    g after the last update
 *   n_selected    number of picks made
 * Returns ORC_OK, ORC_EXHAUSTED (fewer than k candidates) or an error.
 *
 * A pick whose G_pp <= tau * g0_p (a column that rounding made look
 * independent) is dropped from the candidates and the search is repeated.
 */
int orc_select(const double *A, int64_t m, int64_t n, int64_t lda,
               const double *B, int64_t r, int64_t ldb, int32_t k, double tau,
               int64_t *idx, double *obj, double *upsn, double *score, double *gap,
               double *omega_out, double *fg_trace, double *g_final,
               int32_t *n_selected) {
  if (!A || m < 1 || n < 1 || lda < m || k < 1 || !idx) return ORC_ERR_ARG;
  if (B && (r < 1 || ldb < m)) return ORC_ERR_ARG;
  const int self = (B == NULL);
  const int64_t rr = self ? n : r; /* length of upsilon */
  int status = ORC_OK;

  double *f = (double *)malloc(sizeof(double) * n);
  double *g = (double *)malloc(sizeof(double) * n);
  double *g0 = (double *)malloc(sizeof(double) * n);
  unsigned char *excl = (unsigned char *)calloc((size_t)n, 1); /* 1 selected, 2 dropped */
  double *W = (double *)malloc(sizeof(double) * (size_t)k * n);        /* omega history */
  double *Ups = self ? NULL : (double *)malloc(sizeof(double) * (size_t)k * rr);
  double *gcol = (double *)malloc(sizeof(double) * n);
  double *hcol = (double *)malloc(sizeof(double) * rr);
  double *ups = (double *)malloc(sizeof(double) * rr);
  double *hu = (double *)malloc(sizeof(double) * n);
  double *y = (double *)malloc(sizeof(double) * m);
  double *wp = (double *)malloc(sizeof(double) * (k > 0 ? k : 1));
  double *coef = (double *)malloc(sizeof(double) * (k > 0 ? k : 1));
  if (!f || !g || !g0 || !excl || !W || (!self && !Ups) || !gcol || !hcol || !ups ||
      !hu || !y || !wp || !coef) {
    status = ORC_ERR_NOMEM;
    goto done;
  }

  status = orc_init_scores(A, m, n, lda, B, r, ldb, f, g);
  if (status != ORC_OK) goto done;
  memcpy(g0, g, sizeof(double) * n);

  /* F(empty set) = ||B||_F^2 */
  {
    double F0 = 0.0;
    if (self) {
      for (int64_t i = 0; i < n; ++i) F0 += g0[i];
    } else {
      for (int64_t c = 0; c < r; ++c) F0 += dotd(B + c * ldb, B + c * ldb, m);
    }
    if (obj) obj[0] = F0;
  }
  for (int32_t t = 0; t < k; ++t) idx[t] = -1;

  int32_t t = 0;
  while (t < k) {
    if (fg_trace) {
      memcpy(fg_trace + (size_t)t * 2 * n, f, sizeof(double) * n);
      memcpy(fg_trace + (size_t)t * 2 * n + n, g, sizeof(double) * n);
    }
    double s1, s2;
    const int64_t p = best_candidate(f, g, g0, excl, n, tau, &s1, &s2);
    if (p < 0) {
      status = ORC_EXHAUSTED;
      break;
    }

    const double *ap = A + p * lda;
    for (int32_t s = 0; s < t; ++s) wp[s] = W[(size_t)s * n + p];
    residual_gram_column(A, m, n, lda, ap, W, wp, t, gcol);
    const double gpp = gcol[p];
    if (!(gpp > tau * g0[p])) {
      excl[p] = 2; /* rounding made column p look independent */
      continue;
    }
    const double sq = sqrt(gpp);

    if (self)
      memcpy(hcol, gcol, sizeof(double) * n); /* H = G when B = A */
    else
      residual_cross_column(B, m, r, ldb, ap, Ups, wp, t, hcol);

    /* the new history entries: G_{:p} and H_{:p} scaled by 1 / sqrt(G_pp) */
    double *om = W + (size_t)t * n;
    for (int64_t i = 0; i < n; ++i) om[i] = gcol[i] / sq;
    double un = 0.0;
    for (int64_t c = 0; c < rr; ++c) {
      ups[c] = hcol[c] / sq;
      un += ups[c] * ups[c];
    }

    status = deflation_term(A, m, n, lda, B, r, ldb, W, Ups, ups, rr, t, y, coef, hu);
    if (status != ORC_OK) goto done;

    const double sc = f[p] / g[p];
    if (score) score[t] = sc;
    if (gap) gap[t] = (s2 == -INFINITY || s1 <= 0.0) ? 1.0 : (s1 - s2) / s1;
    if (upsn) upsn[t] = un;
    if (obj) obj[t + 1] = obj[t] - sc;
    if (!self) memcpy(Ups + (size_t)t * rr, ups, sizeof(double) * rr);

    rank_one_update(f, g, om, hu, un, n);
    excl[p] = 1;
    idx[t] = p;
    ++t;
  }

  if (obj)
    for (int32_t s = t; s < k; ++s) obj[s + 1] = obj[s];
  if (omega_out) {
    memcpy(omega_out, W, sizeof(double) * (size_t)t * n);
    if (t < k) memset(omega_out + (size_t)t * n, 0, sizeof(double) * (size_t)(k - t) * n);
  }
  if (g_final) memcpy(g_final, g, sizeof(double) * n);
  if (n_selected) *n_selected = t;

done:
  free(f);
  free(g);
  free(g0);
  free(excl);
  free(W);
  free(Ups);
  free(gcol);
  free(hcol);
  free(ups);
  free(hu);
  free(y);
  free(wp);
  free(coef);
  return status;
}

/*
 * Reconstruction error ||B - P_S B||_F^2 (B == NULL: B = A), with
 * S = idx[0..k-1].  P_S projects onto span(A_S) (Section 3.1).  A_S is
 * factored by Householder QR; a column whose remaining part is negligible
 * (dependent on the earlier ones) adds no direction.  With H the product of
 * the reflectors, the part of b outside span(A_S) is the tail of H b below
 * the rank, so the error is the sum of those tail squares over all columns
 * of B.
 */
int orc_error(const double *A, int64_t m, int64_t n, int64_t lda, const int64_t *idx,
              int32_t k, const double *B, int64_t r, int64_t ldb, double *err) {
  if (!A || m < 1 || n < 1 || lda < m || k < 0 || !err) return ORC_ERR_ARG;
  if (B && (r < 1 || ldb < m)) return ORC_ERR_ARG;
  for (int32_t s = 0; s < k; ++s)
    if (idx[s] < 0 || idx[s] >= n) return ORC_ERR_ARG;
  const int64_t nb = B ? r : n;
  double *V = (double *)calloc((size_t)(k > 0 ? k : 1) * m, sizeof(double)); /* reflectors */
  double *x = (double *)malloc(sizeof(double) * m);
  double *col_err = (double *)malloc(sizeof(double) * nb);
  if (!V || !x || !col_err) {
    free(V);
    free(x);
    free(col_err);
    return ORC_ERR_NOMEM;
  }
  int64_t rank = 0;
  for (int32_t s = 0; s < k && rank < m; ++s) {
    const double *a = A + idx[s] * lda;
    memcpy(x, a, sizeof(double) * m);
    double anrm = sqrt(dotd(a, a, m));
    for (int64_t h = 0; h < rank; ++h) { /* apply earlier reflectors */
      const double *v = V + h * m;
      double c = 2.0 * dotd(v + h, x + h, m - h);
      for (int64_t j = h; j < m; ++j) x[j] -= c * v[j];
    }
    double tn = sqrt(dotd(x + rank, x + rank, m - rank));
    if (!(tn > 1e-13 * anrm)) continue; /* dependent column: adds no direction */
    double *v = V + rank * m;
    for (int64_t j = 0; j < m; ++j) v[j] = 0.0;
    for (int64_t j = rank; j < m; ++j) v[j] = x[j];
    v[rank] += (x[rank] >= 0.0 ? tn : -tn);
    double vn = sqrt(dotd(v + rank, v + rank, m - rank));
    for (int64_t j = rank; j < m; ++j) v[j] /= vn;
    ++rank;
  }
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t c = 0; c < nb; ++c) {
    double *b = (double *)malloc(sizeof(double) * m);
    const double *src = B ? (B + c * ldb) : (A + c * lda);
    memcpy(b, src, sizeof(double) * m);
    for (int64_t h = 0; h < rank; ++h) {
      const double *v = V + h * m;
      double cc = 2.0 * dotd(v + h, b + h, m - h);
      for (int64_t j = h; j < m; ++j) b[j] -= cc * v[j];
    }
    col_err[c] = dotd(b + rank, b + rank, m - rank);
    free(b);
  }
  double e = 0.0;
  for (int64_t c = 0; c < nb; ++c) e += col_err[c];
  *err = e;
  free(V);
  free(x);
  free(col_err);
  return ORC_OK;
}

/*
 * Algorithm 4 on one machine: Algorithm 3 with (A_(b), B, l_(b)) on every
 * block b of consecutive columns col_off[b] .. col_off[b+1]-1, then the
 * picked columns are pooled (block order, then pick order within a block)
 * and Algorithm 3 selects k_merge of them against the same B.
 *
 * Budgets: l_(b) = k_blocks[b] (0 <= l_(b) <= k_block; a block with budget 0
 * contributes nothing), or k_block for every block when k_blocks is NULL.
 * Outputs: idx_block[b*k_block + j] global index of block b's j-th pick
 * (-1 if none); idx_merge[k_merge] global indices; obj_merge[k_merge+1].
 */
int orc_select_distributed(const double *A, int64_t m, int64_t n, int64_t lda,
                           const double *B, int64_t r, int64_t ldb, int32_t nblocks,
                           const int64_t *col_off, int32_t k_block, const int32_t *k_blocks,
                           int32_t k_merge, double tau, int64_t *idx_block,
                           int64_t *idx_merge, double *obj_merge, int32_t *n_merge) {
  if (!A || !B || nblocks < 1 || !col_off || k_block < 1 || k_merge < 1) return ORC_ERR_ARG;
  if (col_off[0] != 0 || col_off[nblocks] != n) return ORC_ERR_ARG;
  for (int32_t b = 0; b < nblocks; ++b) {
    if (col_off[b + 1] <= col_off[b]) return ORC_ERR_ARG;
    if (k_blocks && (k_blocks[b] < 0 || k_blocks[b] > k_block)) return ORC_ERR_ARG;
  }
  int64_t npool = 0;
  for (int32_t b = 0; b < nblocks; ++b) {
    int64_t w = col_off[b + 1] - col_off[b];
    int64_t *loc = idx_block + (size_t)b * k_block;
    const int32_t lb = k_blocks ? k_blocks[b] : k_block;
    for (int32_t j = 0; j < k_block; ++j) loc[j] = -1;
    if (lb == 0) continue;
    int32_t ns = 0;
    int st = orc_select(A + col_off[b] * lda, m, w, lda, B, r, ldb, lb, tau, loc, NULL,
                        NULL, NULL, NULL, NULL, NULL, NULL, &ns);
    if (st < 0) return st;
    for (int32_t j = 0; j < lb; ++j)
      if (loc[j] >= 0) {
        loc[j] += col_off[b];
        ++npool;
      }
  }
  if (npool == 0) return ORC_EXHAUSTED;
  double *P = (double *)malloc(sizeof(double) * (size_t)npool * m);
  int64_t *gidx = (int64_t *)malloc(sizeof(int64_t) * npool);
  int64_t *loc = (int64_t *)malloc(sizeof(int64_t) * k_merge);
  if (!P || !gidx || !loc) {
    free(P);
    free(gidx);
    free(loc);
    return ORC_ERR_NOMEM;
  }
  int64_t q = 0;
  for (int32_t b = 0; b < nblocks; ++b)
    for (int32_t j = 0; j < k_block; ++j) {
      int64_t gi = idx_block[(size_t)b * k_block + j];
      if (gi < 0) continue;
      memcpy(P + q * m, A + gi * lda, sizeof(double) * m);
      gidx[q++] = gi;
    }
  int32_t ns = 0;
  int st = orc_select(P, m, npool, m, B, r, ldb, k_merge, tau, loc, obj_merge, NULL, NULL,
                      NULL, NULL, NULL, NULL, &ns);
  for (int32_t j = 0; j < k_merge; ++j) idx_merge[j] = loc[j] >= 0 ? gidx[loc[j]] : -1;
  if (n_merge) *n_merge = ns;
  free(P);
  free(gidx);
  free(loc);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Storage formats                                                          */
/* ------------------------------------------------------------------------ */

/* bfloat16: the upper 16 bits of an IEEE binary32 (1 sign, 8 exponent, 7
 * fraction bits).  Decoding appends 16 zero bits. */
float orc_bf16_decode(uint16_t h) {
  uint32_t b = (uint32_t)h << 16;
  float x;
  memcpy(&x, &b, 4);
  return x;
}

/* Round a binary32 value to the nearest bfloat16, ties to the even code.
 * Done by comparing the two neighbouring bfloat16 values in double. */
uint16_t orc_bf16_encode(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  uint16_t sign = (uint16_t)((b >> 16) & 0x8000u);
  if (isnan(x)) return (uint16_t)(sign | 0x7FC0u);
  uint16_t lo = (uint16_t)(b >> 16) & 0x7FFFu; /* |x| truncated */
  if (lo == 0x7F80u) return (uint16_t)(sign | lo); /* infinity */
  double ax = fabs((double)x);
  double vlo = fabs((double)orc_bf16_decode(lo));
  double vhi = (lo == 0x7F7Fu) ? ldexp(1.0, 128) : fabs((double)orc_bf16_decode((uint16_t)(lo + 1)));
  uint16_t code;
  if (ax - vlo < vhi - ax)
    code = lo;
  else if (ax - vlo > vhi - ax)
    code = (uint16_t)(lo + 1);
  else
    code = (lo & 1u) ? (uint16_t)(lo + 1) : lo;
  return (uint16_t)(sign | code);
}

/* OCP FP8 E4M3 ("e4m3fn"): 1 sign, 4 exponent (bias 7), 3 mantissa bits.
 * Exponent field 0 encodes subnormals m * 2^-9; S.1111.111 is NaN; there
 * are no infinities; the largest finite magnitude is 1.75 * 2^8 = 448. */
double orc_fp8_decode(uint8_t c) {
  int s = (c >> 7) & 1, e = (c >> 3) & 15, mt = c & 7;
  double v;
  if (e == 15 && mt == 7) return NAN;
  if (e == 0)
    v = ldexp((double)mt, -9);
  else
    v = ldexp(1.0 + mt / 8.0, e - 7);
  return s ? -v : v;
}

/* Nearest E4M3 code to x, ties to the even code, magnitudes above 448
 * saturate to 448, NaN stays NaN.  The 127 finite non-negative codes are
 * increasing in value; a binary search finds the largest code not above |x|,
 * then the nearer of it and the next code is taken. */
uint8_t orc_fp8_encode(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  uint8_t sign = (uint8_t)((b >> 24) & 0x80u);
  if (isnan(x)) return (uint8_t)(sign | 0x7Fu);
  double ax = fabs((double)x);
  if (ax >= 448.0) return (uint8_t)(sign | 0x7Eu);
  int lo = 0, hi = 0x7E; /* decode(lo) <= ax < decode(hi) */
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (orc_fp8_decode((uint8_t)mid) <= ax)
      lo = mid;
    else
      hi = mid;
  }
  double vlo = orc_fp8_decode((uint8_t)lo);
  if (vlo == ax) return (uint8_t)(sign | lo);
  double vhi = orc_fp8_decode((uint8_t)(lo + 1));
  uint8_t code;
  if (ax - vlo < vhi - ax)
    code = (uint8_t)lo;
  else if (ax - vlo > vhi - ax)
    code = (uint8_t)(lo + 1);
  else
    code = (lo & 1) ? (uint8_t)(lo + 1) : (uint8_t)lo;
  return (uint8_t)(sign | code);
}

/* Per-column FP8 quantization of a binary32 matrix: scale_i = max_j |A_ji| / 448
 * (binary32 division), 1 for an all-zero column; code = nearest E4M3 of the
 * binary32 quotient A_ji / scale_i. */
void orc_quantize_fp8(const float *A, int64_t m, int64_t n, int64_t lda, uint8_t *out,
                      int64_t ldo, float *scales) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const float *a = A + i * lda;
    float amax = 0.0f;
    for (int64_t j = 0; j < m; ++j) {
      float v = fabsf(a[j]);
      if (v > amax) amax = v;
    }
    float s = (amax > 0.0f) ? amax / 448.0f : 1.0f;
    scales[i] = s;
    for (int64_t j = 0; j < m; ++j) out[i * ldo + j] = orc_fp8_encode(a[j] / s);
    for (int64_t j = m; j < ldo; ++j) out[i * ldo + j] = 0;
  }
}

void orc_quantize_bf16(const float *A, int64_t m, int64_t n, int64_t lda, uint16_t *out,
                       int64_t ldo) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < m; ++j) out[i * ldo + j] = orc_bf16_encode(A[i * lda + j]);
    for (int64_t j = m; j < ldo; ++j) out[i * ldo + j] = 0;
  }
}

/* Decode stored columns to double: dtype 0 binary32, 1 bfloat16, 2 E4M3 with
 * per-column scales (value = scale_i * decode(code)). */
void orc_decode_columns(const void *src, int dtype, int64_t m, int64_t n, int64_t lds,
                        const float *scales, double *dst, int64_t ldd) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < m; ++j) {
      double v;
      if (dtype == 0)
        v = (double)((const float *)src)[i * lds + j];
      else if (dtype == 1)
        v = (double)orc_bf16_decode(((const uint16_t *)src)[i * lds + j]);
      else
        v = (double)scales[i] * orc_fp8_decode(((const uint8_t *)src)[i * lds + j]);
      dst[i * ldd + j] = v;
    }
  }
}
