"""Pins of the quality metric's oracle (Section 7's relative accuracy, the
best rank-l error, the leading singular triplets and the DistApproxSVD
target) to closed forms: matrices built with known singular values and
vectors, and orthogonal columns, where greedy selection, the SVD and the
projections all have exact answers."""
import numpy as np
import pytest

import oracle
from oracle import quality
import synth


def cs(M):
    return synth.to_colstore(M, lda=M.shape[0], dtype=np.float64)


def _known(m, n, s, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, len(s))))
    V, _ = np.linalg.qr(rng.standard_normal((n, len(s))))
    return (U * s) @ V.T, U, V


def test_top_eig_and_best_rank_error_closed_form():
    s = np.array([5.0, 3.0, 2.0, 1.0, 0.5, 0.25])
    A, U, V = _known(20, 40, s, seed=1)
    lam, Uk = quality.top_eig(A, 4)
    np.testing.assert_allclose(lam, s[:4] ** 2, rtol=1e-12)
    # the same vectors as the construction, up to the sign convention
    for j in range(4):
        assert abs(abs(Uk[:, j] @ U[:, j]) - 1.0) <= 1e-12
        i = int(np.argmax(np.abs(Uk[:, j])))
        assert Uk[i, j] > 0
    for l in range(len(s) + 1):
        assert abs(quality.best_rank_error(A, l) - np.sum(s[l:] ** 2)) <= 1e-12 * np.sum(s ** 2)
    B = quality.svd_target(A, 3)
    np.testing.assert_allclose(B.T @ B, np.diag(s[:3] ** 2), atol=1e-12)
    # B B^T is the best rank-3 part of A A^T
    np.testing.assert_allclose(B @ B.T, (U[:, :3] * s[:3] ** 2) @ U[:, :3].T, atol=1e-12)


def test_relative_accuracy_orthogonal_columns():
    """Orthogonal columns: greedy picks the largest norms, which is also the
    best rank-l approximation, so its relative accuracy is exactly 100%; a
    uniform subset's error is the sum of the squared norms it leaves out."""
    d = np.array([9.0, 7.0, 5.0, 4.0, 3.0, 2.0, 1.5, 1.0])
    A = np.zeros((10, 8))
    A[np.arange(8), np.arange(8)] = d
    A = np.linalg.qr(np.random.default_rng(0).standard_normal((10, 10)))[0] @ A
    l = 3
    S = oracle.select(cs(A), 10, l)["idx"]
    assert sorted(S.tolist()) == [0, 1, 2]
    err_s = oracle.error(cs(A), 10, S)
    err_l = quality.best_rank_error(A, l)
    subsets = synth.uniform_subsets(8, l, range(10))
    errs_u = [oracle.error(cs(A), 10, U) for U in subsets]
    for U, e in zip(subsets, errs_u):
        assert abs(e - (np.sum(d ** 2) - np.sum(d[U] ** 2))) <= 1e-10 * np.sum(d ** 2)
    ra = quality.relative_accuracy(err_s, errs_u, err_l)
    assert abs(ra - 100.0) <= 1e-8
    # a hand-computed case: norms eu = mean of roots
    ra2 = quality.relative_accuracy(4.0, [16.0, 36.0], 1.0)
    assert abs(ra2 - (5.0 - 2.0) / (5.0 - 1.0) * 100.0) <= 1e-12


def test_uniform_subsets_are_distinct_and_reproducible():
    a = synth.uniform_subsets(1000, 50, range(10))
    b = synth.uniform_subsets(1000, 50, range(10))
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert all(len(set(x.tolist())) == 50 and x.min() >= 0 and x.max() < 1000 for x in a)
    assert len({tuple(x.tolist()) for x in a}) == 10


def test_svd_target_selection_prefers_leading_directions():
    """With B = U_k Sigma_k, the objective F(S) = ||B - P_S B||^2 of the
    greedy picks never exceeds that of k uniform subsets (sanity of the
    DistApproxSVD target), and F(empty) = sum of the k leading sigma^2."""
    A = synth.spectral_lowrank_dense(30, 200, 20, 1.0, 1e-3, seed=3)
    B = quality.svd_target(A, 5)
    res = oracle.select(cs(A), 30, 5, B=cs(B))
    s = np.linalg.svd(A, compute_uv=False)
    assert abs(res["obj"][0] - np.sum(s[:5] ** 2)) <= 1e-12 * res["obj"][0]
    for U in synth.uniform_subsets(200, 5, range(5)):
        assert res["obj"][5] <= oracle.error(cs(A), 30, U, B=cs(B)) * (1 + 1e-12)
