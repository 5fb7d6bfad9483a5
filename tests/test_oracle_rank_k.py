"""Pins of the oracle's embedding outputs (Section 3: W = Q^T A, Boutsidis et
al.'s rank-k approximation in span(A_S), Eq. ApproxSVD) to facts fixed by
the mathematics, each computed by another route: the truncated SVD of the
projection P_S A (least squares + SVD of the m x n matrix), the explicit
projection error (Householder QR in the C oracle), a search over rank-k
coefficient matrices by alternating least squares, and the SVD of an
exactly low-rank A.
"""
import numpy as np
import pytest

import oracle
from oracle import embed
import synth


def cs(M):
    return synth.to_colstore(M, lda=M.shape[0], dtype=np.float64)


def _case(seed, m=15, n=40, l=6):
    A = synth.spectral_lowrank_dense(m, n, 10, 0.6, 1e-2, seed=seed)
    S = oracle.select(cs(A), m, l)["idx"]
    return A, [int(x) for x in S]


def _proj_truncated(A, S, k):
    """(P_S A)_k by another route: P_S A = A_S X with X the least-squares
    solution of A_S X = A, then the SVD of the m x n matrix."""
    AS = A[:, S]
    X = np.linalg.lstsq(AS, A, rcond=None)[0]
    PA = AS @ X
    U, s, Vt = np.linalg.svd(PA, full_matrices=False)
    return PA, (U[:, :k] * s[:k]) @ Vt[:k], s


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rank_k_is_truncated_svd_of_the_projection(seed):
    A, S = _case(seed)
    for k in range(1, len(S) + 1):
        res = embed.rank_k(A, S, k)
        PA, PAk, s = _proj_truncated(A, S, k)
        np.testing.assert_allclose(res["approx"], PAk, atol=1e-10 * np.abs(A).max())
        np.testing.assert_allclose(res["sigma"], s[:k], rtol=1e-10)
        e_ref = np.sum((A - PA) ** 2) + np.sum(s[k:] ** 2)
        assert abs(res["err"] - e_ref) <= 1e-10 * np.sum(A * A)


def test_rank_l_equals_projection_error():
    A, S = _case(3, m=20, n=50, l=8)
    res = embed.rank_k(A, S, len(S))
    e = oracle.error(cs(A), A.shape[0], S)
    assert abs(res["err"] - e) <= 1e-10 * e


@pytest.mark.parametrize("k", [1, 2, 4])
def test_rank_k_is_optimal_among_rank_k_coefficients(k):
    """min over rank-k T of ||A - A_S T||^2 by alternating least squares from
    random starts reaches, and never beats, the oracle's error; A_S times the
    coefficients of A's own truncated SVD does no better either."""
    A, S = _case(4, m=10, n=16, l=5)
    AS = A[:, S]
    res = embed.rank_k(A, S, k)
    rng = np.random.default_rng(k)
    best = np.inf
    for _ in range(10):
        Y = rng.standard_normal((A.shape[1], k))
        for _ in range(500):
            # X given Y: min ||A - AS X Y^T||: X = pinv(AS) A Y (Y^T Y)^-1
            X = np.linalg.lstsq(AS, A @ Y @ np.linalg.inv(Y.T @ Y), rcond=None)[0]
            # Y given X: rows of A^T against (AS X)
            Y = np.linalg.lstsq(AS @ X, A, rcond=None)[0].T
        best = min(best, float(np.sum((A - AS @ X @ Y.T) ** 2)))
    F = np.sum(A * A)
    assert best >= res["err"] - 1e-10 * F
    assert best <= res["err"] + 1e-7 * F
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    Ak = (U[:, :k] * s[:k]) @ Vt[:k]
    T = np.linalg.lstsq(AS, Ak, rcond=None)[0]
    assert np.sum((A - AS @ T) ** 2) >= res["err"] - 1e-10 * F


def test_exact_low_rank_gives_the_svd_of_a():
    """S spans an exactly rank-r A: the rank-r approximation is A itself and
    the triplets are A's own singular triplets (with the sign convention)."""
    m, n, r = 12, 30, 4
    A = synth.int_lowrank_dense(m, n, r, seed=11)
    S = [int(x) for x in oracle.select(cs(A), m, r)["idx"]]
    res = embed.rank_k(A, S, r)
    assert res["err"] <= 1e-20 * np.sum(A * A)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    np.testing.assert_allclose(res["sigma"], s[:r], rtol=1e-12)
    Uf, Vf = embed.sign_fix(U[:, :r], Vt[:r].T)
    np.testing.assert_allclose(res["U"], Uf, atol=1e-10)
    np.testing.assert_allclose(res["V"], Vf, atol=1e-10)


def test_triplets_are_orthonormal_and_diagonalise_a():
    """U_A^T A V_A = Sigma_k (A = Q W + E with Q^T E = 0), orthonormal
    factors, and each U_A column's largest-magnitude entry is positive."""
    A, S = _case(5, m=25, n=60, l=9)
    res = embed.rank_k(A, S, 6)
    U, V, s = res["U"], res["V"], res["sigma"]
    np.testing.assert_allclose(U.T @ U, np.eye(6), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(6), atol=1e-12)
    np.testing.assert_allclose(U.T @ A @ V, np.diag(s), atol=1e-10 * s[0])
    for j in range(6):
        i = int(np.argmax(np.abs(U[:, j])))
        assert U[i, j] > 0


def test_embedding_matches_the_selection_omega_rows():
    """W from a QR of A_S equals the omega rows of Algorithm 1 up to the sign
    of each basis vector."""
    A, S = _case(6, m=18, n=35, l=5)
    Q, W = embed.embedding(A, S)
    om = oracle.select(cs(A), A.shape[0], 5, omega=True)["omega"]
    np.testing.assert_allclose(np.abs(W), np.abs(om), atol=1e-12 * np.abs(A).max())
