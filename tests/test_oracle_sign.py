"""Pins of the oracle's random sign matrices (Section 5.1: Omega with i.i.d.
+-1 or sparse +-1 entries drawn per column of A): the generator against its
published known-answer vectors, and the entry distribution against its
definition by counting."""
import json
import os

import numpy as np
import pytest

from oracle import rng

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLD, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = np.array([[int(x, 16) for x in v["counter"]]], dtype=np.uint32)
        key = np.array([int(x, 16) for x in v["key"]], dtype=np.uint32)
        out = rng.philox4x32_10(ctr, key)[0]
        assert [f"{int(x):08x}" for x in out] == v["output"]


@pytest.mark.parametrize("n,r", [(40000, 64), (9000, 301)])
def test_sparse_sign_density_and_balance(n, r):
    d = 1.0 / np.sqrt(n)
    Om = rng.omega_rows(0, n, r, seed=7, density=d)
    assert set(np.unique(Om)) <= {-1.0, 0.0, 1.0}
    N = n * r
    p = rng.threshold(d) / 2.0 ** 31
    nnz = int(np.count_nonzero(Om))
    assert abs(nnz - N * p) <= 5 * np.sqrt(N * p * (1 - p))
    pos = int(np.sum(Om > 0))
    assert abs(pos - nnz / 2) <= 5 * np.sqrt(nnz / 4)
    # columns are uncorrelated: Omega^T Omega ~ n p I
    G = Om.T @ Om
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) <= 8 * np.sqrt(n) * p


def test_dense_sign_and_threshold_edges():
    Om = rng.omega_rows(0, 5000, 37, seed=3, density=1.0)
    assert np.all(np.abs(Om) == 1.0)
    assert abs(np.mean(Om)) <= 5 / np.sqrt(Om.size)
    assert rng.threshold(1.0) == 1 << 31
    assert rng.threshold(1e-30) == 1
    assert rng.threshold(0.5) == 1 << 30


def test_rows_are_counter_based():
    """A row depends only on (seed, i): any split into chunks gives the same
    matrix, and both seed words matter."""
    a = rng.omega_rows(0, 300, 13, seed=11, density=0.3)
    b = np.vstack([rng.omega_rows(0, 128, 13, 11, 0.3), rng.omega_rows(128, 300, 13, 11, 0.3)])
    assert np.array_equal(a, b)
    assert np.array_equal(rng.omega_rows(200, 201, 13, 11, 0.3)[0], a[200])
    assert not np.array_equal(a, rng.omega_rows(0, 300, 13, 11 + (1 << 32), 0.3))
    assert not np.array_equal(a, rng.omega_rows(0, 300, 13, 12, 0.3))
    # a row beyond 2^32 uses the counter's high word
    hi = rng.omega_rows((1 << 32) + 5, (1 << 32) + 6, 13, 11, 0.3)[0]
    assert not np.array_equal(hi, a[5]) or np.count_nonzero(a[5]) == 0


def test_projection_is_the_sum_of_column_outer_products():
    """B = sum_i A_i Omega_i: (Section 5.1's map step, accumulated in memory)."""
    rs = np.random.default_rng(0)
    A = rs.standard_normal((30, 500))
    B = rng.project_sign(A, seed=5, density=0.1, r=9, chunk=64)
    Bl = np.zeros((30, 9))
    for i in range(500):
        Bl += np.outer(A[:, i], rng.omega_rows(i, i + 1, 9, 5, 0.1)[0])
    np.testing.assert_allclose(B, Bl, atol=1e-12)


def test_single_column_equals_the_matrix_column():
    Om = rng.omega_rows(0, 3000, 11, seed=9, density=0.05)
    for j in (0, 3, 4, 10):
        assert np.array_equal(rng.omega_column(3000, j, 9, 0.05, chunk=700), Om[:, j])
    Od = rng.omega_rows(0, 500, 6, seed=2, density=1.0)
    assert np.array_equal(rng.omega_column(500, 5, 2, 1.0), Od[:, 5])
