"""Pins of the naive distributed selection (Section 5's first approach):
budgets by their definitions, the naive objective as the sum of the
blocks' projection errors, and the failure the paper describes when all
representative columns sit on one machine."""
import numpy as np

import oracle
from oracle import naive
import synth


def cs(M):
    return synth.to_colstore(M, lda=M.shape[0], dtype=np.float64)


def test_budgets():
    A = np.zeros((3, 10))
    A[:, 0:2] = 3.0      # block 0: ||.||^2 = 54
    A[:, 2:6] = 1.0      # block 1: 12
    A[:, 6:10] = 0.5     # block 2: 3
    off = [0, 2, 6, 10]
    # 7/3 each, block 0 capped at its width 2, the leftover to block 1 (first
    # of the equal remainders with room)
    assert naive.budgets(A, off, 7, "uniform") == [2, 3, 2]
    b = naive.budgets(A, off, 7, "adaptive")
    # shares 7*54/69 = 5.48 (capped at width 2), 1.22, 0.30 -> capacity decides
    assert sum(b) == 7 and b[0] == 2 and b[1] <= 4 and b[2] <= 4
    assert naive.budgets(A, off, 3, "uniform") == [1, 1, 1]
    assert naive.budgets(A, off, 4, "uniform") == [2, 1, 1]


def test_naive_objective_is_sum_of_block_errors():
    A = synth.gauss_lowrank_dense(20, 90, 6, 0.1, seed=3)
    off = [0, 30, 55, 90]
    r = naive.naive_select(A, off, 6)
    tot = 0.0
    for b in range(3):
        Ab = A[:, off[b]:off[b + 1]]
        loc = r["idx_block"][b] - off[b]
        tot += oracle.error(cs(Ab), 20, loc)
    assert abs(tot - sum(r["obj_block"])) <= 1e-10 * np.sum(A * A)


def test_all_representatives_on_one_machine():
    """Section 5: if the relevant columns all sit in one block, uniform
    budgets take too few of them, so the naive union approximates A worse
    than centralized greedy selection with the same number of columns."""
    rng = np.random.default_rng(0)
    m, k = 30, 6
    basis = np.linalg.qr(rng.standard_normal((m, k)))[0] * 10.0
    strong = basis @ rng.standard_normal((k, 12))         # all in block 0
    weak = 0.05 * rng.standard_normal((m, 48))
    A = np.hstack([strong, weak])
    off = [0, 12, 24, 36, 48, 60]
    r = naive.naive_select(A, off, k)
    assert r["budgets"] == [2, 1, 1, 1, 1]
    e_naive = oracle.error(cs(A), m, r["pool"])
    g = oracle.select(cs(A), m, k)
    e_greedy = oracle.error(cs(A), m, g["idx"])
    assert e_naive > 10.0 * e_greedy
    # the adaptive budget gives block 0 all of them and recovers the span
    ra = naive.naive_select(A, off, k, policy="adaptive")
    assert ra["budgets"][0] == k
    assert oracle.error(cs(A), m, ra["pool"]) <= 1.5 * e_greedy
