"""Pins of Algorithm 4's per-block budgets and of Algorithm 4 with them
(Section 5.2, the paragraph after Algorithm 4): the budget rules against
hand-computed cases and their invariants, the budgeted distributed
selection against its composition from single selections, and a planted
mistake in the budget rule that the pins catch."""
import numpy as np
import pytest

import oracle
from oracle import budgets as bud
import synth


def cs(M):
    return synth.to_colstore(M, lda=M.shape[0], dtype=np.float64)


def test_uniform_is_floor_of_l_over_c():
    # the paper's choice: floor(l / c) for every block, whatever is left over
    assert bud.budgets([1, 1, 1], [9, 9, 9], 7, "uniform") == [2, 2, 2]
    assert bud.budgets([1, 1, 1], [9, 1, 9], 7, "uniform") == [2, 1, 2]  # width cap
    assert bud.budgets([1] * 4, [5] * 4, 3, "uniform") == [0, 0, 0, 0]
    assert bud.budgets([1] * 64, [100] * 64, 100, "uniform") == [1] * 64


def test_norm_hand_computed():
    # shares 7*54/69 = 5.478, 7*12/69 = 1.217, 7*3/69 = 0.304 -> floors 5, 1, 0;
    # one column missing: block 0 has the largest remainder but no room
    # (width 5), so the next largest, block 2, takes it
    assert bud.budgets([54.0, 12.0, 3.0], [5, 5, 5], 7, "norm") == [5, 1, 1]
    # with room in block 0 it goes there
    assert bud.budgets([54.0, 12.0, 3.0], [9, 5, 5], 7, "norm") == [6, 1, 0]
    # equal remainders: the lower block first
    assert bud.budgets([1.0, 1.0, 1.0, 1.0], [5] * 4, 6, "norm") == [2, 2, 1, 1]
    # a zero matrix falls back to l / c
    assert bud.budgets([0.0, 0.0, 0.0], [5] * 3, 4, "norm") == [2, 1, 1]
    # l beyond the columns: every block full
    assert bud.budgets([3.0, 1.0], [2, 3], 9, "norm") == [2, 3]


def test_rounding_invariants():
    rng = np.random.default_rng(5)
    for _ in range(300):
        c = int(rng.integers(1, 12))
        widths = [int(x) for x in rng.integers(1, 40, size=c)]
        norms = list(rng.exponential(size=c) * (rng.random(c) > 0.2))
        l = int(rng.integers(0, 2 * sum(widths)))
        for pol in ("even", "norm"):
            b = bud.budgets(norms, widths, l, pol)
            assert sum(b) == min(l, sum(widths))
            assert all(0 <= x <= w for x, w in zip(b, widths))
            share = ([l / c] * c if pol == "even" or sum(norms) == 0
                     else [l * x / sum(norms) for x in norms])
            # largest-remainder rounding never moves a budget a whole column
            # below its share unless the width caps it
            for x, s, w in zip(b, share, widths):
                assert x >= min(int(np.floor(s)), w)
        u = bud.budgets(norms, widths, l, "uniform")
        assert all(x == min(l // c, w) for x, w in zip(u, widths))


def test_equal_norms_make_norm_equal_even():
    widths = [7, 12, 9, 4]
    for l in range(0, 33):
        assert bud.budgets([2.0] * 4, widths, l, "norm") == bud.budgets([0] * 4, widths, l, "even")
    # room decides once the shares overshoot the widths: l = 31 over four
    # blocks gives shares 7.75; blocks 0 and 3 are capped (7 and 4), the
    # rest goes to blocks 1 and 2 by remainder, then wherever there is room
    assert bud.budgets([0] * 4, widths, 31, "even") == [7, 11, 9, 4]
    assert bud.budgets([0] * 4, widths, 40, "even") == [7, 12, 9, 4]


def test_budgeted_distributed_is_blockwise_then_merge():
    m, r = 16, 5
    widths = [7, 12, 9, 5]
    off = np.concatenate([[0], np.cumsum(widths)])
    n = int(off[-1])
    A = synth.gauss_lowrank_dense(m, n, 6, 0.05, seed=71)
    B = A @ synth.omega_gauss(n, r, seed=72).astype(np.float64)
    kbs = [2, 4, 0, 3]  # block 2 contributes nothing
    d = oracle.select_distributed(cs(A), m, cs(B), off, 4, 5, k_blocks=kbs)
    pool = []
    for b in range(4):
        row = list(d["idx_block"][b])
        if kbs[b] == 0:
            assert row == [-1] * 4
            continue
        rb = oracle.select(cs(A[:, off[b]:off[b + 1]]), m, kbs[b], B=cs(B))
        assert row[:kbs[b]] == list(rb["idx"] + off[b])
        assert row[kbs[b]:] == [-1] * (4 - kbs[b])
        pool += list(rb["idx"] + off[b])
    rm = oracle.select(cs(A[:, pool]), m, 5, B=cs(B))
    assert list(d["idx_merge"]) == [pool[i] for i in rm["idx"]]
    np.testing.assert_allclose(d["obj_merge"], rm["obj"], rtol=1e-12)
    # equal budgets through the array give the uniform call
    d2 = oracle.select_distributed(cs(A), m, cs(B), off, 3, 5, k_blocks=[3] * 4)
    d3 = oracle.select_distributed(cs(A), m, cs(B), off, 3, 5)
    np.testing.assert_array_equal(d2["idx_block"], d3["idx_block"])
    np.testing.assert_array_equal(d2["idx_merge"], d3["idx_merge"])
    with pytest.raises(ValueError):
        oracle.select_distributed(cs(A), m, cs(B), off, 3, 5, k_blocks=[3, 3])
    with pytest.raises(RuntimeError):
        oracle.select_distributed(cs(A), m, cs(B), off, 3, 5, k_blocks=[3, 4, 3, 3])


def test_planted_rounding_mistakes_fail_a_pin():
    """Largest remainder replaced by 'the first blocks with room', and the
    width cap dropped: each breaks a pin above."""
    def first_blocks(norms2, widths, l, policy):
        tot = float(sum(norms2))
        share = [l * x / tot for x in norms2]
        out = [min(int(np.floor(s)), w) for s, w in zip(share, widths)]
        b = 0
        while sum(out) < min(l, sum(widths)):
            if out[b] < widths[b]:
                out[b] += 1
            b = (b + 1) % len(widths)
        return out

    def no_cap(norms2, widths, l, policy):
        tot = float(sum(norms2))
        share = [l * x / tot for x in norms2]
        out = [int(np.floor(s)) for s in share]
        while sum(out) < min(l, sum(widths)):
            rem = [s - o for s, o in zip(share, out)]
            out[int(np.argmax(rem))] += 1
        return out

    assert first_blocks([54.0, 12.0, 3.0], [5, 5, 5], 7, "norm") != [5, 1, 1]
    assert no_cap([54.0, 12.0, 3.0], [5, 5, 5], 7, "norm") != [5, 1, 1]
