"""The library's per-block budgets of Algorithm 4 (gcss_block_budgets, host
code, no device needed when the norms are given) against the oracle's
budget rules (Section 5.2, after Algorithm 4): identical integers on
hand-computed and random cases, and the argument checks."""
import numpy as np
import pytest

from oracle import budgets as bud
from paper_1312_6838_amd import _abi


def _off(widths):
    return np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)


@pytest.mark.parametrize("norms,widths,l,pol", [
    ([1, 1, 1], [9, 9, 9], 7, "uniform"),
    ([1, 1, 1], [9, 1, 9], 7, "uniform"),
    ([54.0, 12.0, 3.0], [5, 5, 5], 7, "norm"),
    ([54.0, 12.0, 3.0], [9, 5, 5], 7, "norm"),
    ([1.0, 1.0, 1.0, 1.0], [5] * 4, 6, "norm"),
    ([0.0, 0.0, 0.0], [5] * 3, 4, "norm"),
    ([3.0, 1.0], [2, 3], 9, "norm"),
    ([3.0, 1.0], [2, 3], 9, "even"),
    ([1.0] * 64, [16384] * 64, 100, "even"),
])
def test_hand_cases_match_the_oracle(norms, widths, l, pol):
    got = _abi.block_budgets(None, _off(widths), l, pol, norms)
    assert list(got) == bud.budgets(norms, widths, l, pol)


def test_random_cases_match_the_oracle():
    rng = np.random.default_rng(17)
    for _ in range(400):
        c = int(rng.integers(1, 70))
        widths = [int(x) for x in rng.integers(1, 60, size=c)]
        # exact zeros, ties and wide ranges of block norms
        norms = list(np.round(rng.exponential(size=c) * (rng.random(c) > 0.2), int(rng.integers(0, 3))))
        l = int(rng.integers(0, 2 * sum(widths)))
        for pol in ("uniform", "even", "norm"):
            got = _abi.block_budgets(None, _off(widths), l, pol, norms)
            assert list(got) == bud.budgets(norms, widths, l, pol), (widths, norms, l, pol)


def test_argument_errors():
    off = _off([3, 3])
    with pytest.raises(_abi.GcssError) as e:
        _abi.block_budgets(None, off, 2, "norm", [1.0, -1.0])
    assert e.value.status == _abi.ERR_ARG
    with pytest.raises(_abi.GcssError) as e:
        _abi.block_budgets(None, off, 2, "norm", [1.0, float("nan")])
    assert e.value.status == _abi.ERR_ARG
    with pytest.raises(_abi.GcssError) as e:
        _abi.block_budgets(None, off, 2, "norm", None)  # norms from a context, but no context
    assert e.value.status == _abi.ERR_ARG
    with pytest.raises(_abi.GcssError) as e:
        _abi.block_budgets(None, np.array([0, 3, 3], dtype=np.int64), 2, "even", None)
    assert e.value.status == _abi.ERR_ARG
    with pytest.raises(_abi.GcssError) as e:
        _abi.block_budgets(None, np.array([1, 3], dtype=np.int64), 2, "even", None)
    assert e.value.status == _abi.ERR_ARG
    with pytest.raises(_abi.GcssError) as e:
        _abi.block_budgets(None, off, -1, "even", None)
    assert e.value.status == _abi.ERR_ARG
    # an unknown policy code goes through the C check too
    out = np.zeros(2, dtype=np.int32)
    st = _abi.load().gcss_block_budgets(None, 2, off.ctypes.data, None, 2, 7, out.ctypes.data)
    assert st == _abi.ERR_ARG
