"""Event timing of the streaming passes (gcss_set_profiling / gcss_get_profile,
which bench.py's roofline reads): a profiled selection gives the same picks
and objectives as a replayed one, and counts exactly the passes that read A
-- k - 1 for an explicit target (none follows the last pick), k for B = A
(the last pass returns the last pick's exact decrease), k_block - 1 per
batched selection -- each with a plausible duration."""
import numpy as np
import pytest

import synth
from tests.gpu_util import colstore32, dev, stored_dense

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("target", ["explicit", "self"])
def test_profiled_select_counts_the_passes_over_a(gpu, target):
    m, n, k, r = 512, 20000, 12, 64
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 40, 0.05, seed=31))
    if target == "self":
        s = gpu.Selector(dev(A32), m, k_max=k, self_target=True)
        s.set_target(None)
    else:
        Bcs = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=32).astype(np.float64))
        s = gpu.Selector(dev(A32), m, k_max=k, r_max=r)
        s.set_target(dev(Bcs))
    i0, o0, n0, _ = s.select(k)
    s.profile(True)
    i1, o1, n1, _ = s.select(k)
    i2, o2, n2, _ = s.select(k)
    prof = s.profile()
    s.profile(False)
    s.close()
    assert n0 == n1 == n2 == k
    assert np.array_equal(i0, i1) and np.array_equal(i0, i2)
    assert np.array_equal(o1.view(np.int64), o2.view(np.int64))
    want = (k if target == "self" else k - 1) * 2
    assert prof["selects"] == 2 and prof["stream_launches"] == want, prof
    per = prof["stream_ms"] / prof["stream_launches"]
    # a pass over 20000 columns of 512 binary32 values (41 MB): tens of us
    assert 1e-3 < per < 1.0, per
    assert prof["loop_ms"] > prof["stream_ms"]


def test_profiled_batched_counts_the_passes_over_a(gpu):
    m, r, kb, km = 256, 16, 6, 10
    widths = [3000, 2000, 4000, 2500]
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 20, 0.1, seed=33))
    Bcs = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=34).astype(np.float64))
    s = gpu.Selector(dev(A32), m, k_max=kb, r_max=r, batched=(len(widths), kb, km))
    s.set_target(dev(Bcs))
    a = s.select_batched(off, kb, km)
    s.profile(True)
    b = s.select_batched(off, kb, km)
    prof = s.profile()
    s.profile(False)
    s.close()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert prof["selects"] == 1 and prof["stream_launches"] == kb - 1, prof
    assert prof["stream_ms"] > 0.0
