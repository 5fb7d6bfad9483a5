"""Naive distributed selection on the GPU (per-block self-target contexts
over views of A, the pooled columns gathered by the library, a second
selection over them) against the oracle's composition of Algorithm 1."""
import numpy as np
import pytest

import oracle
from oracle import naive
import synth
from tests.gpu_util import colstore32, dev, f64cs, stored_dense

pytestmark = pytest.mark.gpu


def _prefix(a, b):
    n = 0
    for x, y in zip(a, b):
        if x != y:
            break
        n += 1
    return n


@pytest.mark.parametrize("policy", ["uniform", "adaptive"])
def test_naive_matches_oracle(gpu, policy):
    from paper_1312_6838_amd import distributed
    m = 128
    rng = np.random.default_rng(4)
    widths = [700, 1300, 400, 900]
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    blocks = []
    for b, w in enumerate(widths):
        # 12 planted columns per block: every budget stays within them, so
        # the picks are separated (beyond them only background noise is left,
        # whose order binary32 scores cannot resolve)
        Ab, _ = synth.planted_dense(m, w, 12, 1.5 + 0.5 * b, seed=10 + b)
        blocks.append(Ab * (1.0 + b))
    A = np.hstack(blocks)
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    r = distributed.naive_select(dev(A32), m, off, 16, k_merge=8, policy=policy)
    ro = naive.naive_select(Av, list(off), 16, k_merge=8, policy=policy)
    assert list(r["budgets"]) == list(ro["budgets"])
    for b in range(len(widths)):
        Ab = Av[:, off[b]:off[b + 1]]
        ref = oracle.select(f64cs(Ab), m, int(ro["budgets"][b]))
        sep = int(np.argmax(ref["gap"] < 1e-4)) if np.any(ref["gap"] < 1e-4) else len(ref["gap"])
        assert _prefix(r["idx_block"][b], ro["idx_block"][b]) >= sep, b
        np.testing.assert_allclose(r["obj_block"][b], ro["obj_block"][b], rtol=1e-5)
    assert max(ro["budgets"]) <= 12
    if np.array_equal(r["pool"], ro["pool"]):
        refm = oracle.select(f64cs(Av[:, ro["pool"]]), m, 8)
        sep = int(np.argmax(refm["gap"] < 1e-4)) if np.any(refm["gap"] < 1e-4) else 8
        assert _prefix(r["idx_merge"], ro["idx_merge"]) >= sep
        np.testing.assert_allclose(r["obj_merge"][:sep + 1], ro["obj_merge"][:sep + 1], rtol=1e-5)


def test_gather_columns(gpu):
    import torch
    m, n = 70, 300
    A32 = colstore32(np.random.default_rng(1).standard_normal((m, n)))
    s = gpu.Selector(dev(A32), m, k_max=2, self_target=True)
    idx = np.array([5, 0, 299, 5, 1000, -1], dtype=np.int64)
    P, _ = s.gather(idx)
    Ph = P.cpu().numpy()
    assert np.array_equal(Ph[:4], A32[[5, 0, 299, 5]])
    assert np.all(Ph[4:] == 0.0)                      # out of range: zero columns
    A8, sc = gpu.quantize_tensor(dev(A32), m, "fp8")
    s8 = gpu.Selector(A8, m, k_max=2, self_target=True, scales=sc)
    P8, S8 = s8.gather(idx[:3])
    assert torch.equal(P8, A8[[5, 0, 299]]) and torch.equal(S8, sc[[5, 0, 299]])
