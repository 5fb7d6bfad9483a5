"""Algorithm 4 with a budget per block (Section 5.2, the paragraph after
Algorithm 4) on the GPU: gcss_block_budgets from the context's own column
norms against the oracle's rule on the FP64 block norms, and
gcss_select_batched_budgets against the oracle's budgeted distributed
selection (per-block picks up to the first near-tie, the merge against the
oracle run on the GPU's own pool, the merge error to 1e-5), with a block of
budget zero and budgets below the largest (empty pool slots), the replayed
graph, a change of budgets, and the argument checks."""
import numpy as np
import pytest

import oracle
from oracle import budgets as bud
import synth
from tests.gpu_util import colstore32, dev, f64cs, rel, stored_dense

pytestmark = pytest.mark.gpu


def _prefix_len(a, b):
    n = 0
    for x, y in zip(a, b):
        if x != y:
            break
        n += 1
    return n


def _sep(gaps, k):
    return int(np.argmax(gaps < 1e-4)) if np.any(gaps < 1e-4) else k


def _problem(m, widths, r, seed):
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A = synth.gauss_lowrank_dense(m, n, 24, 0.05, seed=seed, scale=1 / np.sqrt(24))
    # blocks of very different weight, so the norm rule moves budgets
    wts = np.repeat(np.linspace(0.3, 2.0, len(widths)), widths)
    A = A * wts[None, :]
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    Bv = stored_dense(colstore32(Av @ synth.omega_gauss(n, r, seed=seed + 1).astype(np.float64)), m)
    return off, A32, Av, Bv


def test_norm_budgets_from_the_context_match_the_oracle(gpu):
    m, r = 200, 16
    widths = synth.block_widths(12, 40, 400, seed=21)
    off, A32, Av, Bv = _problem(m, widths, r, seed=22)
    s = gpu.Selector(dev(A32), m, k_max=4, r_max=r)
    s.set_target(dev(colstore32(Bv)))
    norms = [float(np.sum(Av[:, off[b]:off[b + 1]] ** 2)) for b in range(len(widths))]
    for l in (0, 7, 30, 61, 200, int(off[-1]) + 5):
        want = bud.budgets(norms, widths, l, "norm")
        # the context sums its own FP64 column norms: only a near-tie of two
        # remainders could round differently, and none here is that close
        tot = sum(norms)
        rem = sorted(l * x / tot - np.floor(l * x / tot) for x in norms)
        assert all(b - a > 1e-9 for a, b in zip(rem, rem[1:])) or l == 0
        got = s.block_budgets(off, l, "norm")
        assert list(got) == want, (l, list(got), want)
        assert list(s.block_budgets(off, l, "norm", norms)) == want
        assert list(s.block_budgets(off, l, "even")) == bud.budgets(norms, widths, l, "even")
        assert list(s.block_budgets(off, l, "uniform")) == bud.budgets(norms, widths, l, "uniform")
    s.close()


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_budgeted_batched_matches_oracle(gpu, dt):
    m, r, l, km = 256, 32, 40, 14
    widths = synth.block_widths(8, 150, 1500, seed=23)
    off, A32, Av, Bv = _problem(m, widths, r, seed=24)
    if dt == "f32":
        Adev, sc = dev(A32), None
    else:
        Adev, sc = gpu.quantize_tensor(dev(A32), m, "bf16")
        Av = oracle.decode_columns(oracle.quantize_bf16(A32, m), m, "bf16").T
    norms = [float(np.sum(Av[:, off[b]:off[b + 1]] ** 2)) for b in range(len(widths))]
    kbs = np.array(bud.budgets(norms, widths, l, "norm"), dtype=np.int32)
    kbs[2] = 0  # a block that selects nothing
    kmax = int(kbs.max())
    assert len(set(kbs.tolist())) > 2
    s = gpu.Selector(Adev, m, k_max=kmax, r_max=r, scales=sc, batched=(len(widths), kmax, km))
    s.set_target(dev(colstore32(Bv)))
    ib, im, om, nm, st = s.select_batched_budgets(off, kbs, km)
    assert ib.shape == (len(widths), kmax)
    ref = oracle.select_distributed(f64cs(Av), m, f64cs(Bv), off, kmax, km, k_blocks=kbs)
    for b in range(len(widths)):
        assert np.all(ib[b, kbs[b]:] == -1), b
        if kbs[b] == 0:
            continue
        rb = oracle.select(f64cs(Av[:, off[b]:off[b + 1]]), m, int(kbs[b]), B=f64cs(Bv))
        sep = _sep(rb["gap"], int(kbs[b]))
        assert _prefix_len(ib[b, :kbs[b]], ref["idx_block"][b][:kbs[b]]) >= sep, b
        assert np.all((ib[b, :kbs[b]] >= off[b]) & (ib[b, :kbs[b]] < off[b + 1]))
    pool = [int(x) for x in ib.ravel() if x >= 0]
    assert len(pool) == int(kbs.sum())
    rm = oracle.select(f64cs(Av[:, pool]), m, km, B=f64cs(Bv))
    got = _prefix_len(im, [pool[i] for i in rm["idx"]])
    assert got >= _sep(rm["gap"], km)
    np.testing.assert_allclose(om[:got + 1], rm["obj"][:got + 1], rtol=1e-5)
    e_gpu = oracle.error(f64cs(Av), m, im, B=f64cs(Bv))
    e_orc = oracle.error(f64cs(Av), m, ref["idx_merge"], B=f64cs(Bv))
    assert rel(e_gpu, e_orc) <= 1e-5
    assert rel(om[km], e_gpu) <= 1e-5
    assert nm == km and st == gpu.OK
    s.close()


def test_budgets_replay_and_change(gpu):
    m, r, km = 128, 16, 10
    widths = [700, 64, 1025, 300]
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 20, 0.1, seed=14))
    Bcs = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=15).astype(np.float64))
    s = gpu.Selector(dev(A32), m, k_max=8, r_max=r, batched=(len(widths), 8, km))
    s.set_target(dev(Bcs))
    # equal budgets through either entry point: bitwise the same
    a = s.select_batched(off, 6, km)
    b = s.select_batched_budgets(off, [6, 6, 6, 6], km)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2].view(np.int64), b[2].view(np.int64))
    # other budgets (a new graph), then the first ones again (identical)
    c = s.select_batched_budgets(off, [8, 1, 5, 2], km)
    assert np.all(c[0][1, 1:] == -1) and np.all(c[0][3, 2:] == -1)
    assert c[3] == km
    d = s.select_batched_budgets(off, [6, 6, 6, 6], km)
    assert np.array_equal(b[0], d[0]) and np.array_equal(b[1], d[1])
    assert np.array_equal(b[2].view(np.int64), d[2].view(np.int64))
    # each block's picks are its own single selection's
    for blk, kb in enumerate([8, 1, 5, 2]):
        sb = gpu.Selector(dev(np.ascontiguousarray(A32[off[blk]:off[blk + 1]])), m, k_max=kb, r_max=r)
        sb.set_target(dev(Bcs))
        i1, _, _, _ = sb.select(kb)
        assert np.array_equal(np.asarray(i1) + off[blk], c[0][blk, :kb]), blk
        sb.close()
    s.close()


def test_budget_argument_errors(gpu):
    m, r, km = 64, 8, 4
    widths = [100, 5, 60]
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 10, 0.1, seed=3))
    s = gpu.Selector(dev(A32), m, k_max=6, r_max=r, batched=(3, 6, km))
    with pytest.raises(gpu.GcssError) as e:  # norms from a context without a target
        s.block_budgets(off, 5, "norm")
    assert e.value.status == gpu.ERR_STATE
    Bcs = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=4).astype(np.float64))
    s.set_target(dev(Bcs))
    for kbs, k_merge in (([2, -1, 2], km), ([2, 6, 2], km), ([0, 0, 0], km), ([1, 1, 1], 4)):
        with pytest.raises(gpu.GcssError) as e:
            s.select_batched_budgets(off, kbs, k_merge)
        assert e.value.status == gpu.ERR_ARG, kbs
    with pytest.raises(gpu.GcssError) as e:  # col_off not ending at n
        s.block_budgets(np.array([0, 10, 20], dtype=np.int64), 5, "even")
    assert e.value.status == gpu.ERR_ARG
    # still usable after the errors
    ib, im, om, nm, st = s.select_batched_budgets(off, [3, 1, 2], km)
    assert nm == km and st == gpu.OK
    s.close()
