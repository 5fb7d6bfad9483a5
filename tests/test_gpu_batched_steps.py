"""The three ways Algorithm 4's block phase can run its per-step work, on
the same inputs: one workgroup per block (k_chain_block), the six chain
kernels with the blocks along gridDim.z, and the general column-dot /
row-update kernels (GCSS_BATCH_STEP=block / chain / general at context
creation).  The arithmetic is the same up to summation order, so on inputs
with separated score gaps the picks are identical and the objectives agree
to FP64 rounding of F_0; all three match the oracle's Algorithm 4.  Also the
basis check's reject branch under the per-block kernel."""
import os

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import colstore32, dev, f64cs, rel, stored_dense
from tests.test_gpu_ties_rejects import TAU, _reject_case

pytestmark = pytest.mark.gpu

MODES = ("block", "chain", "general")


def _sel(gpu, mode, *a, **kw):
    old = os.environ.get("GCSS_BATCH_STEP")
    os.environ["GCSS_BATCH_STEP"] = mode
    try:
        return gpu.Selector(*a, **kw)
    finally:
        if old is None:
            os.environ.pop("GCSS_BATCH_STEP", None)
        else:
            os.environ["GCSS_BATCH_STEP"] = old


def _prefix_len(a, b):
    n = 0
    for x, y in zip(a, b):
        if x != y:
            break
        n += 1
    return n


@pytest.mark.parametrize("m,bdt", [(256, "f32"), (1024, "bf16"), (2048, "f32")])
def test_batched_step_modes_agree(gpu, m, bdt):
    import torch
    r, km, nb = 48, 24, 20
    widths = synth.block_widths(nb, 60, 400, seed=m)
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A = synth.gauss_lowrank_dense(m, n, 40, 0.05, seed=m + 1, scale=1 / np.sqrt(40))
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    Bd = colstore32(Av @ synth.omega_gauss(n, r, seed=m + 2).astype(np.float64))
    B = dev(Bd)
    if bdt == "bf16":
        B = B.to(torch.bfloat16)
    Bv = B.float().cpu().numpy()[:, :m].T.astype(np.float64)
    kbs = np.array([6, 3, 0, 6, 5, 1, 6, 2, 4, 6, 6, 0, 3, 6, 5, 6, 1, 6, 4, 6], dtype=np.int32)
    out = {}
    for mode in MODES:
        s = _sel(gpu, mode, dev(A32), m, k_max=6, r_max=r, batched=(nb, 6, km))
        s.set_target(B)
        out[mode] = s.select_batched_budgets(off, kbs, km)
        s.close()
    ib0, im0, om0, nm0, st0 = out["block"]
    for mode in MODES[1:]:
        ib, im, om, nm, st = out[mode]
        assert np.array_equal(ib, ib0), mode
        assert np.array_equal(im, im0) and nm == nm0 == km, mode
        assert np.max(np.abs(om - om0)) <= 1e-12 * om0[0], mode
    ref = oracle.select_distributed(f64cs(Av), m, f64cs(Bv), off, 6, km, k_blocks=kbs)
    for b in range(nb):
        if kbs[b] == 0:
            assert np.all(ib0[b] == -1)
            continue
        rb = oracle.select(f64cs(Av[:, off[b]:off[b + 1]]), m, int(kbs[b]), B=f64cs(Bv))
        sep = int(np.argmax(rb["gap"] < 1e-4)) if np.any(rb["gap"] < 1e-4) else int(kbs[b])
        assert _prefix_len(ib0[b, :kbs[b]], ref["idx_block"][b][:kbs[b]]) >= sep, b
    e_gpu = oracle.error(f64cs(Av), m, im0, B=f64cs(Bv))
    e_orc = oracle.error(f64cs(Av), m, ref["idx_merge"], B=f64cs(Bv))
    assert rel(e_gpu, e_orc) <= 1e-5


def test_batched_rejections_per_block_kernel(gpu):
    m, r, kb, km = 2048, 16, 6, 8
    A, B, near, planted = _reject_case(m=m)
    n = A.shape[1]
    # 16 blocks, so that the per-block kernel is also the automatic choice
    off = np.concatenate([[0, 1000], np.linspace(1000, n, 16)[1:].astype(np.int64)]).astype(np.int64)
    nb = off.size - 1
    A32, B32 = colstore32(A), colstore32(B)
    Av, Bv = stored_dense(A32, m), stored_dense(B32, m)
    ref = oracle.select_distributed(f64cs(Av), m, f64cs(Bv), off, kb, km, tau=TAU)
    res = {}
    for mode in ("block", "chain"):
        s = _sel(gpu, mode, dev(A32), m, k_max=kb, r_max=r, tau=TAU, batched=(nb, kb, km))
        s.set_target(dev(B32))
        res[mode] = s.select_batched(off, kb, km)
        s.close()
    ib, im, om, nm, st = res["block"]
    assert st == gpu.OK and nm == km and np.all(ib >= 0)
    # the blocks without near copies pick the same columns under both; in the
    # near copies' blocks only the number of rejected picks may differ
    for b in range(nb):
        if not any(off[b] <= j < off[b + 1] for j in near):
            assert np.array_equal(ib[b], res["chain"][0][b]), b
    assert np.array_equal(im, res["chain"][1])
    assert list(im) == list(ref["idx_merge"])
    e_gpu = oracle.error(f64cs(Av), m, im, B=f64cs(Bv))
    assert rel(e_gpu, oracle.error(f64cs(Av), m, ref["idx_merge"], B=f64cs(Bv))) <= 1e-5
