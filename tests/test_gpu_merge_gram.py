"""The merge of Algorithm 4 over a small pool in the Gram form of Algorithm
3 (k_merge.hip: G = A0^T A0 and H = A0^T B in FP64, then one launch per
step), against the oracle run on the GPU's own pool and against the merge
over a sub-context (GCSS_MERGE=sub, the streaming path).  The Gram form is
FP64 from the stored values on, like the oracle, so its picks follow the
oracle's up to near-ties of 1e-9 and its objectives agree to 1e-9 of F_0;
the streaming merge, binary32 in its dot products, agrees to its own 1e-5."""
import os

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import colstore32, dev, f64cs, rel, stored_dense

pytestmark = pytest.mark.gpu


def _sel(gpu, merge, *a, **kw):
    old = os.environ.get("GCSS_MERGE")
    if merge == "sub":
        os.environ["GCSS_MERGE"] = "sub"
    else:
        os.environ.pop("GCSS_MERGE", None)
    try:
        return gpu.Selector(*a, **kw)
    finally:
        if old is None:
            os.environ.pop("GCSS_MERGE", None)
        else:
            os.environ["GCSS_MERGE"] = old


def _values(gpu, A32, m, dt):
    if dt == "f32":
        return dev(A32), None, stored_dense(A32, m)
    Adev, sc = gpu.quantize_tensor(dev(A32), m, dt)
    if dt == "bf16":
        return Adev, sc, oracle.decode_columns(oracle.quantize_bf16(A32, m), m, "bf16").T
    codes, scl = oracle.quantize_fp8(A32, m)
    return Adev, sc, oracle.decode_columns(codes, m, "fp8", scl).T


def _prefix_len(a, b):
    n = 0
    for x, y in zip(a, b):
        if x != y:
            break
        n += 1
    return n


@pytest.mark.parametrize("dt", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("m,nb,kb,km,r", [(256, 8, 5, 30, 32), (1000, 20, 12, 100, 100)])
def test_gram_merge_matches_oracle_on_its_pool(gpu, dt, m, nb, kb, km, r):
    widths = synth.block_widths(nb, 100, 900, seed=m + nb)
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A = synth.gauss_lowrank_dense(m, n, 60, 0.05, seed=m + 3, scale=1 / np.sqrt(60))
    A32 = colstore32(A)
    Adev, sc, Av = _values(gpu, A32, m, dt)
    Bv = stored_dense(colstore32(Av @ synth.omega_gauss(n, r, seed=m + 4).astype(np.float64)), m)
    res = {}
    for merge in ("gram", "sub"):
        s = _sel(gpu, merge, Adev, m, k_max=kb, r_max=r, scales=sc, batched=(nb, kb, km))
        s.set_target(dev(colstore32(Bv)))
        res[merge] = s.select_batched(off, kb, km)
        s.close()
    ib, im, om, nm, st = res["gram"]
    assert st == gpu.OK and nm == km
    assert np.array_equal(ib, res["sub"][0])  # same block phase
    pool = [int(x) for x in ib.ravel() if x >= 0]
    ref = oracle.select(f64cs(Av[:, pool]), m, km, B=f64cs(Bv))
    want = [pool[i] for i in ref["idx"]]
    sep = int(np.argmax(ref["gap"] < 1e-9)) if np.any(ref["gap"] < 1e-9) else km
    got = _prefix_len(im, want)
    assert got >= sep, (got, sep)
    assert np.max(np.abs(om[:got + 1] - ref["obj"][:got + 1])) <= 1e-9 * ref["obj"][0]
    # the streaming merge (binary32 dot products) follows for the first steps
    assert _prefix_len(res["sub"][1], im) >= min(sep, 20)
    e_gram = oracle.error(f64cs(Av), m, im, B=f64cs(Bv))
    assert rel(om[km], e_gram) <= 1e-9


def test_gram_merge_exhausts_a_small_pool(gpu):
    """A pool of rank 3 (every block picks from the same three directions):
    the merge stops after the pool's rank with the exhaustion status."""
    m, r, nb, kb, km = 128, 8, 4, 2, 6
    rng = np.random.default_rng(7)
    X = np.linalg.qr(rng.standard_normal((m, 3)))[0]
    n = 400
    coef = rng.standard_normal((3, n))
    A = X @ coef
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    off = np.array([0, 100, 200, 300, 400], dtype=np.int64)
    Bv = stored_dense(colstore32(Av @ rng.standard_normal((n, r))), m)
    s = gpu.Selector(dev(A32), m, k_max=kb, r_max=r, tau=1e-6, batched=(nb, kb, km))
    s.set_target(dev(colstore32(Bv)))
    ib, im, om, nm, st = s.select_batched(off, kb, km)
    s.close()
    assert nm == 3 and st == gpu.WARN_EXHAUSTED, (nm, st, im)
    assert np.all(im[3:] == -1)
    pool = [int(x) for x in ib.ravel() if x >= 0]
    ref = oracle.select(f64cs(Av[:, pool]), m, km, B=f64cs(Bv), tau=1e-6)
    # the third pick is a tie of every remaining column (each completes the
    # span), so only the first two are compared; after three the error is 0
    assert [pool[i] for i in ref["idx"][:2]] == list(im[:2])
    assert ref["n_selected"] == 3
    assert abs(om[3]) <= 1e-9 * om[0]
    assert oracle.error(f64cs(Av), m, im[:3], B=f64cs(Bv)) <= 1e-9 * om[0]
