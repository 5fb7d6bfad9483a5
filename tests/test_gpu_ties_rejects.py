"""GPU vs oracle on the two places where the paper is silent about numerics in
the argmax step of Algorithms 1, 3 and 4:

* ties: exactly equal scores (duplicate columns, bitwise equal on both
  sides) go to the lowest column index, and in the merge of Algorithm 4 to
  the lowest pooled position;
* rejected picks: a column that only rounding keeps a candidate (its FP64
  residual after re-orthogonalisation is at most tau times its squared
  norm) is dropped when picked and the search is repeated, without costing
  a pick; the oracle, whose FP64 scores see the dependence directly, never
  offers it.  The selection still delivers its k picks, also when more
  picks are rejected than the captured loops have spare steps.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import colstore32, dev, f64cs, rel, stored_dense

pytestmark = pytest.mark.gpu


def _quantized(gpu, A32, m, dt):
    if dt == "f32":
        return dev(A32), None, stored_dense(A32, m)
    Adev, sc = gpu.quantize_tensor(dev(A32), m, dt)
    if dt == "bf16":
        return Adev, sc, oracle.decode_columns(oracle.quantize_bf16(A32, m), m, "bf16").T
    codes, scl = oracle.quantize_fp8(A32, m)
    return Adev, sc, oracle.decode_columns(codes, m, "fp8", scl).T


@pytest.mark.parametrize("target", ["self", "proj"])
@pytest.mark.parametrize("dt", ["f32", "bf16", "fp8"])
def test_duplicate_best_columns_lowest_index_wins(gpu, target, dt):
    m, n, k = 256, 3000, 8
    A, pos = synth.planted_dense(m, n, k, 1.5, seed=5)
    j0 = int(pos[0])
    lo, hi = (0, n - 2) if j0 != 0 else (1, n - 2)
    assert lo < j0 < hi and lo not in pos and hi not in pos
    A[:, lo] = A[:, j0]
    A[:, hi] = A[:, j0]
    Adev, sc, Av = _quantized(gpu, colstore32(A), m, dt)
    if target == "self":
        s = gpu.Selector(Adev, m, k_max=k, self_target=True, scales=sc)
        s.set_target(None)
        ref = oracle.select(f64cs(Av), m, k)
    else:
        Bv = stored_dense(colstore32(Av @ synth.omega_gauss(n, 256, seed=9).astype(np.float64)), m)
        s = gpu.Selector(Adev, m, k_max=k, r_max=256, scales=sc)
        s.set_target(dev(colstore32(Bv)))
        ref = oracle.select(f64cs(Av), m, k, B=f64cs(Bv))
    idx, obj, ns, st = s.select(k)
    # the three copies tie exactly at the top; every later step is separated
    assert ref["idx"][0] == lo and np.min(ref["gap"][1:]) > 1e-3
    assert list(idx) == list(ref["idx"])
    assert j0 not in idx and hi not in idx
    np.testing.assert_allclose(obj, ref["obj"], rtol=1e-5)
    s.close()


# ---- rejected picks -----------------------------------------------------------
TAU = 1e-8


def _reject_case(m=4096, n=2000, r=16, seed=3):
    """Explicit target B = X diag(sqrt(s2)) Y^T with known left singular
    vectors X.  Column 10 is v = 3 (x1 + x2)/sqrt(2) (the best candidate) and
    column 1005 an exact copy of it; columns 1100..1139 are near copies
    c_j (v - 3e-5 w + 1e-6 noise) with w = (x1 - x2)/sqrt(2): their exact
    residual after v is about 9e-10 of their squared norm (below TAU), while
    the binary32 rounding of the dot products that track it is a few 1e-8 of
    it, so some of them stay candidates after v is picked, with scores of
    rounding noise over rounding noise; their first-step score is 2e-5 below
    v's.  The scales c_j (spread over [1.5, 4.5]; a score does not depend on
    a column's scale) give each copy its own rounding, so the sign of the
    noise is not shared by all of them whatever the summation order.  Ten
    more columns are x3 .. x12 (scores s2[2..11], 25% apart) over a 1e-3
    noise background."""
    rng = np.random.default_rng(seed)
    X, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Y, _ = np.linalg.qr(rng.standard_normal((r, r)))
    s2 = np.array([2.0, 1.0] + [0.8 * 0.75 ** j for j in range(r - 2)])
    B = X @ np.diag(np.sqrt(s2)) @ Y.T
    v = (X[:, 0] + X[:, 1]) / math.sqrt(2)
    w = (X[:, 0] - X[:, 1]) / math.sqrt(2)
    A = 1e-3 * rng.standard_normal((m, n)) / math.sqrt(m)
    A[:, 10] = 3.0 * v
    A[:, 1005] = 3.0 * v
    near = list(range(1100, 1140))
    for j in near:
        A[:, j] = rng.uniform(1.5, 4.5) * (v - 3e-5 * w + 1e-6 * rng.standard_normal(m) / math.sqrt(m))
    planted = [50, 120, 300, 777, 900, 1010, 1200, 1500, 1700, 1900]
    for t, j in enumerate(planted):
        A[:, j] = X[:, 2 + t]
    return A, B, near, planted


def test_rejected_picks_match_oracle_and_never_truncate(gpu):
    m, k, r = 4096, 10, 16
    A, B, near, planted = _reject_case()
    n = A.shape[1]
    A32, B32 = colstore32(A), colstore32(B)
    Av, Bv = stored_dense(A32, m), stored_dense(B32, m)
    ref = oracle.select(f64cs(Av), m, k, B=f64cs(Bv), tau=TAU)
    assert list(ref["idx"]) == [10] + planted[:k - 1]
    # step 1 is the exact tie of v and its copy; every later step is separated
    assert ref["gap"][0] == 0.0 and np.min(ref["gap"][1:]) > 1e-4
    s = gpu.Selector(dev(A32), m, k_max=k, r_max=r, tau=TAU)
    s.set_target(dev(B32))
    idx, obj, ns, st = s.select(k)
    fl = s.flags()
    print(f"rejected picks: {fl['rejected']}")
    assert fl["rejected"] > 0, "the construction did not reach the basis check's reject branch"
    assert ns == k and st == gpu.OK and fl["finished"] and not fl["exhausted"]
    assert list(idx) == list(ref["idx"])
    assert not set(idx.tolist()) & set(near + [1005])
    np.testing.assert_allclose(obj, ref["obj"], rtol=1e-5)
    # the captured loop: the same picks, or (more rejections than its spare
    # steps) an unfinished selection that says so
    d_idx, d_obj, d_ns = s.select_async(k)
    fa = s.flags()
    na = int(d_ns.cpu()[0])
    if fa["finished"]:
        assert na == k and np.array_equal(d_idx.cpu().numpy(), idx)
        assert np.array_equal(d_obj.cpu().numpy().view(np.int64), obj.view(np.int64))
    else:
        assert na < k and fa["rejected"] >= gpu.ASYNC_SPARE_STEPS
        assert list(d_idx.cpu().numpy()[:na]) == list(idx[:na])
    s.close()


def test_batched_rejections_and_merge_tie(gpu):
    m, r, kb, km = 4096, 16, 6, 8
    A, B, near, planted = _reject_case()
    n = A.shape[1]
    off = np.array([0, 1000, n], dtype=np.int64)
    A32, B32 = colstore32(A), colstore32(B)
    Av, Bv = stored_dense(A32, m), stored_dense(B32, m)
    ref = oracle.select_distributed(f64cs(Av), m, f64cs(Bv), off, kb, km, tau=TAU)
    want_blocks = [[10] + planted[:5], [1005] + planted[5:]]
    assert ref["idx_block"].tolist() == want_blocks
    # the merge pool holds v twice (positions 0 and 6): the lower position wins
    assert list(ref["idx_merge"]) == [10] + planted[:km - 1]
    s = gpu.Selector(dev(A32), m, k_max=kb, r_max=r, tau=TAU, batched=(2, kb, km))
    s.set_target(dev(B32))
    ib, im, om, nm, st = s.select_batched(off, kb, km)
    assert st == gpu.OK and nm == km
    assert ib.tolist() == want_blocks
    assert list(im) == list(ref["idx_merge"])
    np.testing.assert_allclose(om, ref["obj_merge"], rtol=1e-5)
    e_gpu = oracle.error(f64cs(Av), m, im, B=f64cs(Bv))
    assert rel(e_gpu, oracle.error(f64cs(Av), m, ref["idx_merge"], B=f64cs(Bv))) <= 1e-5
    s.close()
