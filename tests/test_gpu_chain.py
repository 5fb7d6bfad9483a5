"""The per-step chain kernels (k_chain.hip) against the general column-dot /
row-update kernels (k_gemv.hip), and both against the FP64 oracle.

Both compute the same step of Theorem 4 in the q/z form (Gram-Schmidt with
one re-orthogonalisation, upsilon = B^T q, w = B upsilon, z = w - Q Q^T w)
with different summation orders, so on inputs with separated score gaps the
picks are identical and every objective agrees to FP64 rounding (1e-12 of
F_0).  GCSS_CHAIN=0 in the environment at context creation selects the
general kernels.  Shapes cover: the Gram target (B = A), explicit binary32
and bfloat16 targets, FP8 storage, a ragged m (row blocks and 32-row groups
with a tail), m = 8192 (eight row blocks, the chain's maximum), more than
512 picks (the row sums' second load round) and a target wider than 512
columns.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import colstore32, dev, f64cs, rel, stored_dense

pytestmark = pytest.mark.gpu


def _run(gpu, A, m, k, *, general, B=None, scales=None, self_target=False, r_max=0, tau=0.0):
    old = os.environ.get("GCSS_CHAIN")
    if general:
        os.environ["GCSS_CHAIN"] = "0"
    else:
        os.environ.pop("GCSS_CHAIN", None)
    try:
        s = gpu.Selector(A, m, k_max=k, r_max=r_max, self_target=self_target, scales=scales, tau=tau)
    finally:
        if old is None:
            os.environ.pop("GCSS_CHAIN", None)
        else:
            os.environ["GCSS_CHAIN"] = old
    s.set_target(B)
    idx, obj, ns, st = s.select(k)
    fl = s.flags()
    s.close()
    return np.asarray(idx), np.asarray(obj), ns, fl


def _planted(m, n, k, seed):
    """k planted columns c_j u_j (c_j = 1.05^-j, orthonormal u_j) at random
    positions over a background of 1e-4 N(0,1)/sqrt(m): the greedy picks are
    the planted columns in order, consecutive scores 10% apart and every
    planted score far above the background's."""
    return synth.planted_dense(m, n, k, 1.05, seed=seed)


def _check_pair(a, b, k):
    ia, oa, na, fa = a
    ib, ob, nb, fb = b
    assert na == nb == k
    np.testing.assert_array_equal(ia, ib)
    # F_t = F_0 minus the captured part: both orders round the captured part
    # to a few ulps of F_0, so the bound is on |F_t - F_t'| / F_0 (a small
    # F_t carries F_0's rounding relative to itself)
    for j in range(k + 1):
        assert abs(oa[j] - ob[j]) <= 1e-12 * oa[0], (j, oa[j], ob[j])
    assert fa["finished"] and fb["finished"]


@pytest.mark.parametrize("m,n,k", [(300, 2000, 40), (1025, 3000, 60), (4096, 1500, 50)])
def test_gram_target_chain_equals_general(gpu, m, n, k):
    A, pos = _planted(m, n, k, seed=m + n)
    A32 = colstore32(A)
    a = _run(gpu, dev(A32), m, k, general=False, self_target=True)
    b = _run(gpu, dev(A32), m, k, general=True, self_target=True)
    _check_pair(a, b, k)
    np.testing.assert_array_equal(a[0], pos)


@pytest.mark.parametrize("m,n,r,k,bdt", [(777, 2500, 100, 50, "f32"), (1000, 3000, 64, 60, "bf16"),
                                         (8192, 1200, 96, 40, "f32"), (1024, 1400, 32, 600, "f32"),
                                         (640, 1500, 600, 45, "bf16")])
def test_explicit_target_chain_equals_general(gpu, m, n, r, k, bdt):
    import torch
    A = synth.gauss_lowrank_dense(m, n, min(m, n) // 2, 0.05, seed=m + r)
    A32 = colstore32(A)
    Om = synth.omega_gauss(n, r, seed=r + k)
    A64 = stored_dense(A32, m)
    ldb = ((m + 63) // 64) * 64
    Bd = np.zeros((r, ldb), dtype=np.float32)
    Bd[:, :m] = (A64 @ Om.astype(np.float64)).T.astype(np.float32)
    B = dev(Bd)
    if bdt == "bf16":
        B = B.to(torch.bfloat16)
    a = _run(gpu, dev(A32), m, k, general=False, B=B, r_max=r)
    b = _run(gpu, dev(A32), m, k, general=True, B=B, r_max=r)
    # same arithmetic up to summation order: identical picks wherever the
    # oracle's score gaps are separated, objectives to FP64 rounding
    Bval = B.float().cpu().numpy()[:, :m].T.astype(np.float64)
    ref = oracle.select(f64cs(A64), m, k, B=f64cs(Bval), tau=1e-10)
    gaps = ref["gap"]
    pre = next((j for j in range(k) if gaps[j] < 1e-4), k)
    np.testing.assert_array_equal(a[0][:pre], b[0][:pre])
    np.testing.assert_array_equal(a[0][:pre], ref["idx"][:pre])
    if pre == k:
        _check_pair(a, b, k)
    else:
        for j in range(pre + 1):
            assert abs(a[1][j] - b[1][j]) <= 1e-12 * a[1][0]
    # the chain's objective is the explicit error of its picks
    e = oracle.error(f64cs(A64), m, a[0][:k], B=f64cs(Bval))
    assert rel(a[1][k], e) < 1e-5


def test_fp8_storage_chain_equals_general(gpu):
    m, n, r, k = 1500, 4000, 128, 80
    A, pos = _planted(m, n, k, seed=11)
    A32 = colstore32(A)
    codes, sc = gpu.quantize_tensor(dev(A32), m, "fp8")
    c_np, s_np = oracle.quantize_fp8(A32, m, ldo=codes.shape[1])
    Aval = oracle.decode_columns(c_np, m, "fp8", s_np).T
    Om = synth.omega_gauss(n, r, seed=5)
    ldb = ((m + 63) // 64) * 64
    Bd = np.zeros((r, ldb), dtype=np.float32)
    Bd[:, :m] = (Aval @ Om.astype(np.float64)).T.astype(np.float32)
    a = _run(gpu, codes, m, k, general=False, B=dev(Bd), scales=sc, r_max=r)
    b = _run(gpu, codes, m, k, general=True, B=dev(Bd), scales=sc, r_max=r)
    np.testing.assert_array_equal(a[0][:10], b[0][:10])
    ref = oracle.select(f64cs(Aval), m, k, B=f64cs(Bd[:, :m].T.astype(np.float64)), tau=1e-10)
    pre = next((j for j in range(k) if ref["gap"][j] < 1e-4), k)
    np.testing.assert_array_equal(a[0][:pre], ref["idx"][:pre])
    np.testing.assert_array_equal(b[0][:pre], ref["idx"][:pre])
