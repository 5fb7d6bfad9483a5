"""Edge cases of the random sign targets, the embedding outputs and the
eigensolver: single columns, single targets, empty draws, the largest
eigenproblem (l = 2048), blocks as wide as the matrix."""
import math

import numpy as np
import pytest

import oracle
from oracle import embed, quality, rng
import synth
from tests.gpu_util import colstore32, dev, f64cs, stored_dense

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,r,d", [(5, 1, 1, 1.0), (5, 1, 1, 0.5), (37, 3, 2, 1.0), (64, 100, 1, 0.01),
                                     (300, 2000, 7, 1e-9)])
def test_sign_projection_tiny_and_empty(gpu, m, n, r, d):
    A32 = colstore32(np.random.default_rng(m + n).standard_normal((m, n)))
    Av = stored_dense(A32, m)
    s = gpu.Selector(dev(A32), m, k_max=1, r_max=r)
    B = s.project_sign(99, r, density=d).cpu().numpy()[:, :m].T.astype(np.float64)
    Om = rng.omega_rows(0, n, r, 99, d)
    Bref = Av @ Om
    if not np.any(Om):
        assert np.all(B == 0.0)                 # nothing drawn: B is exactly zero
    scale = np.sqrt(np.sum(Av ** 2, axis=1))[:, None] * np.maximum(np.sqrt(np.sum(Om ** 2, axis=0)), 1.0)
    assert np.max(np.abs(B - Bref) / scale) < 1e-6


def test_rank_one_everything(gpu):
    """One pick: W is one row, R is 1 x 1, the rank-1 approximation is the
    projection on that column, and the eigensolver with a block of one."""
    import torch
    m, n = 50, 80
    A = synth.gauss_lowrank_dense(m, n, 5, 0.1, seed=4)
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    s = gpu.Selector(dev(A32), m, k_max=1, self_target=True)
    s.set_target(None)
    W = torch.zeros(1, n, dtype=torch.float32, device="cuda")
    s.set_embedding(W)
    idx, obj, ns, st = s.select(1)
    p = int(idx[0])
    R = gpu.qless_r_tensor(W, n, torch.from_numpy(idx).cuda()).cpu().numpy()
    assert abs(R[0, 0] - np.linalg.norm(Av[:, p])) <= 1e-5 * np.linalg.norm(Av[:, p])
    U, sig, V, err = s.rank_k(1, 1)
    ref = embed.rank_k(Av, [p], 1)
    assert abs(sig[0] - ref["sigma"][0]) <= 1e-6 * ref["sigma"][0]
    assert abs(err - ref["err"]) <= 1e-5 * ref["err"]
    lam, Ue, it, ch = s.top_eig(1, s=1, max_iters=60, tol=1e-12)
    lr, _ = quality.top_eig(Av, 1)
    # a block of one is the power method: converged to 1e-6 of lambda_1
    assert abs(lam[0] - lr[0]) <= 1e-4 * lr[0]


def test_rank_k_largest_eigenproblem(gpu):
    """l = 2048 picks, the largest the eigen-decomposition takes (64 Jacobi
    blocks, L = 2048 exactly)."""
    m, n, l = 2100, 2600, 2048
    A = np.random.default_rng(5).standard_normal((m, n)) * (0.999 ** np.arange(n))[None, :]
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    import torch
    s = gpu.Selector(dev(A32), m, k_max=l, self_target=True, tau=1e-12)
    s.set_target(None)
    W = torch.zeros(l, n, dtype=torch.float32, device="cuda")
    s.set_embedding(W)
    idx, obj, ns, st = s.select(l)
    assert ns == l
    U, sig, V, err = s.rank_k(l, 50, want_v=False)
    Wh = W.double().cpu().numpy()
    sw = np.linalg.svd(Wh, compute_uv=False)
    assert np.max(np.abs(sig - sw[:50])) <= 1e-9 * sw[0]
    assert abs(err - (obj[l] + np.sum(sw[50:] ** 2))) <= 1e-6 * np.sum(Av * Av)


def test_top_eig_full_block(gpu):
    """s = m: the block spans the whole space, so one Rayleigh-Ritz step is
    exact (to the binary32 Gram matrix)."""
    m, n = 96, 700
    A = synth.gauss_lowrank_dense(m, n, 30, 0.2, seed=6)
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    s = gpu.Selector(dev(A32), m, k_max=m, self_target=True)
    s.set_target(None)
    lam, U, it, ch = s.top_eig(m, s=m, max_iters=4, tol=0.0)
    lr = np.linalg.eigvalsh(Av @ Av.T)[::-1]
    assert np.max(np.abs(lam - lr)) <= 1e-6 * lr[0]
