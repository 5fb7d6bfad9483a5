"""Embedding W = Q^T A (Section 3, Eq. CSS_LowDim) and the Q-less R factor
(Section 6) from the GPU's streaming passes, against the oracle's omega rows.

Tolerance: each entry is one dot product A_i . q_t formed in binary32 (the
Gram-target passes form it in FP64) over m terms and stored in binary32, so
|W_gpu - W_ref| <= 1e-5 * ||A_i|| (about sqrt(m) * 2^-24 with a wide margin
for m <= a few thousand); the bases themselves agree to ~1e-14.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import embed
from tests.gpu_util import colstore32, dev, f64cs, stored_dense

pytestmark = pytest.mark.gpu


def _values(gpu, A32, m, dt):
    if dt == "f32":
        return dev(A32), None, stored_dense(A32, m)
    Adev, sc = gpu.quantize_tensor(dev(A32), m, dt)
    if dt == "bf16":
        return Adev, sc, oracle.decode_columns(oracle.quantize_bf16(A32, m), m, "bf16").T
    codes, scl = oracle.quantize_fp8(A32, m)
    return Adev, sc, oracle.decode_columns(codes, m, "fp8", scl).T


def _embedding(k, n, ldw=None, fill=7.0):
    import torch
    ldw = ldw or n + 5
    return torch.full((k, ldw), fill, dtype=torch.float32, device="cuda")


def _check_w(W, Wref, Aval, tol=1e-5):
    norms = np.sqrt(np.sum(Aval * Aval, axis=0))
    err = np.abs(W - Wref) / np.maximum(norms, 1e-300)[None, :]
    t, i = np.unravel_index(int(np.argmax(err)), err.shape)
    assert err[t, i] <= tol, (t, i, W[t, i], Wref[t, i])


@pytest.mark.parametrize("target", ["self", "proj"])
@pytest.mark.parametrize("dt", ["f32", "bf16", "fp8"])
def test_embedding_matches_oracle_omega(gpu, target, dt):
    m, n, k = 256, 3000, 12
    A, _ = synth.planted_dense(m, n, k, 1.5, seed=5)
    A32 = colstore32(A)
    Adev, sc, Aval = _values(gpu, A32, m, dt)
    if target == "self":
        s = gpu.Selector(Adev, m, k_max=k, self_target=True, scales=sc)
        s.set_target(None)
        ref = oracle.select(f64cs(Aval), m, k, omega=True)
    else:
        Bv = stored_dense(colstore32(Aval @ synth.omega_gauss(n, 96, seed=9).astype(np.float64)), m)
        s = gpu.Selector(Adev, m, k_max=k, r_max=96, scales=sc)
        s.set_target(dev(colstore32(Bv)))
        ref = oracle.select(f64cs(Aval), m, k, B=f64cs(Bv), omega=True)
    Wt = _embedding(k, n)
    s.set_embedding(Wt)
    idx, obj, ns, st = s.select(k)
    assert ns == k and list(idx) == list(ref["idx"])
    W = Wt.cpu().numpy()
    assert np.all(W[:, n:] == 7.0)           # padding of each row untouched
    _check_w(W[:, :n].astype(np.float64), ref["omega"], Aval)
    # Q-less R: A_S = Q R with R = W[:, S] upper triangular
    import torch
    R = gpu.qless_r_tensor(Wt, n, torch.from_numpy(idx).cuda()).cpu().numpy().astype(np.float64)
    Rref = ref["omega"][:, idx]
    assert np.all(np.tril(R, -1) == 0.0)
    nS = np.sqrt(np.sum(Aval[:, idx] ** 2, axis=0))
    assert np.max(np.abs(np.triu(R) - np.triu(Rref)) / nS[None, :]) <= 1e-5
    assert np.all(np.diag(R) > 0)
    # what W keeps below the diagonal is rounding residue
    assert np.max(np.abs(np.tril(W[:, idx], -1)) / nS[None, :]) <= 1e-5


@pytest.mark.parametrize("case", ["css_500x1000", "ragged_333x4097_r7"])
def test_embedding_rows_and_decrease(gpu, case):
    """Row t of W holds A^T q_{t+1}; for B = A its squared norm is the
    objective's decrease at that step."""
    if case == "css_500x1000":
        m, n, k, r = 500, 1000, 20, 0
        A = synth.gauss_lowrank_dense(m, n, 50, 0.01, seed=0)
    else:
        m, n, k, r = 333, 4097, 25, 7
        A = synth.gauss_lowrank_dense(m, n, 40, 0.1, seed=2)
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    if r == 0:
        s = gpu.Selector(dev(A32), m, k_max=k, self_target=True)
        s.set_target(None)
    else:
        Bv = stored_dense(colstore32(Av @ synth.omega_gauss(n, r, seed=3).astype(np.float64)), m)
        s = gpu.Selector(dev(A32), m, k_max=k, r_max=r)
        s.set_target(dev(colstore32(Bv)))
    Wt = _embedding(k, n, ldw=n)
    s.set_embedding(Wt)
    idx, obj, ns, st = s.select(k)
    assert ns == k
    W = Wt.cpu().numpy().astype(np.float64)
    Q = s.read(gpu.STATE_Q, m * k, np.float64).reshape(k, m).T
    _check_w(W, Q.T @ Av, Av)
    if r == 0:
        dec = np.sum(W * W, axis=1)
        np.testing.assert_allclose(dec, obj[:-1] - obj[1:], rtol=1e-4, atol=1e-6 * obj[0])


def test_embedding_leaves_selection_unchanged_and_async(gpu):
    """Writing W changes no pick and no objective bit; the graph-replayed loop
    writes the same W; turning it off stops the writes."""
    m, n, k, r = 700, 5000, 30, 64
    A = synth.spectral_lowrank_dense(m, n, 100, 0.5, 1e-3, seed=4)
    A32 = colstore32(A)
    B = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=5).astype(np.float64))
    s = gpu.Selector(dev(A32), m, k_max=k, r_max=r)
    s.set_target(dev(B))
    i0, o0, _, _ = s.select(k)
    W1 = _embedding(k, n)
    s.set_embedding(W1)
    i1, o1, _, _ = s.select(k)
    assert np.array_equal(i0, i1) and np.array_equal(o0.view(np.int64), o1.view(np.int64))
    W2 = _embedding(k, n, fill=-3.0)
    s.set_embedding(W2)
    d_idx, d_obj, _ = s.select_async(k)
    assert np.array_equal(d_idx.cpu().numpy(), i0)
    assert np.array_equal(W1[:, :n].cpu().numpy(), W2[:, :n].cpu().numpy())
    s.set_embedding(None)
    W2.fill_(-3.0)
    s.select(k)
    s.select_async(k)
    import torch
    torch.cuda.synchronize()
    assert bool(torch.all(W2 == -3.0))


def test_embedding_on_exhaustion(gpu):
    """Exactly rank-5 data: 5 picks, 5 rows written, the rest untouched; the
    rows reproduce A = Q W exactly (to rounding)."""
    m, n, rank = 40, 100, 5
    A = synth.int_lowrank_dense(m, n, rank, seed=8)
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    for target in ("self", "proj"):
        if target == "self":
            s = gpu.Selector(dev(A32), m, k_max=10, self_target=True)
            s.set_target(None)
        else:
            s = gpu.Selector(dev(A32), m, k_max=10, r_max=6)
            s.set_target(dev(colstore32(Av @ synth.omega_gauss(n, 6, seed=1).astype(np.float64))))
        Wt = _embedding(10, n)
        s.set_embedding(Wt)
        idx, obj, ns, st = s.select(10)
        assert st == gpu.WARN_EXHAUSTED and ns == rank
        W = Wt.cpu().numpy().astype(np.float64)
        assert np.all(W[rank:] == 7.0)
        Q = s.read(gpu.STATE_Q, m * rank, np.float64).reshape(rank, m).T
        assert np.max(np.abs(Q @ W[:rank, :n] - Av)) <= 1e-5 * np.abs(Av).max()


def test_embedding_argument_errors(gpu):
    import torch
    m, n = 64, 100
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 8, 0.1, seed=1))
    s = gpu.Selector(dev(A32), m, k_max=4, self_target=True)
    bad = torch.zeros(4, n - 1, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        s.set_embedding(bad)
    with pytest.raises(gpu.GcssError) as e:
        gpu.set_embedding(s.h, bad.data_ptr(), n - 1)
    assert e.value.status == gpu.ERR_ARG
    idx = torch.zeros(3, dtype=torch.int64, device="cuda")
    W = torch.zeros(4, n, dtype=torch.float32, device="cuda")
    with pytest.raises(gpu.GcssError):
        gpu.qless_r(W.data_ptr(), n, n, idx.data_ptr(), 3, W.data_ptr(), 2)   # ldr < k
    # a pick outside [0, n) gives a NaN column, not a fault
    idx = torch.tensor([1, n + 7, 2], dtype=torch.int64, device="cuda")
    R = gpu.qless_r_tensor(W, n, idx).cpu().numpy()
    assert np.all(np.isnan(R[:, 1])) and not np.any(np.isnan(R[:, [0, 2]]))


# ---------------------------------------------------------------- rank-k ----
# Tolerances: the GPU's W is binary32 (relative 2^-24 per entry) and its
# Gram matrix and eigen-decomposition are FP64, so sigma_j is within
# ~1e-7 sigma_1 of the oracle's; the triplets agree to ~1e-7 sigma_1 / gap;
# the approximation's entries to 1e-5 ||A_i||.
def _geometric(m, n, rank, ratio, noise, seed):
    """U diag(ratio^j) V^T + noise: singular gaps of (1 - ratio) sigma_j."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, rank)))
    V, _ = np.linalg.qr(rng.standard_normal((n, rank)))
    return (U * ratio ** np.arange(rank)) @ V.T + noise * rng.standard_normal((m, n))


def _rank_case(gpu, target, dt, m, n, kmax, seed=40):
    A = _geometric(m, n, min(3 * kmax, m), 0.85, 1e-6, seed)
    A32 = colstore32(A)
    Adev, sc, Aval = _values(gpu, A32, m, dt)
    # candidates stay eligible down to the noise floor (tau), so that every
    # case makes all kmax picks
    if target == "self":
        s = gpu.Selector(Adev, m, k_max=kmax, self_target=True, scales=sc, tau=1e-12)
        s.set_target(None)
    else:
        Bv = stored_dense(colstore32(Aval @ synth.omega_gauss(n, 64, seed=seed + 1).astype(np.float64)), m)
        s = gpu.Selector(Adev, m, k_max=kmax, r_max=64, scales=sc, tau=1e-12)
        s.set_target(dev(colstore32(Bv)))
    Wt = _embedding(kmax, n)
    s.set_embedding(Wt)
    idx, obj, ns, st = s.select(kmax)
    assert ns == kmax
    return s, Aval, idx, obj


def _check_rank(s, Aval, idx, obj, l, k, target):
    ref = embed.rank_k(Aval, [int(x) for x in idx[:l]], k)
    U, sig, V, err = s.rank_k(l, k)
    U = U.cpu().numpy().T                   # m x k
    V = V.cpu().numpy().astype(np.float64).T  # n x k
    s1 = ref["sigma"][0]
    assert np.max(np.abs(sig - ref["sigma"])) <= 1e-6 * s1, np.max(np.abs(sig - ref["sigma"])) / s1
    assert np.all(np.diff(sig) <= 0)
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-10)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=2e-5)
    # singular vectors where the spectrum separates them; the approximation always
    gap = np.minimum(np.abs(np.diff(np.r_[np.inf, ref["sigma"]])), np.abs(np.diff(np.r_[ref["sigma"], -np.inf])))
    sep = gap > 1e-3 * s1
    assert np.max(np.abs(U - ref["U"])[:, sep]) <= 1e-4
    assert np.max(np.abs(V - ref["V"])[:, sep]) <= 1e-4
    approx = (U * sig[None, :]) @ V.T
    nrm = np.sqrt(np.sum(Aval * Aval, axis=0))
    assert np.max(np.abs(approx - ref["approx"]) / nrm[None, :]) <= 1e-5
    F = np.sum(Aval * Aval)
    d = abs(err - ref["err"])
    if target == "self":
        assert d <= 1e-5 * ref["err"] + 1e-8 * F, (err, ref["err"], F)
    else:
        assert d <= 1e-5 * ref["err"] + 1e-6 * F, (err, ref["err"], F)


@pytest.mark.parametrize("target", ["self", "proj"])
@pytest.mark.parametrize("dt", ["f32", "fp8"])
def test_rank_k_matches_oracle(gpu, target, dt):
    m, n, kmax = 300, 2000, 40
    s, Aval, idx, obj = _rank_case(gpu, target, dt, m, n, kmax)
    for l, k in [(kmax, 1), (kmax, 10), (kmax, kmax), (17, 5)]:
        _check_rank(s, Aval, idx, obj, l, k, target)


@pytest.mark.parametrize("l", [64, 65, 200])
def test_rank_k_several_jacobi_blocks(gpu, l):
    """l spanning one to seven block pairs (padding and ragged sizes)."""
    m, n = 260, 3000
    s, Aval, idx, obj = _rank_case(gpu, "self", "f32", m, n, l, seed=l)
    _check_rank(s, Aval, idx, obj, l, 10, "self")


def test_rank_k_exact_low_rank_is_the_svd(gpu):
    m, n, rank = 40, 100, 5
    A = synth.int_lowrank_dense(m, n, rank, seed=8)
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    s = gpu.Selector(dev(A32), m, k_max=10, self_target=True)
    s.set_target(None)
    Wt = _embedding(10, n)
    s.set_embedding(Wt)
    idx, obj, ns, st = s.select(10)
    assert ns == rank
    U, sig, V, err = s.rank_k(rank, rank)
    sv = np.linalg.svd(Av, compute_uv=False)
    np.testing.assert_allclose(sig, sv[:rank], rtol=1e-6)
    assert err <= 1e-6 * np.sum(Av * Av)
    approx = (U.cpu().numpy().T * sig[None, :]) @ V.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(approx - Av)) <= 1e-5 * np.abs(Av).max()


def test_rank_k_state_and_argument_errors(gpu):
    m, n = 64, 300
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 20, 0.1, seed=3))
    s = gpu.Selector(dev(A32), m, k_max=8, self_target=True)
    s.set_target(None)
    Wt = _embedding(8, n)
    s.set_embedding(Wt)
    with pytest.raises(gpu.GcssError) as e:
        s.rank_k(4, 2)                       # no selection yet
    assert e.value.status == gpu.ERR_STATE
    s.select(6)
    with pytest.raises(gpu.GcssError) as e:
        s.rank_k(7, 2)                       # more picks than the selection made
    assert e.value.status == gpu.ERR_ARG
    with pytest.raises(gpu.GcssError) as e:
        s.rank_k(4, 5)                       # k > l
    assert e.value.status == gpu.ERR_ARG
    s.rank_k(6, 6)
    s.reconstruction_error(np.array([3, 1], dtype=np.int64))   # rebuilds the basis
    with pytest.raises(gpu.GcssError) as e:
        s.rank_k(2, 1)
    assert e.value.status == gpu.ERR_STATE
