"""Pins of the FP64 oracle to facts the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses brute force
(explicit least squares), a closed form, an invariant, a library routine or
a value derived by hand from a definition.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def cs(M):
    """dense m x n -> float64 column store with ld = m."""
    return synth.to_colstore(M, lda=M.shape[0], dtype=np.float64)


def _tiny_cases():
    out = []
    for seed in range(6):
        rng = np.random.default_rng(100 + seed)
        m = int(rng.integers(5, 11))
        n = int(rng.integers(6, 13))
        A = synth.gauss_lowrank_dense(m, n, min(m, 3), 0.2, seed=seed)
        for r in (None, 1, 3):
            B = None if r is None else rng.standard_normal((m, r))
            out.append((seed, A, B))
    return out


# --- P1: every candidate's score is its exact objective decrease (Theorems 1/3,
# Problems 3/6); the pick is the brute-force argmin of F(S + {i}) ------------
@pytest.mark.parametrize("case", range(18))
def test_scores_equal_bruteforce_decrease(case):
    seed, A, B = _tiny_cases()[case]
    m, n = A.shape
    k = min(5, m - 1)
    res = oracle.select(cs(A), m, k, B=None if B is None else cs(B), trace=True)
    S, F, decs = brute.greedy(A, B, k)
    F0 = F[0]
    assert res["n_selected"] == k
    for t in range(k):
        f, g = res["fg"][t]
        cand = ~np.isnan(decs[t])
        score = f[cand] / g[cand]
        np.testing.assert_allclose(score, decs[t][cand], rtol=0, atol=1e-9 * F0)
        # the pick is the argmin when the brute-force gap is not at rounding level
        d = np.sort(decs[t][cand])[::-1]
        if d.size < 2 or d[0] - d[1] > 1e-8 * F0:
            assert res["idx"][t] == S[t]
        else:
            break
        np.testing.assert_allclose(res["obj"][t + 1], F[t + 1], rtol=1e-9, atol=1e-12 * F0)


# --- P11: r = 1 is forward stepwise least squares --------------------------
def test_single_target_vector_is_stepwise_least_squares():
    rng = np.random.default_rng(7)
    m, n = 9, 11
    A = rng.standard_normal((m, n))
    b = rng.standard_normal((m, 1))
    res = oracle.select(cs(A), m, 4, B=cs(b))
    S = list(res["idx"])
    for t in range(1, 5):
        x, *_ = np.linalg.lstsq(A[:, S[:t]], b[:, 0], rcond=None)
        rss = float(np.sum((b[:, 0] - A[:, S[:t]] @ x) ** 2))
        assert abs(res["obj"][t] - rss) <= 1e-10 * float(np.sum(b * b))


# --- P2 and P3: monotone objective; g of a selected column vanishes ---------
@pytest.mark.parametrize("target", ["self", "proj"])
def test_monotone_objective_and_selected_g_vanishes(target):
    m, n = 60, 150
    A = synth.gauss_lowrank_dense(m, n, 10, 0.01, seed=3)
    B = None if target == "self" else A @ synth.omega_gauss(n, 16, seed=4).astype(np.float64)
    res = oracle.select(cs(A), m, 25, B=None if B is None else cs(B))
    obj = res["obj"]
    assert np.all(np.diff(obj) <= 1e-12 * obj[0])
    assert np.all(res["upsn"] >= 0)
    g0 = np.sum(A * A, axis=0)
    sel = res["idx"]
    assert np.all(np.abs(res["g_final"][sel]) <= 1e-12 * g0[sel])


# --- P4: exactly low-rank input is reproduced exactly after rank(A) picks ---
@pytest.mark.parametrize("target", ["self", "proj"])
def test_exact_low_rank_reaches_zero_then_exhausts(target):
    m, n, rank = 12, 30, 4
    A = synth.int_lowrank_dense(m, n, rank, seed=11)
    assert np.linalg.matrix_rank(A) == rank
    B = None if target == "self" else A @ np.round(np.random.default_rng(5).standard_normal((n, 3)) * 4)
    res = oracle.select(cs(A), m, rank + 3, B=None if B is None else cs(B))
    assert res["status"] == oracle.EXHAUSTED
    assert res["n_selected"] == rank
    F0 = res["obj"][0]
    S = res["idx"][:rank]
    assert oracle.error(cs(A), m, S, B=None if B is None else cs(B)) <= 1e-20 * F0
    assert abs(res["obj"][rank]) <= 1e-12 * F0
    assert np.all(res["idx"][rank:] == -1)


# --- P5: orthogonal columns, closed form (golden) ---------------------------
def test_orthogonal_columns_closed_form():
    gold = json.load(open(os.path.join(GOLD, "orthogonal_columns.json")))
    A = synth.orthogonal_columns_dense(gold["sq_norms"])
    m, n = A.shape
    res = oracle.select(cs(A), m, n, tau=1e-12)
    assert list(res["idx"]) == gold["order"]
    np.testing.assert_allclose(res["obj"], gold["objective"], rtol=0, atol=1e-12)


# --- P6 and P12: k = 1 closed form, and greedy >= exhaustive optimum --------
@pytest.mark.parametrize("seed", range(4))
def test_first_pick_closed_form_and_exhaustive(seed):
    rng = np.random.default_rng(seed)
    m, n, r = 7, 9, 3
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((m, r))
    ratio = np.sum((B.T @ A) ** 2, axis=0) / np.sum(A * A, axis=0)
    res = oracle.select(cs(A), m, 1, B=cs(B))
    assert res["idx"][0] == int(np.argmax(ratio))
    assert abs(res["obj"][1] - (np.sum(B * B) - ratio.max())) <= 1e-12 * np.sum(B * B)
    S1, F1 = brute.exhaustive(A, B, 1)
    assert S1 == [res["idx"][0]]
    res3 = oracle.select(cs(A), m, 3, B=cs(B))
    _, F3 = brute.exhaustive(A, B, 3)
    assert res3["obj"][3] >= F3 - 1e-12 * np.sum(B * B)


# --- P7: the omega rows are W = Q^T A; W[:, S] is upper triangular with
# |diag R| of a QR of A_S on its diagonal (Section 6, Q-less QR) ------------
def test_omega_rows_give_qless_qr():
    m, n = 20, 40
    A = synth.gauss_lowrank_dense(m, n, 8, 0.05, seed=21)
    res = oracle.select(cs(A), m, 6, omega=True)
    S = res["idx"]
    W = res["omega"]
    R = W[:, S]
    scale = np.abs(R).max()
    assert np.max(np.abs(np.tril(R, -1))) <= 1e-13 * scale
    _, Rq = np.linalg.qr(A[:, S])
    np.testing.assert_allclose(np.diag(R), np.abs(np.diag(Rq)), rtol=1e-12)
    Q, _ = np.linalg.qr(A[:, S])
    np.testing.assert_allclose(np.abs(W), np.abs(Q.T @ A), atol=1e-12 * scale)


# --- P8: recursive objective equals the explicit error of every prefix ------
@pytest.mark.parametrize("target", ["self", "proj"])
def test_recursive_objective_matches_explicit_error(target):
    m, n = 40, 90
    A = synth.spectral_lowrank_dense(m, n, 15, 0.7, 1e-2, seed=31)
    B = None if target == "self" else A @ synth.omega_gauss(n, 12, seed=32).astype(np.float64)
    res = oracle.select(cs(A), m, 12, B=None if B is None else cs(B))
    F0 = res["obj"][0]
    for t in range(0, 13, 3):
        e_qr = oracle.error(cs(A), m, res["idx"][:t], B=None if B is None else cs(B))
        e_ls = brute.objective(A, B, list(res["idx"][:t]))
        assert abs(e_qr - e_ls) <= 1e-11 * F0
        assert abs(res["obj"][t] - e_qr) <= 1e-11 * F0


# --- P9 invariances and P10 (Omega = I reduces Algorithm 3 to Algorithm 1) ---
def test_invariances():
    m, n, r = 30, 70, 8
    A = synth.gauss_lowrank_dense(m, n, 6, 0.1, seed=41)
    B = A @ synth.omega_gauss(n, r, seed=42).astype(np.float64)
    base = oracle.select(cs(A), m, 10, B=cs(B))
    # column scaling of A leaves the spans, hence picks and objective, unchanged
    D = np.exp(np.random.default_rng(1).uniform(-2, 2, n))
    sc = oracle.select(cs(A * D), m, 10, B=cs(B))
    assert list(sc["idx"]) == list(base["idx"])
    np.testing.assert_allclose(sc["obj"], base["obj"], rtol=1e-9)
    # B -> c B R (R orthogonal): same picks, objective times c^2
    Rm, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((r, r)))
    c = 3.0
    br = oracle.select(cs(A), m, 10, B=cs(c * B @ Rm))
    assert list(br["idx"]) == list(base["idx"])
    np.testing.assert_allclose(br["obj"], c * c * base["obj"], rtol=1e-9)
    # target enters only through B B^T: B = A equals B = chol(A A^T)
    selfres = oracle.select(cs(A), m, 10)
    L = np.linalg.cholesky(A @ A.T)
    fac = oracle.select(cs(A), m, 10, B=cs(L))
    assert list(fac["idx"]) == list(selfres["idx"])
    np.testing.assert_allclose(fac["obj"], selfres["obj"], rtol=1e-9)
    # Omega = I: B = A I = A explicitly gives Algorithm 1's result
    ident = oracle.select(cs(A), m, 10, B=cs(A.copy()))
    assert list(ident["idx"]) == list(selfres["idx"])
    np.testing.assert_allclose(ident["obj"], selfres["obj"], rtol=1e-9)


# --- P13: random projection preserves the error in expectation (Section 5.1) --
def test_projection_preserves_error_on_average():
    m, n = 25, 60
    A = synth.gauss_lowrank_dense(m, n, 5, 0.3, seed=51)
    S = list(range(0, 60, 7))
    eA = oracle.error(cs(A), m, S)
    vals = []
    for s in range(200):
        Om = synth.omega_gauss(n, 20, seed=1000 + s).astype(np.float64)
        vals.append(oracle.error(cs(A), m, S, B=cs(A @ Om)))
    assert abs(np.mean(vals) / eA - 1.0) < 0.05


# --- Algorithm 4 composition --------------------------------------------------
def test_distributed_is_blockwise_then_merge():
    m, r = 16, 5
    widths = [7, 12, 9]
    off = np.concatenate([[0], np.cumsum(widths)])
    n = int(off[-1])
    A = synth.gauss_lowrank_dense(m, n, 6, 0.05, seed=61)
    B = A @ synth.omega_gauss(n, r, seed=62).astype(np.float64)
    d = oracle.select_distributed(cs(A), m, cs(B), off, 3, 4)
    pool = []
    for b in range(3):
        sub = A[:, off[b]:off[b + 1]]
        rb = oracle.select(cs(sub), m, 3, B=cs(B))
        assert list(d["idx_block"][b]) == list(rb["idx"] + off[b])
        pool += list(rb["idx"] + off[b])
    rm = oracle.select(cs(A[:, pool]), m, 4, B=cs(B))
    assert list(d["idx_merge"]) == [pool[i] for i in rm["idx"]]
    np.testing.assert_allclose(d["obj_merge"], rm["obj"], rtol=1e-12)
    # one block holding everything with a large per-block budget is plain Algorithm 3
    d1 = oracle.select_distributed(cs(A), m, cs(B), [0, n], n, 4)
    r1 = oracle.select(cs(A), m, 4, B=cs(B))
    assert list(d1["idx_merge"]) == list(r1["idx"])


# --- storage formats ----------------------------------------------------------
def test_fp8_points_from_definition():
    gold = json.load(open(os.path.join(GOLD, "fp8_e4m3_points.json")))
    for code, val in gold["decode"]:
        v = oracle.fp8_decode(int(code, 16))
        assert v == val and math.copysign(1, v) == math.copysign(1, val)
    for code in gold["nan_codes"]:
        assert math.isnan(oracle.fp8_decode(int(code, 16)))
    for x, code in gold["encode_rne_saturating"]:
        assert oracle.fp8_encode(x) == int(code, 16), (x, code)


def test_fp8_matches_library_and_is_nearest():
    torch = pytest.importorskip("torch")
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    lib_vals = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    ours = np.array([oracle.fp8_decode(c) for c in range(256)])
    both_nan = np.isnan(lib_vals) & np.isnan(ours)
    assert np.all(both_nan | (lib_vals == ours))
    finite = ours[np.isfinite(ours)]
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(-448, 448, 3000), rng.normal(0, 0.02, 3000)]).astype(np.float32)
    lib_codes = torch.from_numpy(xs).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    for x, lc in zip(xs, lib_codes):
        c = oracle.fp8_encode(float(x))
        assert c == lc, (x, c, lc)
        # nearest by brute force over all finite codes
        v = oracle.fp8_decode(c)
        assert abs(v - float(x)) <= np.min(np.abs(finite - float(x))) + 0.0


def test_bf16_matches_library_rne():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    xs = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000),
                         np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 0.0])]).astype(np.float32)
    lib = torch.from_numpy(xs).to(torch.bfloat16).view(torch.int16).numpy().astype(np.uint16)
    for x, lc in zip(xs, lib):
        assert oracle.bf16_encode(float(x)) == lc, x
        assert oracle.bf16_decode(int(lc)) == float(torch.tensor(int(np.int16(lc)), dtype=torch.int16).view(torch.bfloat16).float())


def test_quantized_columns_decode_within_half_step():
    m, n = 37, 20
    A = synth.gauss_lowrank_dense(m, n, 4, 0.1, seed=71)
    A[:, 3] = 0.0
    A32 = synth.to_colstore(A, lda=48)
    codes, sc = oracle.quantize_fp8(A32, m)
    assert sc[3] == 1.0 and np.all(codes[3] == 0)
    dec = oracle.decode_columns(codes, m, "fp8", sc)
    amax = np.max(np.abs(A32[:, :m]), axis=1)
    np.testing.assert_allclose(sc, (amax / np.float32(448)).astype(np.float32) * (amax > 0) + (amax == 0))
    # E4M3 has 3 mantissa bits: relative error <= 2^-4 for normals, abs <= 2^-10 * scale below
    err = np.abs(dec - A32[:, :m].astype(np.float64))
    bound = np.maximum(np.abs(A32[:, :m]) * 2.0 ** -4, 2.0 ** -10 * sc[:, None]) * (1 + 1e-6)
    assert np.all(err <= bound)
    h = oracle.quantize_bf16(A32, m)
    dh = oracle.decode_columns(h, m, "bf16")
    assert np.all(np.abs(dh - A32[:, :m]) <= np.abs(A32[:, :m]) * 2.0 ** -8 * (1 + 1e-9))


# --- the large-input definitions agree with the C oracle and brute force ----
def test_dense_definitions_match_oracle():
    from oracle import dense
    m, n, r = 30, 80, 6
    A = synth.gauss_lowrank_dense(m, n, 8, 0.1, seed=81)
    Om = synth.omega_gauss(n, r, seed=82).astype(np.float64)
    B = dense.project(cs(A), m, Om, chunk=17)
    np.testing.assert_allclose(B, A @ Om, rtol=1e-12, atol=1e-12)
    res = oracle.select(cs(A), m, 7, B=cs(B))
    S = list(res["idx"])
    for t in (0, 3, 7):
        assert abs(dense.error(A[:, S[:t]], B) - oracle.error(cs(A), m, S[:t], B=cs(B))) <= 1e-10 * res["obj"][0]
    # scores given a prefix equal the brute-force objective decrease
    for t in (0, 4):
        sc = dense.scores(A[:, S[:t]], A, B)
        F = brute.objective(A, B, S[:t])
        for i in range(0, n, 9):
            if i in S[:t]:
                continue
            assert abs(sc[i] - (F - brute.objective(A, B, S[:t] + [i]))) <= 1e-9 * res["obj"][0]
    # the picks maximise the criterion
    for t in range(7):
        sc = dense.scores(A[:, S[:t]], A, B)
        sc[S[:t]] = -np.inf
        assert int(np.argmax(sc)) == S[t]
