"""GPU path vs the FP64 oracle, element by element, on seeded inputs.

Tolerances (FP32 arithmetic on the GPU vs FP64 in the oracle):
  * picks: identical on inputs whose score gaps are separated (planted
    inputs, or the prefix before the oracle's gap drops below 1e-4);
  * objective / reconstruction error: relative 1e-5 in FP32 mode;
  * initial scores: f relative 1e-4 (FP32 matrix-core dot products over
    up to a few thousand terms), g relative 1e-12 (FP64 sums of squares).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import colstore32, dev, f64cs, rel, stored_dense

pytestmark = pytest.mark.gpu


def _sel(gpu, A32, m, **kw):
    return gpu.Selector(dev(A32), m, **kw)


# ---------------------------------------------------------------- a0 / K0 ----
@pytest.mark.parametrize("m,n", [(37, 50), (500, 300), (1000, 129)])
def test_quantizers_bit_exact(gpu, m, n):
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)) * 10.0 ** rng.integers(-6, 6, size=(1, n))
    A[:, 3] = 0.0
    A[5 % m, 7] = 1e-30
    A32 = colstore32(A)
    codes_ref, sc_ref = oracle.quantize_fp8(A32, m, ldo=((m + 255) // 256) * 256)
    c, sc = gpu.quantize_tensor(dev(A32), m, "fp8")
    np.testing.assert_array_equal(sc.cpu().numpy(), sc_ref)
    np.testing.assert_array_equal(c.cpu().numpy(), codes_ref)
    h_ref = oracle.quantize_bf16(A32, m, ldo=((m + 127) // 128) * 128)
    h, _ = gpu.quantize_tensor(dev(A32), m, "bf16")
    np.testing.assert_array_equal(h.cpu().numpy().view(np.uint16), h_ref)


@pytest.mark.parametrize("m,n,r", [(37, 300, 7), (300, 1000, 256), (1000, 700, 130),
                                   # 64 <= r <= 128, m >= 256: 256 x 128 tiles (exact and
                                   # ragged row tiles, one short k split)
                                   (1024, 3000, 128), (260, 1500, 64), (256, 300, 64),
                                   (512, 257, 128)])
def test_projection_matches_oracle_dots(gpu, m, n, r):
    import torch
    A = synth.gauss_lowrank_dense(m, n, 10, 0.1, seed=m)
    A32 = colstore32(A)
    Om = synth.omega_gauss(n, r, seed=r)
    s = _sel(gpu, A32, m, k_max=4, r_max=r)
    B = s.project_target(dev(Om)).cpu().numpy()[:, :m].T.astype(np.float64)
    Bref = stored_dense(A32, m) @ Om.astype(np.float64)
    # each entry is one FP64 dot of a row of A with a column of Omega
    scale = np.sqrt(np.sum(stored_dense(A32, m) ** 2, axis=1))[:, None] * np.sqrt(np.sum(Om.astype(np.float64) ** 2, axis=0))[None, :]
    assert np.max(np.abs(B - Bref) / scale) < 1e-6
    torch.cuda.synchronize()


def _quantized(gpu, A32, m, dt):
    """Stored codes on the GPU and the values they decode to (oracle decoder)."""
    Adev, sc = gpu.quantize_tensor(dev(A32), m, dt)
    if dt == "bf16":
        Aval = oracle.decode_columns(oracle.quantize_bf16(A32, m), m, "bf16").T
    else:
        codes, scl = oracle.quantize_fp8(A32, m)
        Aval = oracle.decode_columns(codes, m, "fp8", scl).T
    return Adev, sc, Aval


@pytest.mark.parametrize("m,n,r,dt", [(300, 1000, 256, "bf16"), (520, 700, 200, "fp8"),
                                        (516, 900, 260, "bf16"), (1028, 1500, 512, "fp8"),
                                        (516, 2000, 96, "bf16"), (300, 1500, 128, "fp8"),
                                        (1024, 1300, 124, "bf16")])
def test_projection_quantized_storage(gpu, m, n, r, dt):
    """B = A_hat Omega from BF16 / FP8 codes (large-tile path), entry by entry."""
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 10, 0.1, seed=m + 1))
    Om = synth.omega_gauss(n, r, seed=r + 1)
    Adev, sc, Aval = _quantized(gpu, A32, m, dt)
    s = gpu.Selector(Adev, m, k_max=4, r_max=r, scales=sc)
    B = s.project_target(dev(Om)).cpu().numpy()[:, :m].T.astype(np.float64)
    Bref = Aval @ Om.astype(np.float64)
    scale = np.sqrt(np.sum(Aval ** 2, axis=1))[:, None] * np.sqrt(np.sum(Om.astype(np.float64) ** 2, axis=0))[None, :]
    assert np.max(np.abs(B - Bref) / scale) < 1e-6


@pytest.mark.parametrize("m,n", [(300, 500), (601, 1333), (256, 4096)])
def test_gram_binary32_matches_fp64(gpu, m, n):
    """C = A A^T of binary32 A (large-tile path: bfloat16 matrix cores with
    three-part operands) entry by entry against the FP64 product, exactly
    symmetric.  Tolerance relative to sqrt(C_ii C_jj): binary32 accumulation
    over n terms, 2^-24 sqrt(n) plus 1e-6 (the split's dropped products are
    below 2^-23 |a b| each); measured 1.0e-6 - 1.5e-6 on these cases, against
    2.0e-6 - 3.3e-6 for the binary32 matrix-core kernel."""
    A = synth.gauss_lowrank_dense(m, n, 40, 0.1, seed=m)
    A[:, 7] *= 1e-3                      # columns of very different scales
    A[:, 9] *= 1e3
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    s = gpu.Selector(dev(A32), m, k_max=4, self_target=True)
    s.set_target(None)
    C = s.read(gpu.STATE_GRAM, m * m, np.float32).reshape(m, m).astype(np.float64)
    Cr = Av @ Av.T
    assert np.array_equal(C, C.T)
    scale = np.sqrt(np.outer(np.diag(Cr), np.diag(Cr)))
    assert np.max(np.abs(C - Cr) / scale) <= 6e-8 * np.sqrt(n) + 1e-6


@pytest.mark.parametrize("m,n,dt", [(300, 500, "bf16"), (257, 400, "fp8")])
def test_gram_quantized_storage(gpu, m, n, dt):
    """C = A_hat A_hat^T from BF16 / FP8 codes (large-tile path), exactly symmetric."""
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 12, 0.05, seed=m + 2))
    Adev, sc, Aval = _quantized(gpu, A32, m, dt)
    s = gpu.Selector(Adev, m, k_max=4, self_target=True, scales=sc)
    s.set_target(None)
    C = s.read(gpu.STATE_GRAM, m * m, np.float32).reshape(m, m).astype(np.float64)
    Cr = Aval @ Aval.T
    assert np.array_equal(C, C.T)
    np.testing.assert_allclose(C, Cr, rtol=0, atol=1e-5 * np.abs(Cr).max())
    f = s.read(gpu.STATE_F0, n, np.float64)
    fr, _ = oracle.init_scores(f64cs(Aval), m)
    np.testing.assert_allclose(f, fr, rtol=1e-4)


# ---------------------------------------------------------------- a1 ---------
@pytest.mark.parametrize("m,n,r,dt", [(37, 70, 3, "f32"), (500, 1000, 64, "f32"), (1000, 300, 256, "f32"),
                                      (300, 500, 300, "f32"), (600, 400, 130, "bf16"), (700, 333, 40, "fp8"),
                                      # n >= 1024: the bfloat16 matrix-core kernel with
                                      # 128-row chunks (64 <= r <= 128) or 256-row chunks
                                      # (r >= 192), binary32 128-row tiles between, ragged tiles
                                      (1024, 3000, 128, "f32"), (1000, 2500, 150, "bf16"),
                                      (520, 1100, 128, "fp8"), (300, 2049, 200, "f32"),
                                      (1000, 2500, 96, "bf16"), (516, 1500, 64, "f32"),
                                      (260, 1030, 100, "fp8"), (256, 1024, 128, "bf16"),
                                      (256, 1024, 64, "fp8")])
def test_initial_scores_factor(gpu, m, n, r, dt):
    A = synth.gauss_lowrank_dense(m, n, 8, 0.05, seed=n)
    A[:, 5] = 0.0
    A32 = colstore32(A)
    B = np.random.default_rng(r).standard_normal((m, r))
    Bcs = colstore32(B)
    if dt == "f32":
        Adev, sc, Aval = dev(A32), None, stored_dense(A32, m)
    else:
        Adev, sc = gpu.quantize_tensor(dev(A32), m, dt)
        if dt == "bf16":
            Aval = oracle.decode_columns(oracle.quantize_bf16(A32, m), m, "bf16").T
        else:
            codes, scl = oracle.quantize_fp8(A32, m)
            Aval = oracle.decode_columns(codes, m, "fp8", scl).T
    s = gpu.Selector(Adev, m, k_max=4, r_max=r, scales=sc)
    s.set_target(dev(Bcs))
    f = s.read(gpu.STATE_F0, n, np.float64)
    g = s.read(gpu.STATE_G0, n, np.float64)
    fr, gr = oracle.init_scores(f64cs(Aval), m, B=f64cs(stored_dense(Bcs, m)))
    np.testing.assert_allclose(g, gr, rtol=1e-12, atol=0)
    np.testing.assert_allclose(f, fr, rtol=1e-4, atol=1e-6 * fr.max())


@pytest.mark.parametrize("m,n", [(37, 90), (500, 1000), (260, 300)])
def test_initial_scores_self_target(gpu, m, n):
    A = synth.gauss_lowrank_dense(m, n, 12, 0.05, seed=m)
    A32 = colstore32(A)
    s = _sel(gpu, A32, m, k_max=4, self_target=True)
    s.set_target(None)
    C = s.read(gpu.STATE_GRAM, m * m, np.float32).reshape(m, m).astype(np.float64)
    Av = stored_dense(A32, m)
    Cr = Av @ Av.T
    assert np.array_equal(C, C.T)  # exactly symmetric
    np.testing.assert_allclose(C, Cr, rtol=0, atol=1e-5 * np.abs(Cr).max())
    f = s.read(gpu.STATE_F0, n, np.float64)
    fr, gr = oracle.init_scores(f64cs(Av), m)
    np.testing.assert_allclose(f, fr, rtol=1e-4)


# ---------------------------------------------------------------- a2-a5 ------
@pytest.mark.parametrize("target", ["self", "proj"])
@pytest.mark.parametrize("dt", ["f32", "bf16", "fp8"])
def test_planted_gap_indices_identical(gpu, target, dt):
    m, n, k = 256, 3000, 12
    A, pos = synth.planted_dense(m, n, k, 1.5, seed=5)
    A32 = colstore32(A)
    if dt == "f32":
        Adev, sc, Aval = dev(A32), None, stored_dense(A32, m)
    elif dt == "bf16":
        Adev, sc = gpu.quantize_tensor(dev(A32), m, "bf16")
        Aval = oracle.decode_columns(oracle.quantize_bf16(A32, m), m, "bf16").T
    else:
        Adev, sc = gpu.quantize_tensor(dev(A32), m, "fp8")
        codes, scl = oracle.quantize_fp8(A32, m)
        Aval = oracle.decode_columns(codes, m, "fp8", scl).T
    if target == "self":
        s = gpu.Selector(Adev, m, k_max=k, self_target=True, scales=sc)
        s.set_target(None)
        ref = oracle.select(f64cs(Aval), m, k)
    else:
        B = Aval @ synth.omega_gauss(n, 256, seed=9).astype(np.float64)
        Bcs = colstore32(B)
        s = gpu.Selector(Adev, m, k_max=k, r_max=256, scales=sc)
        s.set_target(dev(Bcs))
        ref = oracle.select(f64cs(Aval), m, k, B=f64cs(stored_dense(Bcs, m)))
    idx, obj, ns, st = s.select(k)
    assert ns == k and st == gpu.OK
    assert np.min(ref["gap"]) > 1e-3
    assert list(idx) == list(ref["idx"])
    np.testing.assert_allclose(obj, ref["obj"], rtol=1e-5)


def _prefix_len(a, b):
    n = 0
    for x, y in zip(a, b):
        if x != y:
            break
        n += 1
    return n


@pytest.mark.parametrize("case", ["css_500x1000", "gcss_1000x20000_r128", "ragged_333x4097_r7",
                                  "gcss_odd_601x3000_r512"])
def test_selection_matches_oracle(gpu, case):
    if case == "css_500x1000":
        m, n, k = 500, 1000, 20
        A = synth.gauss_lowrank_dense(m, n, 50, 0.01, seed=0)
        r = 0
    elif case == "gcss_odd_601x3000_r512":
        # odd m with many target columns (several column dots per workgroup)
        m, n, k, r = 601, 3000, 15, 512
        A = synth.gauss_lowrank_dense(m, n, 60, 0.05, seed=21)
    elif case == "gcss_1000x20000_r128":
        m, n, k, r = 1000, 20000, 30, 128
        A = synth.spectral_lowrank_dense(m, n, 256, 0.7, 1e-3, seed=1)
    else:
        m, n, k, r = 333, 4097, 25, 7
        A = synth.gauss_lowrank_dense(m, n, 40, 0.1, seed=2)
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    if r == 0:
        s = _sel(gpu, A32, m, k_max=k, self_target=True)
        s.set_target(None)
        Bv = None
    else:
        Bv = stored_dense(colstore32(Av @ synth.omega_gauss(n, r, seed=3).astype(np.float64)), m)
        s = _sel(gpu, A32, m, k_max=k, r_max=r)
        s.set_target(dev(colstore32(Bv)))
    idx, obj, ns, st = s.select(k)
    ref = oracle.select(f64cs(Av), m, k, B=None if Bv is None else f64cs(Bv))
    # identical picks up to the first step whose oracle score gap is below 1e-4
    sep = int(np.argmax(ref["gap"] < 1e-4)) if np.any(ref["gap"] < 1e-4) else k
    assert _prefix_len(idx, ref["idx"]) >= sep
    Bc = None if Bv is None else f64cs(Bv)
    e_gpu = oracle.error(f64cs(Av), m, idx, B=Bc)
    e_orc = oracle.error(f64cs(Av), m, ref["idx"], B=Bc)
    assert rel(e_gpu, e_orc) <= 1e-5
    # the GPU's recursive objective is the explicit error of every prefix
    for t in (1, k // 2, k):
        assert rel(obj[t], oracle.error(f64cs(Av), m, idx[:t], B=Bc)) <= 1e-5
    assert np.all(np.diff(obj) <= 0)
    # a7: the library's reconstruction error of its own picks and of the oracle's
    assert rel(s.reconstruction_error(idx), e_gpu) <= 1e-5
    assert rel(s.reconstruction_error(ref["idx"]), e_orc) <= 1e-5


def test_basis_orthonormal_and_reproducible(gpu):
    m, n, k, r = 700, 5000, 40, 64
    A = synth.spectral_lowrank_dense(m, n, 100, 0.5, 1e-3, seed=4)
    A32 = colstore32(A)
    B = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=5).astype(np.float64))
    s = _sel(gpu, A32, m, k_max=k, r_max=r)
    s.set_target(dev(B))
    i1, o1, _, _ = s.select(k)
    Q = s.read(gpu.STATE_Q, m * k, np.float64).reshape(k, m).T
    assert np.max(np.abs(Q.T @ Q - np.eye(k))) < 1e-13
    # span(Q) = span(A_S): the residual of A_S on Q vanishes
    AS = stored_dense(A32, m)[:, i1]
    R = AS - Q @ (Q.T @ AS)
    assert np.max(np.abs(R)) < 1e-10 * np.max(np.abs(AS))
    i2, o2, _, _ = s.select(k)
    assert np.array_equal(i1, i2) and np.array_equal(o1.view(np.int64), o2.view(np.int64))
    d_idx, d_obj, d_ns = s.select_async(k)
    assert np.array_equal(d_idx.cpu().numpy(), i1)
    assert np.array_equal(d_obj.cpu().numpy().view(np.int64), o1.view(np.int64))
    assert int(d_ns.cpu()[0]) == k


def test_scores_after_steps_follow_the_recursion(gpu):
    m, n, k, r = 300, 2000, 8, 32
    A = synth.gauss_lowrank_dense(m, n, 30, 0.1, seed=6)
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    Bv = stored_dense(colstore32(Av @ synth.omega_gauss(n, r, seed=7).astype(np.float64)), m)
    s = _sel(gpu, A32, m, k_max=k, r_max=r)
    s.set_target(dev(colstore32(Bv)))
    idx, _, _, _ = s.select(k)
    ref = oracle.select(f64cs(Av), m, k, B=f64cs(Bv), trace=True)
    assert list(idx) == list(ref["idx"])
    # after k picks the GPU has applied k-1 updates: compare with the oracle's
    # scores just before pick k
    f = s.read(gpu.STATE_F, n, np.float64)
    g = s.read(gpu.STATE_G, n, np.float64)
    fr, gr = ref["fg"][k - 1]
    f0, g0 = ref["fg"][0]
    dg = np.abs(g - gr) / g0
    df = np.abs(f - fr) / (f0 + 1e-9 * f0.max())
    ig, jf = int(np.argmax(dg)), int(np.argmax(df))
    assert dg[ig] <= 1e-5, f"g: col {ig} gpu {g[ig]!r} oracle {gr[ig]!r} g0 {g0[ig]!r} picked {ig in set(idx)}"
    assert df[jf] <= 1e-5, f"f: col {jf} gpu {f[jf]!r} oracle {fr[jf]!r} f0 {f0[jf]!r} picked {jf in set(idx)}"


# ---------------------------------------------------------------- edges ------
def test_exact_low_rank_exhausts(gpu):
    m, n, rank = 40, 100, 5
    A = synth.int_lowrank_dense(m, n, rank, seed=8)
    A32 = colstore32(A)
    s = _sel(gpu, A32, m, k_max=10, self_target=True)
    s.set_target(None)
    idx, obj, ns, st = s.select(10)
    assert st == gpu.WARN_EXHAUSTED and ns == rank
    assert np.all(idx[rank:] == -1)
    assert abs(obj[rank]) <= 1e-6 * obj[0]
    assert np.all(obj[rank:] == obj[rank])
    assert oracle.error(f64cs(stored_dense(A32, m)), m, idx[:rank]) <= 1e-12 * obj[0]


def test_degenerate_columns_never_picked(gpu):
    m, n = 64, 200
    A = synth.gauss_lowrank_dense(m, n, 20, 0.1, seed=9)
    A[:, 10] = 0.0                 # zero column
    A[:, 20] = A[:, 21]            # duplicate
    A[:, 30] = np.nan              # non-finite
    A32 = colstore32(A)
    s = _sel(gpu, A32, m, k_max=40, self_target=False, r_max=8)
    B = colstore32(np.nan_to_num(A) @ synth.omega_gauss(n, 8, seed=1).astype(np.float64))
    s.set_target(dev(B))
    idx, obj, ns, st = s.select(40)
    picked = set(idx[idx >= 0].tolist())
    assert 10 not in picked and 30 not in picked
    assert not ({20, 21} <= picked)
    assert len(picked) == ns


@pytest.mark.parametrize("m,n,k", [(5, 1, 1), (64, 40, 40), (20, 65, 20), (8192, 70, 5), (4097, 300, 6)])
def test_small_and_extreme_shapes(gpu, m, n, k):
    A = np.random.default_rng(m * n).standard_normal((m, n))
    A32 = colstore32(A)
    s = _sel(gpu, A32, m, k_max=k, self_target=True)
    s.set_target(None)
    idx, obj, ns, st = s.select(k)
    ref = oracle.select(f64cs(stored_dense(A32, m)), m, k, tau=1e-4)
    assert ns == ref["n_selected"]
    sep = int(np.argmax(ref["gap"] < 1e-4)) if np.any(ref["gap"] < 1e-4) else k
    assert _prefix_len(idx, ref["idx"]) >= sep
    if k == n:
        assert sorted(idx) == list(range(n))
    np.testing.assert_allclose(obj, ref["obj"], rtol=1e-5, atol=1e-6 * obj[0])


def test_single_row_ties(gpu):
    # m = 1: every column spans the same line, all scores tie in exact
    # arithmetic; one pick explains everything, then nothing is left
    m, n = 1, 10
    A = np.random.default_rng(3).standard_normal((m, n)) + 3.0
    s = _sel(gpu, colstore32(A), m, k_max=3, self_target=True)
    s.set_target(None)
    idx, obj, ns, st = s.select(3)
    assert ns == 1 and st == gpu.WARN_EXHAUSTED and 0 <= idx[0] < n
    assert abs(obj[1]) <= 1e-6 * obj[0]


def test_argument_and_state_errors(gpu):
    m, n = 50, 100
    A32 = colstore32(np.random.default_rng(0).standard_normal((m, n)))
    s = _sel(gpu, A32, m, k_max=5, r_max=4)
    with pytest.raises(gpu.GcssError) as ei:
        s.select(3)
    assert ei.value.status == gpu.ERR_STATE
    with pytest.raises(gpu.GcssError) as ei:
        s.set_target(None)  # self target not reserved
    assert ei.value.status == gpu.ERR_STATE
    B = colstore32(np.random.default_rng(1).standard_normal((m, 4)))
    s.set_target(dev(B))
    with pytest.raises(gpu.GcssError) as ei:
        s.select(6)
    assert ei.value.status == gpu.ERR_ARG
    with pytest.raises(gpu.GcssError):
        s.reconstruction_error([1, 1])
    with pytest.raises(gpu.GcssError):
        s.reconstruction_error([n])


# ---------------------------------------------------------------- a6 ---------
# m = 256: in binary32 every lane's chunks lie inside m (the unmasked column
# loop); in BF16, and at the ragged m = 333 (a partial last chunk) in both,
# the masked loop
@pytest.mark.parametrize("dt,m", [("f32", 256), ("bf16", 256), ("f32", 333), ("bf16", 333)])
def test_batched_blocks_and_merge_match_oracle(gpu, dt, m):
    r, kb, km = 32, 5, 12
    widths = synth.block_widths(8, 150, 1500, seed=3)
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A = synth.gauss_lowrank_dense(m, n, 24, 0.05, seed=12, scale=1 / np.sqrt(24))
    A32 = colstore32(A)
    if dt == "f32":
        Adev, sc, Av = dev(A32), None, stored_dense(A32, m)
    else:
        Adev, sc = gpu.quantize_tensor(dev(A32), m, "bf16")
        Av = oracle.decode_columns(oracle.quantize_bf16(A32, m), m, "bf16").T
    Bv = stored_dense(colstore32(Av @ synth.omega_gauss(n, r, seed=13).astype(np.float64)), m)
    s = gpu.Selector(Adev, m, k_max=kb, r_max=r, scales=sc, batched=(len(widths), kb, km))
    s.set_target(dev(colstore32(Bv)))
    ib, im, om, nm, st = s.select_batched(off, kb, km)
    ref = oracle.select_distributed(f64cs(Av), m, f64cs(Bv), off, kb, km)
    for b in range(len(widths)):
        rb = oracle.select(f64cs(Av[:, off[b]:off[b + 1]]), m, kb, B=f64cs(Bv))
        sep = int(np.argmax(rb["gap"] < 1e-4)) if np.any(rb["gap"] < 1e-4) else kb
        assert _prefix_len(ib[b], ref["idx_block"][b]) >= sep, b
    # the merge against the oracle run on the GPU's own pool (block order,
    # then pick order), whatever the blocks picked
    pool = [int(x) for x in ib.ravel() if x >= 0]
    rm = oracle.select(f64cs(Av[:, pool]), m, km, B=f64cs(Bv))
    sep = int(np.argmax(rm["gap"] < 1e-4)) if np.any(rm["gap"] < 1e-4) else km
    got = _prefix_len(im, [pool[i] for i in rm["idx"]])
    assert got >= sep
    np.testing.assert_allclose(om[:got + 1], rm["obj"][:got + 1], rtol=1e-5)
    if np.array_equal(ib, ref["idx_block"]):
        np.testing.assert_allclose(om, ref["obj_merge"], rtol=1e-5)
    e_gpu = oracle.error(f64cs(Av), m, im, B=f64cs(Bv))
    e_orc = oracle.error(f64cs(Av), m, ref["idx_merge"], B=f64cs(Bv))
    assert rel(e_gpu, e_orc) <= 1e-5
    assert nm == km and st == gpu.OK


def test_batched_on_dirty_workspace(gpu):
    """A workspace holding all-ones bytes (NaN as float, -1 as int64) gives
    the same picks as a zero-filled one: nothing is read before written."""
    import torch
    m, r, kb, km = 128, 16, 6, 10
    widths = [700, 64, 1025, 300]
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 20, 0.1, seed=14))
    Bcs = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=15).astype(np.float64))
    probe = gpu.Selector(dev(A32), m, k_max=kb, r_max=r, batched=(len(widths), kb, km))
    nbytes = probe.ws_bytes
    probe.close()
    res = []
    for fill in (0x00, 0xFF):
        ws = torch.full((nbytes,), fill, dtype=torch.uint8, device="cuda")
        s = gpu.Selector(dev(A32), m, k_max=kb, r_max=r, batched=(len(widths), kb, km), workspace=ws)
        s.set_target(dev(Bcs))
        ib, im, om, nm, st = s.select_batched(off, kb, km)
        assert nm == km and st == gpu.OK and np.all(ib >= 0), (fill, ib)
        i1, o1, n1, _ = s.select(kb)
        res.append((ib, im, om, i1, o1))
        s.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_batched_equals_blockwise_single_runs(gpu):
    m, r, kb, km = 128, 16, 6, 10
    widths = [700, 64, 1025, 300]
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 20, 0.1, seed=14))
    Bcs = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=15).astype(np.float64))
    s = gpu.Selector(dev(A32), m, k_max=kb, r_max=r, batched=(len(widths), kb, km))
    s.set_target(dev(Bcs))
    ib, im, om, nm, st = s.select_batched(off, kb, km)
    ib2, im2, om2, _, _ = s.select_batched(off, kb, km)  # replayed graph: identical
    assert np.array_equal(ib, ib2) and np.array_equal(im, im2)
    assert np.array_equal(om.view(np.int64), om2.view(np.int64))
    for b in range(len(widths)):
        sb = gpu.Selector(dev(np.ascontiguousarray(A32[off[b]:off[b + 1]])), m, k_max=kb, r_max=r)
        sb.set_target(dev(Bcs))
        i1, _, _, _ = sb.select(kb)
        assert list(ib[b]) == [int(x) + int(off[b]) for x in i1], b
