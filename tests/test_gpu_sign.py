"""Random sign targets drawn on the GPU (Section 5.1) against the oracle:
the generated Omega bit for bit (through A = I, where B = Omega exactly),
B = A Omega entry by entry for both kernels (sparse gather, matrix cores
with generated tiles) and every storage type, and the selection it drives.

Tolerance of B: each entry is a binary32 sum of +-A_ij terms, compared with
the FP64 sum relative to ||A_row|| ||Omega_col|| (1e-6, as for the Gaussian
projection)."""
import math

import numpy as np
import pytest

import oracle
from oracle import rng
import synth
from tests.gpu_util import colstore32, dev, f64cs, stored_dense

pytestmark = pytest.mark.gpu
SEED = 0x0123456789ABCDEF


def _values(gpu, A32, m, dt):
    if dt == "f32":
        return dev(A32), None, stored_dense(A32, m)
    Adev, sc = gpu.quantize_tensor(dev(A32), m, dt)
    if dt == "bf16":
        return Adev, sc, oracle.decode_columns(oracle.quantize_bf16(A32, m), m, "bf16").T
    codes, scl = oracle.quantize_fp8(A32, m)
    return Adev, sc, oracle.decode_columns(codes, m, "fp8", scl).T


@pytest.mark.parametrize("density", ["sparse", 0.3, 1.0])
def test_generated_omega_is_bit_exact(gpu, density):
    """A = I (n x n): B = Omega itself, exactly, for the sparse kernel
    (d r <= 4) and the matrix-core kernel with generated tiles."""
    n = 600
    r = 96 if density == "sparse" else 300      # d r = 3.9 (sparse kernel) or >= 90
    d = 1.0 / math.sqrt(n) if density == "sparse" else density
    A32 = colstore32(np.eye(n))
    s = gpu.Selector(dev(A32), n, k_max=2, r_max=r)
    B = s.project_sign(SEED, r, density=d).cpu().numpy()[:, :n].T.astype(np.float64)
    ref = rng.omega_rows(0, n, r, SEED, d)
    assert np.array_equal(B, ref)
    B2 = s.project_sign(SEED, r, density=d).cpu().numpy()[:, :n].T.astype(np.float64)
    assert np.array_equal(B2, B)


@pytest.mark.parametrize("m,n,r,density,dt", [
    (300, 5000, 100, "sparse", "f32"), (300, 5000, 100, "sparse", "bf16"),
    (520, 7000, 64, "sparse", "fp8"), (8192, 900, 40, "sparse", "f32"),
    (300, 3000, 256, 1.0, "f32"), (257, 2000, 200, 1.0, "fp8"), (600, 1500, 70, 0.2, "bf16")])
def test_sign_projection_matches_oracle(gpu, m, n, r, density, dt):
    d = 1.0 / math.sqrt(n) if density == "sparse" else density
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 10, 0.1, seed=m + r))
    Adev, sc, Aval = _values(gpu, A32, m, dt)
    s = gpu.Selector(Adev, m, k_max=2, r_max=r, scales=sc)
    B = s.project_sign(SEED + 1, r, density=d).cpu().numpy()[:, :m].T.astype(np.float64)
    Om = rng.omega_rows(0, n, r, SEED + 1, d)
    Bref = Aval @ Om
    scale = (np.sqrt(np.sum(Aval ** 2, axis=1))[:, None]
             * np.maximum(np.sqrt(np.sum(Om ** 2, axis=0)), 1.0)[None, :])
    assert np.max(np.abs(B - Bref) / scale) < 1e-6


@pytest.mark.parametrize("density", ["sparse", 1.0])
def test_sign_target_selection_matches_oracle(gpu, density):
    m, n, k, r = 256, 3000, 12, 128
    d = 1.0 / math.sqrt(n) if density == "sparse" else density
    A, _ = synth.planted_dense(m, n, k, 1.5, seed=5)
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    s = gpu.Selector(dev(A32), m, k_max=k, r_max=r)
    s.project_sign(7, r, density=d)
    idx, obj, ns, st = s.select(k)
    Bref = rng.project_sign(Av, 7, d, r)
    ref = oracle.select(f64cs(Av), m, k, B=f64cs(Bref))
    assert ns == k and np.min(ref["gap"]) > 1e-3
    assert list(idx) == list(ref["idx"])
    np.testing.assert_allclose(obj, ref["obj"], rtol=1e-5)


def test_sign_argument_errors(gpu):
    import torch
    m, n = 64, 300
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 8, 0.1, seed=1))
    s = gpu.Selector(dev(A32), m, k_max=4, r_max=16)
    B = torch.empty(16, 64, dtype=torch.float32, device="cuda")
    for dd, rr in [(0.0, 8), (1.5, 8), (float("nan"), 8), (0.5, 17), (0.5, 0)]:
        with pytest.raises(gpu.GcssError) as e:
            gpu.project_sign(s.h, 1, dd, rr, B.data_ptr(), 64)
        assert e.value.status == gpu.ERR_ARG
