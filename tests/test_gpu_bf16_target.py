"""A bfloat16 target B (the FP8 workload's configuration: B = A Omega stored
in bfloat16).  The target is the matrix of its bfloat16 values: the oracle
runs on those values decoded by its own bfloat16 decoder."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import colstore32, dev, f64cs, rel, stored_dense

pytestmark = pytest.mark.gpu


def _bf16_store(Bv):
    """m x r float64 -> (GPU bfloat16 column store, the values it holds as
    m x r float64), rounded to binary32 then to bfloat16 by the oracle's
    encoder."""
    import torch
    m = Bv.shape[0]
    b32 = colstore32(Bv)
    codes = oracle.quantize_bf16(b32, m, ldo=b32.shape[1])
    vals = oracle.decode_columns(codes, m, "bf16").T
    t = torch.from_numpy(codes.view(np.int16)).cuda().view(torch.bfloat16)
    return t, vals


@pytest.mark.parametrize("dt", ["f32", "fp8"])
def test_bf16_target_planted_matches_oracle(gpu, dt):
    m, n, k, r = 512, 4000, 10, 128
    A, _ = synth.planted_dense(m, n, k, 1.5, seed=7)
    A32 = colstore32(A)
    if dt == "f32":
        Adev, sc, Av = dev(A32), None, stored_dense(A32, m)
    else:
        Adev, sc = gpu.quantize_tensor(dev(A32), m, "fp8")
        codes, scl = oracle.quantize_fp8(A32, m)
        Av = oracle.decode_columns(codes, m, "fp8", scl).T
    Bt, Bv = _bf16_store(Av @ synth.omega_gauss(n, r, seed=8).astype(np.float64))
    s = gpu.Selector(Adev, m, k_max=k, r_max=r, scales=sc)
    s.set_target(Bt)
    # the context holds the target's values exactly
    Bread = s.read(gpu.STATE_B, m * r, np.float32).reshape(r, m).T.astype(np.float64)
    assert np.array_equal(Bread, Bv)
    f0 = s.read(gpu.STATE_F0, n, np.float64)
    fr, _ = oracle.init_scores(f64cs(Av), m, B=f64cs(Bv))
    np.testing.assert_allclose(f0, fr, rtol=1e-4, atol=1e-6 * fr.max())
    idx, obj, ns, st = s.select(k)
    ref = oracle.select(f64cs(Av), m, k, B=f64cs(Bv))
    assert np.min(ref["gap"]) > 1e-3
    assert list(idx) == list(ref["idx"])
    np.testing.assert_allclose(obj, ref["obj"], rtol=1e-5)
    assert rel(s.reconstruction_error(idx), oracle.error(f64cs(Av), m, idx, B=f64cs(Bv))) <= 1e-5
    s.close()


@pytest.mark.parametrize("m,n,r", [(300, 2000, 64), (1000, 3000, 256)])
def test_bf16_projection_is_the_rounded_binary32_projection(gpu, m, n, r):
    """project_target with a bfloat16 output holds, bit for bit, the nearest
    bfloat16 (ties to even, the oracle's encoder) of the binary32 projection
    the same context computes; rows m..ldb-1 are zero; the selection then
    runs on those values."""
    import torch
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 20, 0.1, seed=m))
    Om = dev(synth.omega_gauss(n, r, seed=r))
    s = gpu.Selector(dev(A32), m, k_max=6, r_max=r)
    B32 = s.project_target(Om).cpu().numpy()
    Bh = s.project_target(Om, b_dtype="bf16")
    assert Bh.dtype == torch.bfloat16
    codes = Bh.view(torch.int16).cpu().numpy().view(np.uint16)
    ref = oracle.quantize_bf16(B32, m, ldo=B32.shape[1])
    assert np.array_equal(codes, ref)
    Bv = oracle.decode_columns(codes, m, "bf16").T
    idx, obj, ns, st = s.select(6)
    Av = stored_dense(A32, m)
    assert rel(obj[-1], oracle.error(f64cs(Av), m, idx, B=f64cs(Bv))) <= 1e-5
    s.close()
