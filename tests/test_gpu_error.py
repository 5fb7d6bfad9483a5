"""Reconstruction error of an explicit target (Problem 5's objective
||B - P_S B||_F^2 for a given set of picks) on the GPU against the oracle's
Householder-QR error: tiled FP64 passes over Q^T B and the residual, at
shapes with ragged row and column tiles, one and several row splits, no
picks, one pick and more picks than one tile of the basis holds."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import colstore32, dev, f64cs, rel, stored_dense

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,r,k", [
    (100, 300, 7, 0), (100, 300, 7, 1), (257, 900, 65, 33), (640, 1500, 64, 64),
    (1000, 2000, 130, 150), (4099, 1200, 200, 97), (8192, 700, 96, 300),
])
def test_error_matches_oracle(gpu, m, n, r, k):
    rng = np.random.default_rng(m + r + k)
    A = rng.standard_normal((m, n))
    A32 = colstore32(A)
    Av = stored_dense(A32, m)
    Bd = colstore32(rng.standard_normal((m, r)))
    Bv = stored_dense(Bd, m)
    s = gpu.Selector(dev(A32), m, k_max=max(k, 1), r_max=r)
    s.set_target(dev(Bd))
    idx = rng.choice(n, size=k, replace=False).astype(np.int64)
    e = s.reconstruction_error(idx)
    ref = oracle.error(f64cs(Av), m, idx, B=f64cs(Bv))
    # both FP64 residuals of well-conditioned picks (Gaussian columns)
    assert rel(e, ref) <= 1e-10, (e, ref)
    if k == 0:
        assert rel(e, float(np.sum(Bv ** 2))) <= 1e-12
    s.close()
