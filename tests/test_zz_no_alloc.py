"""The entry point that allocates no device memory (gcss_select_static)
against the context path it is a variant of (gcss_create, gcss_set_target,
gcss_select_async with a caller workspace), through the C ABI: two calls in
a row on the one static array, the second on a smaller input, and a problem
too large for the array."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import colstore32, dev, f64cs, stored_dense

pytestmark = pytest.mark.gpu


def _context_path(gpu, Adev, m, k, Bdev):
    import torch
    r = 0 if Bdev is None else int(Bdev.shape[0])
    s = gpu.Selector(Adev, m, k_max=k, r_max=r, self_target=Bdev is None)
    s.set_target(Bdev)
    out = s.select_async(k)
    torch.cuda.synchronize()
    res = [o.cpu().numpy() for o in out]
    s.close()
    return res


def _static_path(gpu, Adev, m, k, Bdev):
    import torch
    out = gpu.select_static_tensor(Adev, m, k, Bdev)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def test_static_selection_matches_context_path_twice(gpu):
    import torch
    # call 1: explicit target B = A Omega, 300 x 5000, k = 16
    m1, n1, k1, r1 = 300, 5000, 16, 64
    A1, _ = synth.planted_dense(m1, n1, k1, 1.5, seed=31)
    A1c = colstore32(A1)
    A1v = stored_dense(A1c, m1)
    B1v = stored_dense(colstore32(A1v @ synth.omega_gauss(n1, r1, seed=32).astype(np.float64)), m1)
    A1d, B1d = dev(A1c), dev(colstore32(B1v))
    got1 = _static_path(gpu, A1d, m1, k1, B1d)
    # call 2, on the array call 1 left behind: a smaller problem, B = A
    m2, n2, k2 = 200, 1500, 7
    A2, _ = synth.planted_dense(m2, n2, k2, 1.5, seed=33)
    A2c = colstore32(A2)
    A2d = dev(A2c)
    got2 = _static_path(gpu, A2d, m2, k2, None)
    torch.cuda.synchronize()

    ref1 = _context_path(gpu, A1d, m1, k1, B1d)
    ref2 = _context_path(gpu, A2d, m2, k2, None)
    for got, ref, k in ((got1, ref1, k1), (got2, ref2, k2)):
        assert int(got[2][0]) == int(ref[2][0]) == k
        assert np.array_equal(got[0], ref[0])
        # same kernels, same launch setting: the objective agrees bit for bit
        assert np.array_equal(got[1].view(np.int64), ref[1].view(np.int64))
    # and both agree with the oracle on these separated-gap inputs
    o1 = oracle.select(f64cs(A1v), m1, k1, B=f64cs(B1v))
    o2 = oracle.select(f64cs(stored_dense(A2c, m2)), m2, k2)
    assert list(got1[0]) == list(o1["idx"]) and list(got2[0]) == list(o2["idx"])
    np.testing.assert_allclose(got1[1], o1["obj"], rtol=1e-5)
    np.testing.assert_allclose(got2[1], o2["obj"], rtol=1e-5)


def test_static_selection_rejects_a_problem_beyond_the_array(gpu):
    import torch
    A = torch.zeros(16, 64, dtype=torch.float32, device="cuda")
    desc = gpu.make_desc(64, 4_000_000, 64, gpu.F32, A.data_ptr(), None, 8, 16, False)
    need = gpu.workspace_size(desc)
    assert need > gpu.STATIC_SCRATCH_BYTES
    idx = torch.empty(8, dtype=torch.int64, device="cuda")
    with pytest.raises(gpu.GcssError) as ei:
        gpu.select_static(desc, A.data_ptr(), 16, 64, 8, idx.data_ptr(), None, None)
    assert ei.value.status == gpu.ERR_UNSUPPORTED
    assert str(need) in str(ei.value)
