"""GPU selections against the FP64 oracle's own selections on the workload
configurations (Algorithms 1, 3 and 4), not only on the small cases:

* the batched workload in full: 64 blocks of uneven width (m = 1024, about
  1.1 M columns), one shared B = A Omega (r = 128), 20 picks per block, merge
  of 100, binary32 and bfloat16 storage;
* the other workloads on a leading column slice of the configured matrix
  (same m, storage type, target kind and generator, so the same streaming
  kernel as the full size): A 4096 x 8192 of the 4096 x 65536 B = A workload
  (k = 200), A 2048 x 131072 of the 2048 x 2^20 projection workload in
  binary32 and bfloat16 (r = 256, k = 100), A 8192 x 16384 of the FP8 E4M3
  workload (r = 512 stored in bfloat16 as configured, k = 500).

The oracle runs on the stored values (decoded bfloat16 / E4M3 codes from its
own quantizer, which must equal the GPU's codes) and on the same target B,
formed on the host in FP64 as A_s Omega_s and rounded once to binary32
(then to bfloat16 where the workload stores B so).
Checks (the benchmark spec tolerances, binary32 arithmetic on the GPU):
  * A1: identical picks up to the first step whose oracle score gap
    (s1 - s2)/s1 is below 1e-4;
  * A2: ||B - P_S B||^2 of the GPU's picks within relative 1e-5 of the
    oracle picks', both evaluated by the oracle in FP64;
  * A3: the GPU's objective F_t equals the FP64 error of its first t picks
    (relative 1e-5), and the oracle's F_t where the picks agree.
For Algorithm 4 each block is compared with the oracle on that block, and
the merge with the oracle run on the GPU's own pool of block picks.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import dense
import synth
from tests.gpu_util import rel

pytestmark = pytest.mark.gpu

DELTA = 1e-4
TOL = 1e-5


def _sep(gap, k):
    small = np.nonzero(gap[:k] < DELTA)[0]
    return int(small[0]) if small.size else k


def _prefix(a, b):
    n = 0
    for x, y in zip(a, b):
        if int(x) != int(y):
            break
        n += 1
    return n


def _host_cs(A, m, rows=None):
    """GPU column store rows -> float64 (c, m) host column store (ld = m)."""
    X = A if rows is None else A[rows]
    return np.ascontiguousarray(X[:, :m].double().cpu().numpy())


def _stored_host(A32, m, dt, sl):
    """The values the selection streams for columns sl of the binary32 store
    A32 (GPU), as the oracle's quantizer stores them; plus the GPU's codes
    for the same columns, which must be identical."""
    import paper_1312_6838_amd as g
    import torch
    a32 = np.ascontiguousarray(A32[sl].cpu().numpy())
    if dt == "f32":
        return np.ascontiguousarray(a32[:, :m].astype(np.float64)), A32[sl].contiguous(), None
    if dt == "bf16":
        codes = oracle.quantize_bf16(a32, m)
        dcodes, _ = g.quantize_tensor(A32[sl].contiguous(), m, "bf16")
        gc = dcodes.cpu().numpy().view(np.uint16)
        assert np.array_equal(gc[:, :m], codes[:, :m])
        return oracle.decode_columns(codes, m, "bf16"), dcodes, None
    codes, scl = oracle.quantize_fp8(a32, m)
    dcodes, dsc = g.quantize_tensor(A32[sl].contiguous(), m, "fp8")
    assert np.array_equal(dcodes.cpu().numpy()[:, :m], codes[:, :m])
    assert np.array_equal(dsc.cpu().numpy(), scl)
    return oracle.decode_columns(codes, m, "fp8", scl), dcodes, dsc


def _target(Acs, m, Om, ldb, bdt="f32"):
    """B = A Omega in FP64 (oracle definition), rounded once to binary32 (and,
    for a bfloat16 target, from there to bfloat16 by the oracle's encoder):
    host values (r, m) float64 and the GPU column store (r, ldb)."""
    import torch
    B64 = dense.project(Acs, m, Om.astype(np.float64), chunk=16384)       # m x r
    B32 = B64.astype(np.float32)
    Bcs = np.zeros((B32.shape[1], ldb), dtype=np.float32)
    Bcs[:, :m] = B32.T
    if bdt == "bf16":
        codes = oracle.quantize_bf16(Bcs, m, ldo=ldb)
        vals = oracle.decode_columns(codes, m, "bf16")
        return vals, torch.from_numpy(codes.view(np.int16)).cuda().view(torch.bfloat16)
    return np.ascontiguousarray(B32.T.astype(np.float64)), torch.from_numpy(Bcs).cuda()


def _check_selection(idx, obj, ns, Acs, m, k, Bh):
    ref = oracle.select(Acs, m, k, B=Bh)
    assert ns == ref["n_selected"] == k
    sep = _sep(ref["gap"], k)
    got = _prefix(idx, ref["idx"])
    print(f"matched prefix {got} (oracle gap below {DELTA} first at step {sep}; "
          f"min gap {ref['gap'][:k].min():.2e})")
    assert got >= sep
    e_gpu = oracle.error(Acs, m, idx, B=Bh)
    e_orc = oracle.error(Acs, m, ref["idx"], B=Bh)
    print(f"error of GPU picks {e_gpu!r}, of oracle picks {e_orc!r}")
    assert rel(e_gpu, e_orc) <= TOL
    np.testing.assert_allclose(obj[:got + 1], ref["obj"][:got + 1], rtol=TOL)
    for t in sorted({1, k // 4, k // 2, k}):
        assert rel(obj[t], oracle.error(Acs, m, idx[:t], B=Bh)) <= TOL, t
    assert np.all(np.diff(obj) <= 0)


@pytest.mark.parametrize("name,dt,ns", [
    ("css_4096x65536_k200", "f32", 8192),
    ("gcss_2048x1048576_r256_k100", "f32", 131072),
    ("gcss_2048x1048576_r256_k100", "bf16", 131072),
    ("gcss_fp8_8192x262144_r512_k500", "fp8", 16384),
])
def test_config_slice_matches_oracle(gpu, name, dt, ns):
    import torch
    w = synth.workload(name)
    m, n, k = w["m"], w["n"], w["k"]
    A32 = synth.spectral_lowrank_torch(m, n, w["rank"], w["decay"], w["noise"], seed=0)
    sl = slice(0, ns)
    Acs, Adev, sc = _stored_host(A32, m, dt, sl)
    if w["target"] == "self":
        del A32
        s = gpu.Selector(Adev, m, k_max=k, self_target=True, scales=sc)
        s.set_target(None)
        Bh = None
    else:
        Om = synth.omega_gauss_torch(n, w["r"], seed=1)[sl].cpu().numpy()
        del A32
        Bh, Bdev = _target(Acs, m, Om, synth.lda_for(m, 4), w.get("b_dtype", "f32"))
        s = gpu.Selector(Adev, m, k_max=k, r_max=w["r"], scales=sc)
        s.set_target(Bdev)
    torch.cuda.synchronize()
    idx, obj, nsel, st = s.select(k)
    s.close()
    _check_selection(idx, obj, nsel, Acs, m, k, Bh)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_batched_workload_in_full_matches_oracle(gpu, dt):
    import torch
    name = "batched_1024_64blocks_r128"
    w = synth.workload(name)
    m, r, kb, km = w["m"], w["r"], w["k_block"], w["k_merge"]
    widths = synth.block_widths(w["nblocks"], w["wlo"], w["whi"], 0)
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    nb = len(widths)
    A32 = synth.gauss_lowrank_torch(m, n, w["rank"], w["noise"], 0, scale=1.0 / math.sqrt(w["rank"]))
    Om = synth.omega_gauss_torch(n, r, 1).cpu().numpy()
    Acs, Adev, sc = _stored_host(A32, m, dt, slice(0, n))
    del A32
    Bh, Bdev = _target(Acs, m, Om, synth.lda_for(m, 4))
    del Om
    s = gpu.Selector(Adev, m, k_max=kb, r_max=r, scales=sc, batched=(nb, kb, km))
    s.set_target(Bdev)
    ib, im, om, nm, st = s.select_batched(off, kb, km)
    s.close()
    del Adev
    torch.cuda.synchronize()
    assert st == gpu.OK and nm == km and np.all(ib >= 0)
    # every block against the oracle on that block
    short = []
    for b in range(nb):
        rb = oracle.select(Acs[off[b]:off[b + 1]], m, kb, B=Bh)
        sep = _sep(rb["gap"], kb)
        got = _prefix(ib[b] - off[b], rb["idx"])
        short.append((got, sep))
        assert got >= sep, (b, got, sep)
        assert rel(oracle.error(Acs[off[b]:off[b + 1]], m, ib[b] - off[b], B=Bh),
                   oracle.error(Acs[off[b]:off[b + 1]], m, rb["idx"], B=Bh)) <= TOL, b
    print(f"blocks: matched prefix >= gap rule in all {nb}; "
          f"full match in {sum(1 for g_, _ in short if g_ == kb)}")
    # the merge against the oracle on the GPU's own pool (block order, pick order)
    pool = [int(x) for x in ib.ravel()]
    rm = oracle.select(np.ascontiguousarray(Acs[pool]), m, km, B=Bh)
    sep = _sep(rm["gap"], km)
    got = _prefix(im, [pool[i] for i in rm["idx"]])
    print(f"merge: matched prefix {got} (gap rule {sep})")
    assert got >= sep
    np.testing.assert_allclose(om[:got + 1], rm["obj"][:got + 1], rtol=TOL)
    for t in (1, km // 2, km):
        assert rel(om[t], oracle.error(Acs, m, im[:t], B=Bh)) <= TOL, t
    # Algorithm 4 composed by the oracle from scratch: the merged picks' error
    ref = oracle.select_distributed(Acs, m, Bh, off, kb, km)
    e_gpu = oracle.error(Acs, m, im, B=Bh)
    e_orc = oracle.error(Acs, m, ref["idx_merge"], B=Bh)
    print(f"merged error: GPU {e_gpu!r}, oracle {e_orc!r}")
    assert rel(e_gpu, e_orc) <= TOL
