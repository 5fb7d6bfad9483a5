"""Launch settings of the streaming passes, their autotuner, and the HBM
read probe.

A setting spreads the same per-column arithmetic differently over the chip,
so the picks, the scores and the explicit-target objectives must be bitwise
those of the default setting (the Gram target's objective decrements are
FP64 sums over per-workgroup partials, so there only the picks are bitwise
and the objective agrees to FP64 rounding).  The probe's sink must fold to
the XOR of every 32-bit word of its buffer, which holds only if each word was
read exactly once (an odd number of times, with the grid-stride indexing).
"""
import json

import numpy as np
import pytest

import synth
from tests.gpu_util import colstore32, dev, stored_dense

pytestmark = pytest.mark.gpu

SETTINGS = [
    dict(stream_pd=2, stream_upw=4),
    dict(stream_pd=1, stream_upw=1),
    dict(stream_pd=2, stream_upw=16),
    dict(stream_pd=1, stream_upw=64),
]


def _explicit(gpu, m=256, n=20011, r=32, k=24, dt="f32"):
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 40, 0.05, seed=21))
    Bcs = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=22).astype(np.float64))
    Adev, sc = dev(A32), None
    if dt != "f32":
        Adev, sc = gpu.quantize_tensor(Adev, m, dt)
    s = gpu.Selector(Adev, m, k_max=k, r_max=r, scales=sc)
    s.set_target(dev(Bcs))
    return s


@pytest.mark.parametrize("dt", ["f32", "bf16", "fp8"])
def test_settings_do_not_change_explicit_target_results(gpu, dt):
    k = 24
    s = _explicit(gpu, k=k, dt=dt)
    assert s.tuning() == dict(stream_pd=1, stream_upw=4, batch_group=64, batch_wg_per_cu=0)
    i0, o0, n0, _ = s.select(k)
    f0 = s.read(gpu.STATE_F, 20011, np.float64)
    for st in SETTINGS:
        s.tuning(**st)
        i1, o1, n1, _ = s.select(k)
        assert np.array_equal(i0, i1), st
        assert np.array_equal(o0.view(np.int64), o1.view(np.int64)), st
        assert np.array_equal(f0.view(np.int64), s.read(gpu.STATE_F, 20011, np.float64).view(np.int64)), st
        # the captured loop is captured again under the new setting
        ia, oa, na = s.select_async(k)
        assert np.array_equal(i0, ia.cpu().numpy()), st
        assert np.array_equal(o0.view(np.int64), oa.cpu().numpy().view(np.int64)), st


def test_settings_gram_target_same_picks(gpu):
    m, n, k = 192, 9001, 30
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 60, 0.05, seed=23))
    s = gpu.Selector(dev(A32), m, k_max=k, self_target=True)
    s.set_target(None)
    i0, o0, _, _ = s.select(k)
    for st in SETTINGS:
        s.tuning(**st)
        i1, o1, _, _ = s.select(k)
        assert np.array_equal(i0, i1), st
        np.testing.assert_allclose(o1, o0, rtol=1e-12, atol=1e-12 * o0[0])


def test_bad_settings_rejected(gpu):
    s = _explicit(gpu, n=3000, k=4)
    for bad in (dict(stream_pd=3), dict(stream_upw=0), dict(stream_upw=65), dict(batch_group=48),
                dict(batch_wg_per_cu=-1)):
        with pytest.raises(gpu.GcssError) as ei:
            s.tuning(**bad)
        assert ei.value.status == gpu.ERR_ARG
    assert s.tuning() == dict(stream_pd=1, stream_upw=4, batch_group=64, batch_wg_per_cu=0)


def test_autotune_select_and_cache(gpu, tmp_path):
    k = 12
    s = _explicit(gpu, k=k)
    i0, o0, _, _ = s.select(k)
    cache = str(tmp_path / "tune.json")
    r = s.autotune(k, reps=3, cache=cache)
    assert r["candidates"] == 8            # the entry setting and 7 others
    assert r["best_ms"] > 0 and r["initial_ms"] > 0 and r["best_ms"] <= r["initial_ms"]
    assert s.tuning() == r["best"]
    data = json.load(open(cache))
    key = "gfx950 select m=256 n2=15 f32 explicit"
    assert list(data) == [key]
    assert {kk: data[key][kk] for kk in r["best"]} == r["best"]
    i1, o1, _, _ = s.select(k)
    assert np.array_equal(i0, i1) and np.array_equal(o0.view(np.int64), o1.view(np.int64))
    # a second context of the same shape takes the setting from the cache
    s2 = _explicit(gpu, k=k)
    r2 = s2.autotune(k, reps=3, cache=cache)
    assert r2["candidates"] == 0 and r2["best"] == r["best"] and r2["initial_ms"] == 0.0
    assert s2.tuning() == r["best"]
    # a malformed cache file is reported, not overwritten
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    with pytest.raises(gpu.GcssError) as ei:
        s2.autotune(k, cache=str(bad))
    assert ei.value.status == gpu.ERR_ARG
    assert bad.read_text() == "{not json"


def test_autotune_needs_target(gpu):
    m, n = 64, 500
    s = gpu.Selector(dev(colstore32(np.random.default_rng(2).standard_normal((m, n)))), m,
                     k_max=4, r_max=8)
    with pytest.raises(gpu.GcssError) as ei:
        s.autotune(4)
    assert ei.value.status == gpu.ERR_STATE


def test_autotune_batched_keeps_results(gpu, tmp_path):
    m, r, kb, km = 128, 16, 6, 10
    widths = [700, 64, 1025, 300, 2000, 129]
    off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    n = int(off[-1])
    A32 = colstore32(synth.gauss_lowrank_dense(m, n, 20, 0.1, seed=14))
    Bcs = colstore32(stored_dense(A32, m) @ synth.omega_gauss(n, r, seed=15).astype(np.float64))
    s = gpu.Selector(dev(A32), m, k_max=kb, r_max=r, batched=(len(widths), kb, km))
    s.set_target(dev(Bcs))
    ib, im, om, nm, st = s.select_batched(off, kb, km)
    cache = str(tmp_path / "tune.json")
    res = s.autotune_batched(off, kb, km, reps=3, cache=cache)
    assert res["candidates"] == 9
    assert s.tuning() == res["best"]
    assert "gfx950 batched m=128 n2=13 f32 blocks=6" in json.load(open(cache))
    for g_ in (16, 32):
        s.tuning(batch_group=g_, batch_wg_per_cu=2)
        ib2, im2, om2, nm2, st2 = s.select_batched(off, kb, km)
        assert np.array_equal(ib, ib2) and np.array_equal(im, im2), g_
        assert np.array_equal(om.view(np.int64), om2.view(np.int64)), g_


@pytest.mark.parametrize("nbytes", [16, 16 * 1000003, 64 << 20])
def test_hbm_probe_reads_every_word_once(gpu, nbytes):
    import torch
    g = torch.Generator(device="cuda").manual_seed(nbytes & 0xFFFF)
    buf = torch.randint(-2**31, 2**31 - 1, (nbytes // 4,), dtype=torch.int32, device="cuda",
                        generator=g)
    sec, sink = gpu.hbm_probe_tensor(buf, reps=2)
    assert sec > 0
    words = buf.cpu().numpy().view(np.uint32)
    want = np.bitwise_xor.reduce(words) if words.size else np.uint32(0)
    got = np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32))
    assert got == want


def test_hbm_probe_rate_is_plausible(gpu):
    import torch
    buf = torch.zeros(2 << 30, dtype=torch.uint8, device="cuda")   # 2 GiB, beyond the caches
    sec, _ = gpu.hbm_probe_tensor(buf, reps=5)
    rate = buf.numel() / sec
    assert 2.0e12 < rate < 8.0e12 * 1.02, rate
