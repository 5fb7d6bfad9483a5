"""The C-ABI library loads, exports every declared entry point and rejects bad
arguments before touching a device.  No compute calls: runs without a GPU."""
import ctypes
import os
import re

import pytest

import paper_1312_6838_amd as g
from paper_1312_6838_amd import _abi

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gcss.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gcss_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = g.load()
    names = declared_functions()
    assert "gcss_select" in names and len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_abi.EXPORTS) == names


def test_version_and_error_string():
    assert "gfx950" in g.version()
    d = g.make_desc(0, 10, 16, g.F32, 0x1000, None, 1, 4, False)
    with pytest.raises(g.GcssError) as ei:
        g.workspace_size(d)
    assert ei.value.status == g.ERR_ARG
    assert "m and n" in g.last_error()


def _desc(**kw):
    base = dict(m=100, n=1000, lda=128, a_dtype=g.F32, a_ptr=0x10000, scale_ptr=None, k_max=10,
                r_max=16, self_target=False)
    base.update(kw)
    return g.make_desc(base["m"], base["n"], base["lda"], base["a_dtype"], base["a_ptr"],
                       base["scale_ptr"], base["k_max"], base["r_max"], base["self_target"])


def test_workspace_size_valid_and_monotone():
    s1 = g.workspace_size(_desc())
    s2 = g.workspace_size(_desc(n=100000))
    s3 = g.workspace_size(_desc(self_target=True))
    assert 0 < s1 < s2 and s1 < s3
    assert s1 % 256 == 0


@pytest.mark.parametrize("kw,status", [
    (dict(m=0), g.ERR_ARG),
    (dict(lda=50), g.ERR_ARG),            # lda < m
    (dict(lda=101), g.ERR_ARG),           # lda * 4 not a multiple of 16
    (dict(k_max=0), g.ERR_ARG),
    (dict(k_max=1001), g.ERR_ARG),        # k_max > n
    (dict(a_dtype=7), g.ERR_ARG),
    (dict(r_max=0, self_target=False), g.ERR_ARG),
    (dict(m=9000, lda=9008), g.ERR_UNSUPPORTED),
    (dict(a_dtype=g.BF16, lda=100), g.ERR_ARG),  # 200 bytes, not a multiple of 16
])
def test_workspace_size_rejects(kw, status):
    with pytest.raises(g.GcssError) as ei:
        g.workspace_size(_desc(**kw))
    assert ei.value.status == status


def test_create_checks_arguments_first():
    lib = g.load()
    h = ctypes.c_void_p(0)
    d = _desc(a_ptr=None)
    assert lib.gcss_create(ctypes.byref(d), None, 0, ctypes.byref(h)) == g.ERR_ARG
    d = _desc(a_ptr=0x10008)  # misaligned A
    assert lib.gcss_create(ctypes.byref(d), None, 0, ctypes.byref(h)) == g.ERR_ARG
    d = _desc(a_dtype=g.FP8_E4M3, lda=128)  # FP8 without scales
    assert lib.gcss_create(ctypes.byref(d), None, 0, ctypes.byref(h)) == g.ERR_ARG
    assert h.value is None


def test_create_without_workspace_or_device():
    lib = g.load()
    h = ctypes.c_void_p(0)
    d = _desc()
    st = lib.gcss_create(ctypes.byref(d), None, 0, ctypes.byref(h))
    # no GPU here: device error; on a GPU machine: workspace error
    assert st in (g.ERR_DEVICE, g.ERR_WORKSPACE)
    assert h.value is None


def test_null_context_calls_fail_cleanly():
    lib = g.load()
    idx = (ctypes.c_int64 * 4)()
    assert lib.gcss_select(None, 4, idx, None, None) == g.ERR_ARG
    assert lib.gcss_set_target(None, None, 0, 0, 0) == g.ERR_ARG
    err = ctypes.c_double()
    assert lib.gcss_reconstruction_error(None, idx, 1, ctypes.byref(err)) == g.ERR_ARG
    lib.gcss_destroy(None)  # NULL-safe
    assert lib.gcss_quantize(None, 1, 1, 1, g.BF16, None, 1, None, None) == g.ERR_ARG
    assert lib.gcss_quantize(0x1000, 1, 1, 1, g.F32, 0x2000, 1, None, None) == g.ERR_ARG


def test_product_package_does_not_import_the_oracle():
    import sys
    import subprocess
    code = ("import sys, paper_1312_6838_amd as g; g.load(); "
            "bad=[m for m in sys.modules if m=='oracle' or m.startswith('oracle.')]; "
            "print(bad); sys.exit(1 if bad else 0)")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def test_tuning_and_probe_check_arguments_first():
    lib = g.load()
    t = _abi.Tuning(1, 4, 64, 0)
    res = _abi.TuneResult()
    assert lib.gcss_get_tuning(None, ctypes.byref(t)) == g.ERR_ARG
    assert lib.gcss_set_tuning(None, ctypes.byref(t)) == g.ERR_ARG
    assert lib.gcss_autotune_select(None, 4, 3, None, ctypes.byref(res)) == g.ERR_ARG
    off = (ctypes.c_int64 * 3)(0, 5, 10)
    assert lib.gcss_autotune_batched(None, 2, off, 2, 2, 3, None, ctypes.byref(res)) == g.ERR_ARG
    sec = ctypes.c_double()
    sink = 0x20000
    assert lib.gcss_hbm_probe(None, 1024, sink, 1, None, ctypes.byref(sec)) == g.ERR_ARG
    assert lib.gcss_hbm_probe(0x10008, 1024, sink, 1, None, ctypes.byref(sec)) == g.ERR_ARG  # misaligned
    assert lib.gcss_hbm_probe(0x10000, 1000, sink, 1, None, ctypes.byref(sec)) == g.ERR_ARG  # not 16k bytes
    assert lib.gcss_hbm_probe(0x10000, 0, sink, 1, None, ctypes.byref(sec)) == g.ERR_ARG
    assert lib.gcss_hbm_probe(0x10000, 1024, sink, 0, None, ctypes.byref(sec)) == g.ERR_ARG  # reps
    assert lib.gcss_hbm_probe(0x10000, 1024, None, 1, None, ctypes.byref(sec)) == g.ERR_ARG
    assert g.PROBE_SINK_FLOATS == 4096


def test_static_selection_checks_arguments_before_the_device():
    """gcss_select_static validates and sizes on the host first: a null
    descriptor or a bad k is an argument error, a problem whose workspace
    exceeds the static array is unsupported, all without touching a device."""
    lib = g.load()
    assert lib.gcss_select_static(None, None, 0, 0, 0, 1, 0x1000, None, None) == g.ERR_ARG
    d = _desc()
    assert lib.gcss_select_static(ctypes.byref(d), None, 0, 0, 0, 0, 0x1000, None, None) == g.ERR_ARG
    assert lib.gcss_select_static(ctypes.byref(d), None, 0, 0, 0, 11, 0x1000, None, None) == g.ERR_ARG
    big = _desc(n=4_000_000, m=64, lda=64)
    assert g.workspace_size(big) > g.STATIC_SCRATCH_BYTES
    st = lib.gcss_select_static(ctypes.byref(big), None, 0, 0, 0, 8, 0x1000, None, None)
    assert st == g.ERR_UNSUPPORTED
    assert "static scratch" in g.last_error()
