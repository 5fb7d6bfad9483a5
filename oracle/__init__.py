"""FP64 CPU oracle for greedy column subset selection -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code
with it.

Matrices are passed as *column stores*: an m x n matrix is a 2-D array of
shape (n, ld) whose row i is column i (column-major with leading dimension
ld).  ``B=None`` selects the centralized problem B = A.

Functions follow the paper (Farahat et al., "Greedy Column Subset Selection
for Large-scale Data Sets"):

* :func:`select`               Algorithm 3 / Algorithm 1 (C, FP64)
* :func:`error`                objective of Problem 1 / Problem 5 via Householder QR
* :func:`select_distributed`   Algorithm 4 on one machine
* :func:`init_scores`          initial f, g of Algorithms 1 and 3
* storage formats: bfloat16 and OCP FP8 E4M3 encode/decode and quantizers
* :mod:`oracle.brute`          numpy brute force (explicit least squares)
* :mod:`oracle.embed`          embedding W = Q^T A and the rank-k approximation
                               in span(A_S) (Section 3)
* :mod:`oracle.rng`            counter-based (Philox4x32-10) dense and sparse
                               random sign Omega and B = A Omega (Section 5.1)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gcss_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_vp = ctypes.c_void_p

EXHAUSTED = 1


def build_sanitized(out_path: str) -> str:
    """Compile the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
    with the ROCm toolchain's clang (its shared runtime, which the caller
    preloads, is the one the library's sanitized host code uses too)."""
    cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libasan",
           "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", out_path, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    lib.orc_select.restype = ctypes.c_int
    lib.orc_select.argtypes = [_vp, _i64, _i64, _i64, _vp, _i64, _i64, _i32, _dbl,
                               _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.orc_init_scores.restype = ctypes.c_int
    lib.orc_init_scores.argtypes = [_vp, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _vp]
    lib.orc_error.restype = ctypes.c_int
    lib.orc_error.argtypes = [_vp, _i64, _i64, _i64, _vp, _i32, _vp, _i64, _i64, _vp]
    lib.orc_select_distributed.restype = ctypes.c_int
    lib.orc_select_distributed.argtypes = [_vp, _i64, _i64, _i64, _vp, _i64, _i64, _i32,
                                           _vp, _i32, _vp, _i32, _dbl, _vp, _vp, _vp, _vp]
    lib.orc_bf16_decode.restype = ctypes.c_float
    lib.orc_bf16_decode.argtypes = [ctypes.c_uint16]
    lib.orc_bf16_encode.restype = ctypes.c_uint16
    lib.orc_bf16_encode.argtypes = [ctypes.c_float]
    lib.orc_fp8_decode.restype = ctypes.c_double
    lib.orc_fp8_decode.argtypes = [ctypes.c_uint8]
    lib.orc_fp8_encode.restype = ctypes.c_uint8
    lib.orc_fp8_encode.argtypes = [ctypes.c_float]
    lib.orc_quantize_fp8.restype = None
    lib.orc_quantize_fp8.argtypes = [_vp, _i64, _i64, _i64, _vp, _i64, _vp]
    lib.orc_quantize_bf16.restype = None
    lib.orc_quantize_bf16.argtypes = [_vp, _i64, _i64, _i64, _vp, _i64]
    lib.orc_decode_columns.restype = None
    lib.orc_decode_columns.argtypes = [_vp, ctypes.c_int, _i64, _i64, _i64, _vp, _vp, _i64]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    return lib


def _load():
    global _lib
    if _lib is None:
        # GCSS_ORACLE_LIBRARY: another build of the same source (the
        # sanitizer test's), loaded as is
        other = os.environ.get("GCSS_ORACLE_LIBRARY")
        if other:
            _lib = _configure(ctypes.CDLL(other))
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def source() -> str:
    """Text of the C oracle (the tests compile altered copies of it to check
    that the pins catch planted mistakes)."""
    with open(_SRC) as f:
        return f.read()


def build_variant(text: str, out_dir: str, tag: str):
    """Compile C oracle source text (e.g. a copy with a planted mistake) into
    out_dir and return the loaded library, ready to stand in for the oracle's
    own (``oracle._lib``)."""
    src = os.path.join(out_dir, f"orc_{tag}.c")
    lib = os.path.join(out_dir, f"liborc_{tag}.so")
    with open(src, "w") as f:
        f.write(text)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", lib, src,
                    "-lm"], check=True)
    return _configure(ctypes.CDLL(lib))


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def init_scores(A, m, B=None):
    """Initial scores: f_i = ||B^T A_i||^2, g_i = ||A_i||^2 (B=None: B = A)."""
    lib = _load()
    A = _f64(A)
    n, lda = A.shape
    f = np.empty(n)
    g = np.empty(n)
    if B is not None:
        B = _f64(B)
        r, ldb = B.shape
    else:
        r, ldb = 0, 0
    st = lib.orc_init_scores(_p(A), m, n, lda, _p(B), r, ldb, _p(f), _p(g))
    if st != 0:
        raise RuntimeError(f"orc_init_scores status {st}")
    return f, g


def select(A, m, k, B=None, tau=1e-10, trace=False, omega=False):
    """Algorithm 3 (or Algorithm 1 when B is None) in FP64.

    Returns a dict with idx (int64[k], -1 for missing picks), obj (F_0..F_k),
    upsn, score, gap (per step), n_selected, status, and optionally
    omega (k x n rows of W = Q^T A), fg (k x 2 x n scores before each pick)
    and g_final.
    """
    lib = _load()
    A = _f64(A)
    n, lda = A.shape
    if B is not None:
        B = _f64(B)
        r, ldb = B.shape
    else:
        r, ldb = 0, 0
    idx = np.full(k, -1, dtype=np.int64)
    obj = np.zeros(k + 1)
    upsn = np.zeros(k)
    score = np.zeros(k)
    gap = np.zeros(k)
    om = np.zeros((k, n)) if omega else None
    fg = np.zeros((k, 2, n)) if trace else None
    gfin = np.zeros(n)
    ns = _i32(0)
    st = lib.orc_select(_p(A), m, n, lda, _p(B), r, ldb, k, tau, _p(idx), _p(obj),
                        _p(upsn), _p(score), _p(gap), _p(om), _p(fg), _p(gfin),
                        ctypes.addressof(ns))
    if st < 0:
        raise RuntimeError(f"orc_select status {st}")
    out = dict(idx=idx, obj=obj, upsn=upsn, score=score, gap=gap, n_selected=ns.value,
               status=st, g_final=gfin)
    if omega:
        out["omega"] = om
    if trace:
        out["fg"] = fg
    return out


def error(A, m, idx, B=None):
    """||B - P_S B||_F^2 for S = idx (B=None: B = A), FP64 Householder QR."""
    lib = _load()
    A = _f64(A)
    n, lda = A.shape
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    idx = idx[idx >= 0]
    if B is not None:
        B = _f64(B)
        r, ldb = B.shape
    else:
        r, ldb = 0, 0
    e = np.zeros(1)
    st = lib.orc_error(_p(A), m, n, lda, _p(idx), int(idx.size), _p(B), r, ldb, _p(e))
    if st != 0:
        raise RuntimeError(f"orc_error status {st}")
    return float(e[0])


def select_distributed(A, m, B, col_off, k_block, k_merge, tau=1e-10, k_blocks=None):
    """Algorithm 4 on one machine: per-block Algorithm 3, then the merge.

    k_block: the per-block budget, or with k_blocks (one budget per block,
    each in [0, k_block]) the row length of idx_block."""
    lib = _load()
    A = _f64(A)
    B = _f64(B)
    n, lda = A.shape
    r, ldb = B.shape
    col_off = np.ascontiguousarray(np.asarray(col_off, dtype=np.int64))
    nb = col_off.size - 1
    kbs = None
    if k_blocks is not None:
        kbs = np.ascontiguousarray(np.asarray(k_blocks, dtype=np.int32))
        if kbs.size != nb:
            raise ValueError("k_blocks needs one budget per block")
    ib = np.full(nb * k_block, -1, dtype=np.int64)
    im = np.full(k_merge, -1, dtype=np.int64)
    om = np.zeros(k_merge + 1)
    nm = _i32(0)
    st = lib.orc_select_distributed(_p(A), m, n, lda, _p(B), r, ldb, nb, _p(col_off),
                                    k_block, _p(kbs), k_merge, tau, _p(ib), _p(im), _p(om),
                                    ctypes.addressof(nm))
    if st < 0:
        raise RuntimeError(f"orc_select_distributed status {st}")
    return dict(idx_block=ib.reshape(nb, k_block), idx_merge=im, obj_merge=om,
                n_merge=nm.value, status=st)


# ----------------------------------------------------------------- formats --
def bf16_decode(h: int) -> float:
    return float(_load().orc_bf16_decode(int(h)))


def bf16_encode(x: float) -> int:
    return int(_load().orc_bf16_encode(float(x)))


def fp8_decode(c: int) -> float:
    return float(_load().orc_fp8_decode(int(c)))


def fp8_encode(x: float) -> int:
    return int(_load().orc_fp8_encode(float(x)))


def quantize_fp8(A32, m, ldo=None):
    """Column store float32 (n, lda) -> (codes uint8 (n, ldo), scales float32 (n,))."""
    lib = _load()
    A32 = np.ascontiguousarray(A32, dtype=np.float32)
    n, lda = A32.shape
    ldo = lda if ldo is None else ldo
    out = np.zeros((n, ldo), dtype=np.uint8)
    sc = np.zeros(n, dtype=np.float32)
    lib.orc_quantize_fp8(_p(A32), m, n, lda, _p(out), ldo, _p(sc))
    return out, sc


def quantize_bf16(A32, m, ldo=None):
    """Column store float32 (n, lda) -> bfloat16 codes uint16 (n, ldo)."""
    lib = _load()
    A32 = np.ascontiguousarray(A32, dtype=np.float32)
    n, lda = A32.shape
    ldo = lda if ldo is None else ldo
    out = np.zeros((n, ldo), dtype=np.uint16)
    lib.orc_quantize_bf16(_p(A32), m, n, lda, _p(out), ldo)
    return out


def decode_columns(src, m, dtype, scales=None):
    """Stored column store (float32 / uint16 bf16 / uint8 fp8) -> float64 (n, m)."""
    lib = _load()
    src = np.ascontiguousarray(src)
    n, lds = src.shape
    code = {np.dtype(np.float32): 0, np.dtype(np.uint16): 1, np.dtype(np.uint8): 2}[src.dtype]
    if dtype is not None:
        assert {"f32": 0, "bf16": 1, "fp8": 2}[dtype] == code
    if code == 2:
        scales = np.ascontiguousarray(scales, dtype=np.float32)
    dst = np.zeros((n, m))
    lib.orc_decode_columns(_p(src), code, m, n, lds, _p(scales), _p(dst), m)
    return dst
