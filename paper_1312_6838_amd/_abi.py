"""ctypes binding of libgcss.so (include/gcss.h).  Argument marshalling only:
every computation runs in the HIP library.  The library is loaded from this
package's directory; a missing library raises instead of falling back.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GCSS_LIBRARY names another build of the same library (e.g. a host-sanitizer
# build for the CPU tests)
LIB_PATH = os.environ.get("GCSS_LIBRARY") or os.path.join(_HERE, "libgcss.so")

OK = 0
WARN_EXHAUSTED = 1
ERR_ARG = -1
ERR_STATE = -2
ERR_DEVICE = -3
ERR_WORKSPACE = -4
ERR_UNSUPPORTED = -5

F32 = 0
BF16 = 1
FP8_E4M3 = 2

(STATE_F0, STATE_G0, STATE_F, STATE_G, STATE_Q, STATE_Z, STATE_B, STATE_GRAM, STATE_NREJECT,
 STATE_FLAGS) = range(10)
ASYNC_SPARE_STEPS = 8

EXPORTS = [
    "gcss_workspace_size", "gcss_create", "gcss_destroy", "gcss_set_target",
    "gcss_project_target", "gcss_select", "gcss_select_async", "gcss_reconstruction_error",
    "gcss_select_batched", "gcss_batched_workspace_size", "gcss_quantize", "gcss_read_state",
    "gcss_last_error", "gcss_version", "gcss_set_profiling", "gcss_get_profile",
    "gcss_set_embedding", "gcss_qless_r", "gcss_rank_k", "gcss_project_sign", "gcss_top_eig",
    "gcss_gather_columns", "gcss_get_tuning", "gcss_set_tuning", "gcss_autotune_select",
    "gcss_autotune_batched", "gcss_hbm_probe", "gcss_select_static", "gcss_block_budgets",
    "gcss_select_batched_budgets",
]

BUDGET_UNIFORM, BUDGET_EVEN, BUDGET_NORM = 0, 1, 2
_BUDGET = {"uniform": BUDGET_UNIFORM, "even": BUDGET_EVEN, "norm": BUDGET_NORM}

STATIC_SCRATCH_BYTES = 64 << 20

PROBE_SINK_FLOATS = 4096


class GcssError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gcss status {status}: {msg}")
        self.status = status


class Desc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
        ("a_dtype", ctypes.c_int32), ("a", ctypes.c_void_p), ("a_scale", ctypes.c_void_p),
        ("k_max", ctypes.c_int32), ("r_max", ctypes.c_int64), ("self_target", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("tau", ctypes.c_double), ("stream", ctypes.c_void_p),
    ]


class Profile(ctypes.Structure):
    _fields_ = [("stream_launches", ctypes.c_int64), ("stream_ms", ctypes.c_double),
                ("selects", ctypes.c_int64), ("loop_ms", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("stream_pd", ctypes.c_int32), ("stream_upw", ctypes.c_int32),
                ("batch_group", ctypes.c_int32), ("batch_wg_per_cu", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("best", Tuning), ("best_ms", ctypes.c_double), ("initial_ms", ctypes.c_double),
                ("candidates", ctypes.c_int32)]


_lib = None
_i64, _i32, _vp, _dbl, _sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double, ctypes.c_size_t
_P = ctypes.POINTER


def load():
    """Load libgcss.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1312_6838_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    lib.gcss_workspace_size.argtypes = [_P(Desc), _P(_sz)]
    lib.gcss_workspace_size.restype = st
    lib.gcss_create.argtypes = [_P(Desc), _vp, _sz, _P(_vp)]
    lib.gcss_create.restype = st
    lib.gcss_destroy.argtypes = [_vp]
    lib.gcss_destroy.restype = None
    lib.gcss_set_target.argtypes = [_vp, _vp, _i32, _i64, _i64]
    lib.gcss_set_target.restype = st
    lib.gcss_project_target.argtypes = [_vp, _vp, _i64, _vp, _i32, _i64]
    lib.gcss_project_target.restype = st
    lib.gcss_select.argtypes = [_vp, _i32, _vp, _vp, _vp]
    lib.gcss_select.restype = st
    lib.gcss_select_async.argtypes = [_vp, _i32, _vp, _vp, _vp]
    lib.gcss_select_async.restype = st
    lib.gcss_reconstruction_error.argtypes = [_vp, _vp, _i32, _vp]
    lib.gcss_reconstruction_error.restype = st
    lib.gcss_select_batched.argtypes = [_vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp, _vp]
    lib.gcss_select_batched.restype = st
    lib.gcss_select_batched_budgets.argtypes = [_vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp]
    lib.gcss_select_batched_budgets.restype = st
    lib.gcss_block_budgets.argtypes = [_vp, _i32, _vp, _vp, _i32, _i32, _vp]
    lib.gcss_block_budgets.restype = st
    lib.gcss_batched_workspace_size.argtypes = [_P(Desc), _i32, _i32, _i32, _P(_sz)]
    lib.gcss_batched_workspace_size.restype = st
    lib.gcss_quantize.argtypes = [_vp, _i64, _i64, _i64, _i32, _vp, _i64, _vp, _vp]
    lib.gcss_quantize.restype = st
    lib.gcss_read_state.argtypes = [_vp, _i32, _vp, _sz, _P(_sz)]
    lib.gcss_read_state.restype = st
    lib.gcss_set_embedding.argtypes = [_vp, _vp, _i64]
    lib.gcss_set_embedding.restype = st
    lib.gcss_qless_r.argtypes = [_vp, _i64, _i64, _vp, _i32, _vp, _i64, _vp]
    lib.gcss_qless_r.restype = st
    lib.gcss_rank_k.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _i64, _vp, _i64, _vp, _vp]
    lib.gcss_rank_k.restype = st
    lib.gcss_project_sign.argtypes = [_vp, ctypes.c_uint64, _dbl, _i64, _vp, _i64]
    lib.gcss_project_sign.restype = st
    lib.gcss_top_eig.argtypes = [_vp, _i32, _i32, _dbl, ctypes.c_uint64, _i32, _vp, _vp, _i64, _vp,
                                 _i64, _vp, _vp]
    lib.gcss_top_eig.restype = st
    lib.gcss_gather_columns.argtypes = [_vp, _vp, _i64, _vp, _vp]
    lib.gcss_gather_columns.restype = st
    lib.gcss_set_profiling.argtypes = [_vp, _i32]
    lib.gcss_set_profiling.restype = st
    lib.gcss_get_profile.argtypes = [_vp, _P(Profile)]
    lib.gcss_get_profile.restype = st
    lib.gcss_get_tuning.argtypes = [_vp, _P(Tuning)]
    lib.gcss_get_tuning.restype = st
    lib.gcss_set_tuning.argtypes = [_vp, _P(Tuning)]
    lib.gcss_set_tuning.restype = st
    lib.gcss_autotune_select.argtypes = [_vp, _i32, _i32, ctypes.c_char_p, _P(TuneResult)]
    lib.gcss_autotune_select.restype = st
    lib.gcss_autotune_batched.argtypes = [_vp, _i32, _vp, _i32, _i32, _i32, ctypes.c_char_p,
                                          _P(TuneResult)]
    lib.gcss_autotune_batched.restype = st
    lib.gcss_hbm_probe.argtypes = [_vp, _sz, _vp, _i32, _vp, _P(_dbl)]
    lib.gcss_hbm_probe.restype = st
    lib.gcss_select_static.argtypes = [_P(Desc), _vp, _i32, _i64, _i64, _i32, _vp, _vp, _vp]
    lib.gcss_select_static.restype = st
    lib.gcss_last_error.argtypes = []
    lib.gcss_last_error.restype = ctypes.c_char_p
    lib.gcss_version.argtypes = []
    lib.gcss_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    return load().gcss_last_error().decode()


def version() -> str:
    return load().gcss_version().decode()


def _check(status, allow=(OK,)):
    if status not in allow:
        raise GcssError(status, last_error())
    return status


def make_desc(m, n, lda, a_dtype, a_ptr, scale_ptr, k_max, r_max, self_target, tau=0.0,
              stream=0) -> Desc:
    return Desc(m, n, lda, a_dtype, a_ptr, scale_ptr, k_max, r_max, int(bool(self_target)), 0,
                float(tau), stream)


def workspace_size(desc: Desc) -> int:
    out = _sz(0)
    _check(load().gcss_workspace_size(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def create(desc: Desc, ws_ptr: int, ws_bytes: int) -> int:
    h = _vp(0)
    _check(load().gcss_create(ctypes.byref(desc), ws_ptr, ws_bytes, ctypes.byref(h)))
    return h.value


def destroy(h: int) -> None:
    load().gcss_destroy(h)


def set_target(h: int, b_ptr: int | None, r: int, ldb: int, b_dtype: int = F32) -> None:
    _check(load().gcss_set_target(h, b_ptr, b_dtype, r, ldb))


def project_target(h: int, omega_ptr: int, r: int, b_ptr: int, ldb: int, b_dtype: int = F32) -> None:
    _check(load().gcss_project_target(h, omega_ptr, r, b_ptr, b_dtype, ldb))


def select(h: int, k: int):
    """Returns (idx int64[k], objective float64[k+1], n_selected, status)."""
    idx = np.full(k, -1, dtype=np.int64)
    obj = np.zeros(k + 1, dtype=np.float64)
    ns = _i32(0)
    s = _check(load().gcss_select(h, k, idx.ctypes.data, obj.ctypes.data, ctypes.byref(ns)),
               allow=(OK, WARN_EXHAUSTED))
    return idx, obj, ns.value, s


def select_async(h: int, k: int, d_idx: int, d_obj: int | None, d_nsel: int | None) -> None:
    _check(load().gcss_select_async(h, k, d_idx, d_obj, d_nsel))


def select_static(desc: Desc, b_ptr: int | None, r: int, ldb: int, k: int, d_idx: int,
                  d_obj: int | None, d_nsel: int | None, b_dtype: int = F32) -> None:
    """The selection without device allocation (workspace in the library's
    static device array); device outputs, no synchronisation."""
    _check(load().gcss_select_static(ctypes.byref(desc), b_ptr, b_dtype, r, ldb, k, d_idx, d_obj,
                                     d_nsel))


def reconstruction_error(h: int, idx) -> float:
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    err = ctypes.c_double(0.0)
    _check(load().gcss_reconstruction_error(h, idx.ctypes.data if idx.size else None,
                                            int(idx.size), ctypes.byref(err)))
    return err.value


def batched_workspace_size(desc: Desc, nblocks: int, k_block: int, k_merge: int) -> int:
    out = _sz(0)
    _check(load().gcss_batched_workspace_size(ctypes.byref(desc), nblocks, k_block, k_merge,
                                              ctypes.byref(out)))
    return out.value


def select_batched(h: int, col_off, k_block: int, k_merge: int):
    """Returns (idx_block (nblocks, k_block), idx_merge, obj_merge, n_merge, status)."""
    col_off = np.ascontiguousarray(np.asarray(col_off, dtype=np.int64))
    nb = col_off.size - 1
    ib = np.full(nb * k_block, -1, dtype=np.int64)
    im = np.full(k_merge, -1, dtype=np.int64)
    om = np.zeros(k_merge + 1, dtype=np.float64)
    nm = _i32(0)
    s = _check(load().gcss_select_batched(h, nb, col_off.ctypes.data, k_block, k_merge,
                                          ib.ctypes.data, im.ctypes.data, om.ctypes.data,
                                          ctypes.byref(nm)), allow=(OK, WARN_EXHAUSTED))
    return ib.reshape(nb, k_block), im, om, nm.value, s


def select_batched_budgets(h: int, col_off, k_blocks, k_merge: int):
    """Algorithm 4 with budget k_blocks[b] for block b.  Returns
    (idx_block (nblocks, max budget), idx_merge, obj_merge, n_merge, status)."""
    col_off = np.ascontiguousarray(np.asarray(col_off, dtype=np.int64))
    kb = np.ascontiguousarray(np.asarray(k_blocks, dtype=np.int32))
    nb = col_off.size - 1
    if kb.size != nb:
        raise ValueError("one budget per block")
    kmax = int(kb.max()) if kb.size else 0
    ib = np.full(nb * max(kmax, 1), -1, dtype=np.int64)
    im = np.full(max(k_merge, 1), -1, dtype=np.int64)
    om = np.zeros(max(k_merge, 1) + 1, dtype=np.float64)
    nm = _i32(0)
    s = _check(load().gcss_select_batched_budgets(h, nb, col_off.ctypes.data, kb.ctypes.data,
                                                  k_merge, ib.ctypes.data, im.ctypes.data,
                                                  om.ctypes.data, ctypes.byref(nm)),
               allow=(OK, WARN_EXHAUSTED))
    return ib.reshape(nb, max(kmax, 1)), im[:k_merge], om[:k_merge + 1], nm.value, s


def block_budgets(h, col_off, l: int, policy: str, norms2=None):
    """Per-block budgets of Algorithm 4 (policy 'uniform', 'even' or 'norm');
    norms2 None takes the block norms from context h.  Returns int32 array."""
    col_off = np.ascontiguousarray(np.asarray(col_off, dtype=np.int64))
    nb = col_off.size - 1
    out = np.zeros(max(nb, 1), dtype=np.int32)
    nrm = None
    if norms2 is not None:
        nrm = np.ascontiguousarray(np.asarray(norms2, dtype=np.float64))
    _check(load().gcss_block_budgets(h, nb, col_off.ctypes.data,
                                     nrm.ctypes.data if nrm is not None else None, int(l),
                                     _BUDGET[policy], out.ctypes.data))
    return out[:nb]


def quantize(a_ptr: int, m: int, n: int, lda: int, dtype: int, out_ptr: int, ldo: int,
             scales_ptr: int | None, stream: int = 0) -> None:
    _check(load().gcss_quantize(a_ptr, m, n, lda, dtype, out_ptr, ldo, scales_ptr, stream))


def read_state(h: int, item: int, nbytes: int) -> bytes:
    buf = (ctypes.c_char * nbytes)()
    got = _sz(0)
    _check(load().gcss_read_state(h, item, buf, nbytes, ctypes.byref(got)))
    return bytes(buf[: got.value])


def project_sign(h: int, seed: int, density: float, r: int, b_ptr: int, ldb: int) -> None:
    _check(load().gcss_project_sign(h, int(seed) & 0xFFFFFFFFFFFFFFFF, float(density), r, b_ptr,
                                    ldb))


def top_eig(h: int, s: int, max_iters: int, tol: float, seed: int, k: int, u_ptr: int | None,
            ldu: int, b_ptr: int | None = None, ldb: int = 0):
    """-> (lambda float64[k], iterations, last relative change)"""
    lam = np.zeros(k, dtype=np.float64)
    it = _i32(0)
    ch = ctypes.c_double(0.0)
    _check(load().gcss_top_eig(h, s, max_iters, float(tol), int(seed) & 0xFFFFFFFFFFFFFFFF, k,
                               lam.ctypes.data, u_ptr, ldu, b_ptr, ldb, ctypes.byref(it),
                               ctypes.byref(ch)))
    return lam, it.value, ch.value


def gather_columns(h: int, idx_ptr: int, count: int, out_ptr: int, scales_ptr: int | None) -> None:
    _check(load().gcss_gather_columns(h, idx_ptr, count, out_ptr, scales_ptr))


def set_embedding(h: int, w_ptr: int | None, ldw: int) -> None:
    _check(load().gcss_set_embedding(h, w_ptr, ldw))


def qless_r(w_ptr: int, n: int, ldw: int, idx_ptr: int, k: int, r_ptr: int, ldr: int,
            stream: int = 0) -> None:
    _check(load().gcss_qless_r(w_ptr, n, ldw, idx_ptr, k, r_ptr, ldr, stream))


def rank_k(h: int, w_ptr: int, ldw: int, l: int, k: int, u_ptr: int | None, ldu: int,
           v_ptr: int | None, ldv: int):
    """-> (sigma float64[k], err)"""
    sigma = np.zeros(k, dtype=np.float64)
    err = ctypes.c_double(0.0)
    _check(load().gcss_rank_k(h, w_ptr, ldw, l, k, u_ptr, ldu, v_ptr, ldv, sigma.ctypes.data,
                              ctypes.byref(err)))
    return sigma, err.value


def set_profiling(h: int, enable: bool) -> None:
    _check(load().gcss_set_profiling(h, int(bool(enable))))


def get_profile(h: int) -> dict:
    p = Profile()
    _check(load().gcss_get_profile(h, ctypes.byref(p)))
    return dict(stream_launches=p.stream_launches, stream_ms=p.stream_ms, selects=p.selects,
                loop_ms=p.loop_ms)


def _tuning_dict(t: Tuning) -> dict:
    return dict(stream_pd=t.stream_pd, stream_upw=t.stream_upw, batch_group=t.batch_group,
                batch_wg_per_cu=t.batch_wg_per_cu)


def get_tuning(h: int) -> dict:
    t = Tuning()
    _check(load().gcss_get_tuning(h, ctypes.byref(t)))
    return _tuning_dict(t)


def set_tuning(h: int, stream_pd: int, stream_upw: int, batch_group: int,
               batch_wg_per_cu: int) -> None:
    t = Tuning(stream_pd, stream_upw, batch_group, batch_wg_per_cu)
    _check(load().gcss_set_tuning(h, ctypes.byref(t)))


def _result_dict(r: TuneResult) -> dict:
    return dict(best=_tuning_dict(r.best), best_ms=r.best_ms, initial_ms=r.initial_ms,
                candidates=r.candidates)


def autotune_select(h: int, k: int, reps: int, cache_path: str | None) -> dict:
    r = TuneResult()
    path = cache_path.encode() if cache_path else None
    _check(load().gcss_autotune_select(h, k, reps, path, ctypes.byref(r)))
    return _result_dict(r)


def autotune_batched(h: int, col_off, k_block: int, k_merge: int, reps: int,
                     cache_path: str | None) -> dict:
    col_off = np.ascontiguousarray(np.asarray(col_off, dtype=np.int64))
    r = TuneResult()
    path = cache_path.encode() if cache_path else None
    _check(load().gcss_autotune_batched(h, col_off.size - 1, col_off.ctypes.data, k_block,
                                        k_merge, reps, path, ctypes.byref(r)))
    return _result_dict(r)


def hbm_probe(buf_ptr: int, nbytes: int, sink_ptr: int, reps: int, stream: int = 0) -> float:
    """-> mean seconds of one read pass over the buffer"""
    sec = ctypes.c_double(0.0)
    _check(load().gcss_hbm_probe(buf_ptr, nbytes, sink_ptr, reps, stream, ctypes.byref(sec)))
    return sec.value
