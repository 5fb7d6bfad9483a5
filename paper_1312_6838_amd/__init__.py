"""Greedy generalized column subset selection on MI355X (gfx950).

The computation lives in the HIP library ``libgcss.so`` (C ABI in
``include/gcss.h``).  This package only marshals arguments: torch supplies
device memory and the stream, :mod:`._abi` forwards the calls.

    sel = Selector(A, m, k_max=100, r_max=256)     # A: (n, lda) cuda tensor
    sel.project_target(Omega)                      # B = A Omega
    idx, obj, nsel, status = sel.select(100)
"""
from __future__ import annotations

from . import _abi
from ._abi import (  # noqa: F401
    BF16, ERR_ARG, ERR_DEVICE, ERR_STATE, ERR_UNSUPPORTED, ERR_WORKSPACE, EXPORTS, F32,
    FP8_E4M3, OK, STATE_B, STATE_F, STATE_F0, STATE_G, STATE_G0, STATE_GRAM, STATE_NREJECT,
    STATE_FLAGS, ASYNC_SPARE_STEPS, STATIC_SCRATCH_BYTES, select_static,
    STATE_Q, STATE_Z, WARN_EXHAUSTED, Desc, GcssError, batched_workspace_size, create, destroy,
    last_error, load, make_desc, project_target, quantize, read_state, reconstruction_error,
    select, select_async, select_batched, set_target, version, workspace_size,
    set_profiling, get_profile, set_embedding, qless_r, rank_k, project_sign, top_eig,
    gather_columns, get_tuning, set_tuning, autotune_select, autotune_batched, hbm_probe,
    PROBE_SINK_FLOATS, BUDGET_UNIFORM, BUDGET_EVEN, BUDGET_NORM, block_budgets,
    select_batched_budgets,
)

__all__ = ["Selector", "quantize_tensor", "qless_r_tensor", "hbm_probe_tensor",
           "select_static_tensor", "load", "version", "GcssError"]


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return BF16
    if t.dtype in (torch.uint8, torch.float8_e4m3fn):
        return FP8_E4M3
    raise TypeError(f"unsupported A dtype {t.dtype}")


def _target_code(B):
    import torch
    if B.dtype == torch.float32:
        return F32
    if B.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return BF16
    raise TypeError(f"unsupported target dtype {B.dtype} (float32 or bfloat16)")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Selector:
    """One selection context over a column store A (n, lda) on the GPU.

    Holds references to every tensor the library borrows (A, scales, the
    workspace, the target) so they outlive the context.  ``workspace`` may be
    a caller-owned uint8 cuda tensor of at least the required size; by
    default one is allocated.
    """

    def __init__(self, A, m, *, k_max, r_max=0, self_target=False, scales=None, tau=0.0,
                 stream=None, batched=None, workspace=None):
        import torch
        if not A.is_cuda or A.dim() != 2 or not A.is_contiguous():
            raise ValueError("A must be a contiguous 2-D cuda tensor of shape (n, lda)")
        load()
        self.A, self.scales, self.m = A, scales, int(m)
        n, lda = A.shape
        self.n, self.lda = int(n), int(lda)
        self.dtype = _dtype_code(A)
        self.stream = stream
        self.desc = make_desc(self.m, self.n, self.lda, self.dtype, A.data_ptr(),
                              scales.data_ptr() if scales is not None else None, int(k_max),
                              int(r_max), self_target, tau, _stream_ptr(stream))
        nbytes = workspace_size(self.desc)
        if batched is not None:
            nbytes += batched_workspace_size(self.desc, *batched)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
        elif (workspace.dtype != torch.uint8 or not workspace.is_cuda
              or not workspace.is_contiguous() or workspace.numel() < nbytes):
            raise ValueError(f"workspace must be a contiguous uint8 cuda tensor of >= {nbytes} bytes")
        self.ws = workspace
        self.ws_bytes = nbytes
        self.h = create(self.desc, self.ws.data_ptr(), nbytes)
        self.B = None
        self.r = 0

    # -- targets --
    def set_target(self, B=None):
        """B: (r, ldb) float32 or bfloat16 column store on the GPU, or None for B = A."""
        if B is None:
            set_target(self.h, None, 0, 0)
            self.B, self.r = None, 0
        else:
            r, ldb = B.shape
            set_target(self.h, B.data_ptr(), int(r), int(ldb), _target_code(B))
            self.B, self.r = B, int(r)

    def project_target(self, Omega, ldb=None, b_dtype="f32"):
        """B = A Omega; Omega (n, r) float32 row-major on the GPU.  b_dtype "f32"
        keeps the binary32 product, "bf16" rounds it to bfloat16.  Returns B
        (r, ldb) as float32 or bfloat16."""
        import torch
        n, r = Omega.shape
        ldb = ldb or ((self.m + 63) // 64) * 64
        tdt = {"f32": torch.float32, "bf16": torch.bfloat16}[b_dtype]
        B = torch.empty(int(r), int(ldb), dtype=tdt, device=self.A.device)
        project_target(self.h, Omega.data_ptr(), int(r), B.data_ptr(), int(ldb), _target_code(B))
        self.B, self.r, self._omega = B, int(r), Omega
        return B

    def project_sign(self, seed, r, density=None, ldb=None):
        """B = A Omega with a random sign Omega drawn on the device (Philox4x32-10,
        counter (column, j/4)); density None = 1/sqrt(n) (sparse), 1 = dense.
        Returns B (r, ldb)."""
        import math
        import torch
        d = 1.0 / math.sqrt(self.n) if density is None else float(density)
        ldb = ldb or ((self.m + 63) // 64) * 64
        B = torch.empty(int(r), int(ldb), dtype=torch.float32, device=self.A.device)
        project_sign(self.h, int(seed), d, int(r), B.data_ptr(), int(ldb))
        self.B, self.r = B, int(r)
        return B

    # -- selection --
    def select(self, k):
        return select(self.h, int(k))

    def select_async(self, k, out=None):
        """Device outputs (idx int64[k], obj float64[k+1], nsel int32[1]); no sync."""
        import torch
        if out is None:
            dev = self.A.device
            out = (torch.empty(k, dtype=torch.int64, device=dev),
                   torch.empty(k + 1, dtype=torch.float64, device=dev),
                   torch.empty(1, dtype=torch.int32, device=dev))
        select_async(self.h, int(k), out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr())
        return out

    def set_embedding(self, W=None):
        """Have selections write W = Q^T A into W, a (k_max, ldw) float32 cuda
        tensor (row t = A^T q_{t+1}, ldw >= n); None turns it off."""
        import torch
        if W is None:
            set_embedding(self.h, None, 0)
        else:
            if (W.dtype != torch.float32 or not W.is_cuda or W.dim() != 2
                    or W.stride(1) != 1 or W.shape[1] < self.n):
                raise ValueError("W must be a float32 cuda tensor (rows, ldw >= n), unit column stride")
            set_embedding(self.h, W.data_ptr(), int(W.stride(0)))
        self.W = W

    def rank_k(self, l, k, want_u=True, want_v=True):
        """Rank-k approximation in the span of the first l picks of the last
        selection, from the embedding set with set_embedding.  Returns
        (U (k, m) float64 rows = columns of U_A, sigma (k,), V (k, n) float32
        rows = columns of V_A, err)."""
        import torch
        if getattr(self, "W", None) is None:
            raise ValueError("no embedding set")
        dev = self.A.device
        U = torch.empty(int(k), self.m, dtype=torch.float64, device=dev) if want_u else None
        V = torch.empty(int(k), self.n, dtype=torch.float32, device=dev) if want_v else None
        sigma, err = rank_k(self.h, self.W.data_ptr(), int(self.W.stride(0)), int(l), int(k),
                            U.data_ptr() if U is not None else None, self.m,
                            V.data_ptr() if V is not None else None, self.n)
        return U, sigma, V, err

    def top_eig(self, k, s=None, max_iters=20, tol=1e-7, seed=1, want_u=True):
        """Leading eigenpairs of A A^T (needs the self target): returns
        (lambda (k,), U (k, m) float64 rows = left singular vectors or None,
        iterations, last relative change)."""
        import torch
        s = int(s or min(2 * k, self.desc.k_max, self.m))
        U = torch.empty(int(k), self.m, dtype=torch.float64, device=self.A.device) if want_u else None
        lam, it, ch = top_eig(self.h, s, int(max_iters), float(tol), int(seed), int(k),
                              U.data_ptr() if U is not None else None, self.m)
        return lam, U, it, ch

    def svd_target(self, k, s=None, max_iters=20, tol=1e-7, seed=1, ldb=None):
        """The DistApproxSVD target B = U_k Sigma_k of A (leading singular
        triplets by subspace iteration on A A^T; needs the self target), set as
        the explicit target.  Returns (B (k, ldb) float32, lambda, iterations)."""
        import torch
        s = int(s or min(2 * k, self.desc.k_max, self.m))
        ldb = ldb or ((self.m + 63) // 64) * 64
        U = torch.empty(int(k), self.m, dtype=torch.float64, device=self.A.device)
        B = torch.empty(int(k), int(ldb), dtype=torch.float32, device=self.A.device)
        lam, it, ch = top_eig(self.h, s, int(max_iters), float(tol), int(seed), int(k),
                              U.data_ptr(), self.m, B.data_ptr(), int(ldb))
        self.set_target(B)
        return B, lam, it

    def gather(self, idx):
        """Stored columns idx of A as a new column store (count, lda) on the GPU
        (and their FP8 scales).  Returns (A_sub, scales_sub or None)."""
        import torch
        idx = torch.as_tensor(idx, dtype=torch.int64).to(self.A.device).contiguous()
        out = torch.empty(int(idx.numel()), self.lda, dtype=self.A.dtype, device=self.A.device)
        sc = (torch.empty(int(idx.numel()), dtype=torch.float32, device=self.A.device)
              if self.scales is not None else None)
        gather_columns(self.h, idx.data_ptr(), int(idx.numel()), out.data_ptr(),
                       sc.data_ptr() if sc is not None else None)
        return out, sc

    def reconstruction_error(self, idx):
        return reconstruction_error(self.h, idx)

    def select_batched(self, col_off, k_block, k_merge):
        return select_batched(self.h, col_off, int(k_block), int(k_merge))

    def select_batched_budgets(self, col_off, k_blocks, k_merge):
        return select_batched_budgets(self.h, col_off, k_blocks, int(k_merge))

    def block_budgets(self, col_off, l, policy, norms2=None):
        return block_budgets(self.h, col_off, int(l), policy, norms2)

    def read(self, item, count, np_dtype):
        import numpy as np
        raw = read_state(self.h, item, int(count) * np.dtype(np_dtype).itemsize)
        return np.frombuffer(raw, dtype=np_dtype).copy()

    def flags(self):
        """State of the last selection: dict(picks, finished, exhausted, rejected)."""
        import numpy as np
        v = self.read(STATE_FLAGS, 4, np.int32)
        return dict(picks=int(v[0]), finished=bool(v[1]), exhausted=bool(v[2]),
                    rejected=int(v[3]))

    def tuning(self, **setting):
        """Read the streaming passes' launch setting, or change some of its
        fields (stream_pd, stream_upw, batch_group, batch_wg_per_cu)."""
        if setting:
            cur = get_tuning(self.h)
            cur.update(setting)
            set_tuning(self.h, cur["stream_pd"], cur["stream_upw"], cur["batch_group"],
                       cur["batch_wg_per_cu"])
        return get_tuning(self.h)

    def autotune(self, k, reps=3, cache=None):
        """Time select(k) under each candidate launch setting and keep the
        fastest (cache: JSON path or None).  Returns the tuner's result."""
        return autotune_select(self.h, int(k), int(reps), cache)

    def autotune_batched(self, col_off, k_block, k_merge, reps=3, cache=None):
        return autotune_batched(self.h, col_off, int(k_block), int(k_merge), int(reps), cache)

    def profile(self, enable=None):
        """Turn stream-kernel event timing on/off (clears counters), or read them."""
        if enable is not None:
            set_profiling(self.h, enable)
        return get_profile(self.h)

    def close(self):
        if getattr(self, "h", None):
            destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def select_static_tensor(A, m, k, B=None, *, scales=None, tau=0.0, stream=None, out=None):
    """One selection through the entry point that allocates no device memory
    (its workspace is the library's static device array).  A: (n, lda) column
    store; B: (r, ldb) float32 or bfloat16 column store, or None for B = A.  out: optional
    (idx int64[k], obj float64[k+1], nsel int32[1]) cuda tensors, else
    allocated here by torch.  Returns out; nothing is synchronised."""
    import torch
    if not A.is_cuda or A.dim() != 2 or not A.is_contiguous():
        raise ValueError("A must be a contiguous 2-D cuda tensor of shape (n, lda)")
    n, lda = A.shape
    r, ldb = (0, 0) if B is None else B.shape
    desc = make_desc(int(m), int(n), int(lda), _dtype_code(A), A.data_ptr(),
                     scales.data_ptr() if scales is not None else None, int(k), int(r),
                     B is None, tau, _stream_ptr(stream))
    if out is None:
        dev = A.device
        out = (torch.empty(k, dtype=torch.int64, device=dev),
               torch.empty(k + 1, dtype=torch.float64, device=dev),
               torch.empty(1, dtype=torch.int32, device=dev))
    select_static(desc, None if B is None else B.data_ptr(), int(r), int(ldb), int(k),
                  out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                  F32 if B is None else _target_code(B))
    return out


def hbm_probe_tensor(buf, reps=5, stream=None):
    """Mean seconds of one read pass over a cuda tensor's bytes, and the sink
    (uint32 cuda tensor whose XOR over all entries is the XOR of the buffer's
    32-bit words)."""
    import torch
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous cuda tensor")
    sink = torch.empty(PROBE_SINK_FLOATS, dtype=torch.int32, device=buf.device)
    sec = hbm_probe(buf.data_ptr(), buf.numel() * buf.element_size(), sink.data_ptr(), int(reps),
                    _stream_ptr(stream))
    return sec, sink


def qless_r_tensor(W, n, idx, stream=None):
    """Upper triangular R (k, k) float32 with A_S = Q R, from the embedding W
    (rows, ldw) and the picks idx (int64 cuda tensor, k entries)."""
    import torch
    k = int(idx.numel())
    if W.stride(1) != 1 or idx.dtype != torch.int64 or not idx.is_contiguous():
        raise ValueError("W needs unit column stride and idx a contiguous int64 tensor")
    R = torch.empty(k, k, dtype=torch.float32, device=W.device)
    qless_r(W.data_ptr(), int(n), int(W.stride(0)), idx.data_ptr(), k, R.data_ptr(), k,
            _stream_ptr(stream))
    return R


def quantize_tensor(A32, m, dtype, stream=None):
    """Quantize a float32 column store (n, lda) on the GPU.

    dtype "bf16" -> (codes uint16-as-int16 (n, ldo), None);
    dtype "fp8"  -> (codes uint8 (n, ldo), scales float32 (n,)).
    """
    import torch
    n, lda = A32.shape
    if dtype == "bf16":
        ldo = ((m + 127) // 128) * 128
        out = torch.zeros(n, ldo, dtype=torch.int16, device=A32.device)
        quantize(A32.data_ptr(), m, n, lda, BF16, out.data_ptr(), ldo, None, _stream_ptr(stream))
        return out, None
    if dtype == "fp8":
        ldo = ((m + 255) // 256) * 256
        out = torch.zeros(n, ldo, dtype=torch.uint8, device=A32.device)
        sc = torch.zeros(n, dtype=torch.float32, device=A32.device)
        quantize(A32.data_ptr(), m, n, lda, FP8_E4M3, out.data_ptr(), ldo, sc.data_ptr(),
                 _stream_ptr(stream))
        return out, sc
    raise ValueError(dtype)
