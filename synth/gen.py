"""Seeded generators for the matrices the selection method runs on.

Layout convention ("column store"): an m x n matrix A is held column-major
with a leading dimension ``lda >= m``; as a 2-D array it has shape
``(n, lda)`` and row ``i`` holds column ``A[:, i]`` followed by
``lda - m`` zero pad entries.  The same layout is what the GPU library takes.

The random-projection matrix Omega (n x r) is held row-major with shape
``(n, r)``: row i is the r-vector drawn for column i of A, the way the
paper's projection draws one row of Omega per input column (Section 5.1).

Generators return float64 dense matrices (``*_dense``) or float32 column
stores; the numpy generators draw in float64 and round once to the storage
type.  Large workloads are drawn on the GPU with torch (``*_torch``) using
float32 matrix products only (the small Cholesky factors of the orthonormal
factors are taken on the host); those are only used where the data would
not fit a CPU test.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "lda_for", "to_colstore", "from_colstore",
    "gauss_lowrank_dense", "spectral_lowrank_dense", "planted_dense",
    "int_lowrank_dense", "orthogonal_columns_dense", "omega_gauss",
    "block_widths", "uniform_subsets", "workload", "WORKLOADS",
    "spectral_lowrank_torch", "gauss_lowrank_torch", "omega_gauss_torch",
]


def lda_for(m: int, elem_bytes: int) -> int:
    """Smallest leading dimension >= m whose row of bytes is a 256-byte multiple."""
    per = 256 // elem_bytes
    return ((m + per - 1) // per) * per


def to_colstore(A: np.ndarray, lda: int | None = None, dtype=np.float32) -> np.ndarray:
    """m x n dense matrix -> (n, lda) column store (zero padded)."""
    m, n = A.shape
    if lda is None:
        lda = lda_for(m, np.dtype(dtype).itemsize)
    out = np.zeros((n, lda), dtype=dtype)
    out[:, :m] = A.T.astype(dtype)
    return out


def from_colstore(S: np.ndarray, m: int) -> np.ndarray:
    """(n, lda) column store -> m x n dense float64 matrix."""
    return np.ascontiguousarray(S[:, :m].T.astype(np.float64))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _orthonormal(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Random orthonormal columns: QR of a Gaussian, signs fixed so diag(R) > 0."""
    G = rng.standard_normal((rows, cols))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def gauss_lowrank_dense(m, n, rank, noise, seed, scale=1.0):
    """A = scale * U V^T + noise * N(0,1), with U (m x rank), V (n x rank) i.i.d. N(0,1)."""
    rng = _rng(seed)
    U = rng.standard_normal((m, rank))
    V = rng.standard_normal((n, rank))
    return scale * (U @ V.T) + noise * rng.standard_normal((m, n))


def spectral_lowrank_dense(m, n, rank, decay, noise, seed):
    """A = U diag(s) V^T + noise * N(0,1); U, V random orthonormal, s_j = j^-decay."""
    rng = _rng(seed)
    U = _orthonormal(rng, m, rank)
    V = _orthonormal(rng, n, rank)
    s = np.arange(1, rank + 1, dtype=np.float64) ** (-decay)
    return (U * s) @ V.T + noise * rng.standard_normal((m, n))


def planted_dense(m, n, k, ratio, seed, background=1e-4):
    """k planted columns c_j u_j (c_j = ratio^-j, u_j orthonormal) at random
    positions over a background of background * N(0,1) / sqrt(m).

    Returns (A, positions) where positions[j] is the column holding c_j u_j.
    """
    rng = _rng(seed)
    A = background * rng.standard_normal((m, n)) / math.sqrt(m)
    U = _orthonormal(rng, m, k)
    pos = rng.permutation(n)[:k]
    for j in range(k):
        A[:, pos[j]] = ratio ** (-j) * U[:, j]
    return A, pos


def int_lowrank_dense(m, n, rank, seed, lo=-2, hi=2):
    """Exactly rank-`rank` integer matrix: U V^T with integer factors in [lo, hi].

    Entries are small integers, so the matrix is exact in float32 and float64.
    """
    rng = _rng(seed)
    U = rng.integers(lo, hi + 1, size=(m, rank)).astype(np.float64)
    V = rng.integers(lo, hi + 1, size=(n, rank)).astype(np.float64)
    return U @ V.T


def orthogonal_columns_dense(sq_norms, m=None):
    """Column i = sqrt(sq_norms[i]) * e_i (mutually orthogonal columns)."""
    d = np.asarray(sq_norms, dtype=np.float64)
    n = d.size
    m = n if m is None else m
    A = np.zeros((m, n))
    A[np.arange(n), np.arange(n)] = np.sqrt(d)
    return A


def omega_gauss(n, r, seed, dtype=np.float32):
    """Omega (n x r), i.i.d. N(0, 1/r), row-major: row i is drawn for column i."""
    rng = _rng(seed)
    return (rng.standard_normal((n, r)) / math.sqrt(r)).astype(dtype)


def uniform_subsets(n, l, seeds):
    """UniNoRep column subsets: l distinct columns drawn uniformly, one per seed."""
    return [np.sort(_rng(int(s)).choice(n, l, replace=False)).astype(np.int64) for s in seeds]


def block_widths(nblocks, lo, hi, seed):
    """Uneven block widths drawn uniformly from the integers [lo, hi]."""
    rng = _rng(seed)
    return rng.integers(lo, hi + 1, size=nblocks).astype(np.int64)


# ---------------------------------------------------------------------------
# Named workloads (shapes and value models of the paper-sized runs)
# ---------------------------------------------------------------------------
WORKLOADS = {
    # centralized, B = A, small enough for the oracle to run whole
    "css_500x1000_k20": dict(m=500, n=1000, kind="gauss", rank=50, noise=0.01,
                             target="self", k=20),
    # centralized, B = A
    "css_4096x65536_k200": dict(m=4096, n=65536, kind="spectral", rank=512, decay=1.0,
                                noise=1e-3, target="self", k=200),
    # generalized, B = A Omega
    "gcss_2048x1048576_r256_k100": dict(m=2048, n=1048576, kind="spectral", rank=1024,
                                        decay=0.7, noise=1e-3, target="proj", r=256,
                                        k=100),
    # batched partitions sharing one B, then the merge selection
    "batched_1024_64blocks_r128": dict(m=1024, nblocks=64, wlo=2048, whi=32768,
                                       kind="gauss_scaled", rank=256, noise=0.01,
                                       target="proj", r=128, k_block=20, k_merge=100),
    # fp8 stream
    "gcss_fp8_8192x262144_r512_k500": dict(m=8192, n=262144, kind="spectral", rank=2048,
                                           decay=0.5, noise=1e-3, target="proj", r=512,
                                           k=500, b_dtype="bf16"),
}


def workload(name: str) -> dict:
    return dict(WORKLOADS[name])


# ---------------------------------------------------------------------------
# GPU-side generators (torch), for sizes a CPU test cannot hold
# ---------------------------------------------------------------------------
def _torch_gen(seed, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def _orthonormal_torch(rows, cols, gen, device, chunk=65536):
    """Random orthonormal columns (float32, on `device`): Cholesky QR of a Gaussian,
    twice.  Only plain float32 matrix products run on the device; the small
    cols x cols Cholesky factor and its inverse are computed on the host."""
    import numpy as np
    import torch
    G = torch.randn(rows, cols, generator=gen, device=device, dtype=torch.float32)
    for _ in range(2):
        S = torch.zeros(cols, cols, dtype=torch.float64)
        for i0 in range(0, rows, chunk):
            Gc = G[i0:i0 + chunk]
            S += (Gc.T @ Gc).double().cpu()
        R = np.linalg.cholesky(S.numpy()).T            # upper, S = R^T R
        Rinv = np.linalg.inv(R)
        Rinv_d = torch.from_numpy(Rinv.astype(np.float32)).to(device)
        for i0 in range(0, rows, chunk):
            G[i0:i0 + chunk] = G[i0:i0 + chunk] @ Rinv_d
    return G


def spectral_lowrank_torch(m, n, rank, decay, noise, seed, device="cuda", lda=None,
                           chunk=65536):
    """Float32 column store (n, lda) on `device` of U diag(s) V^T + noise N(0,1)."""
    import torch
    lda = lda_for(m, 4) if lda is None else lda
    gen = _torch_gen(seed, device)
    U = _orthonormal_torch(m, rank, gen, device)
    s = torch.arange(1, rank + 1, device=device, dtype=torch.float32) ** (-decay)
    SUt = (U * s).T.contiguous()                      # rank x m
    del U
    V = _orthonormal_torch(n, rank, gen, device)      # n x rank
    out = torch.zeros(n, lda, device=device, dtype=torch.float32)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        blk = V[i0:i1] @ SUt                          # columns i0..i1 of A, transposed
        blk += noise * torch.randn(i1 - i0, m, generator=gen, device=device,
                                   dtype=torch.float32)
        out[i0:i1, :m] = blk
    del V
    return out


def gauss_lowrank_torch(m, n, rank, noise, seed, device="cuda", lda=None, scale=1.0,
                        chunk=65536):
    """Float32 column store of scale * U V^T + noise N(0,1) with Gaussian factors."""
    import torch
    lda = lda_for(m, 4) if lda is None else lda
    gen = _torch_gen(seed, device)
    Ut = torch.randn(rank, m, generator=gen, device=device, dtype=torch.float32) * scale
    out = torch.zeros(n, lda, device=device, dtype=torch.float32)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        V = torch.randn(i1 - i0, rank, generator=gen, device=device, dtype=torch.float32)
        blk = V @ Ut
        blk += noise * torch.randn(i1 - i0, m, generator=gen, device=device,
                                   dtype=torch.float32)
        out[i0:i1, :m] = blk
    return out


def omega_gauss_torch(n, r, seed, device="cuda"):
    """Omega (n x r) float32 i.i.d. N(0, 1/r), row-major, drawn on `device`."""
    import torch
    gen = _torch_gen(seed, device)
    return (torch.randn(n, r, generator=gen, device=device, dtype=torch.float32)
            / math.sqrt(r))
