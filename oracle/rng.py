"""Counter-based random sign matrices for the concise target -- TEST
INFRASTRUCTURE (numpy, exact integer arithmetic).

Section 5.1 of the paper (Farahat et al., "Greedy Column Subset Selection for
Large-scale Data Sets") draws the n x r projection Omega with i.i.d. entries
from a univariate distribution Psi, one row per column of A, so that a
mapper can sample Omega_i: as it reads column i and no one stores Omega.
Besides Gaussian matrices it names uniform random sign (+-1) matrices and
sparse random sign matrices; for the sparse ones a note in the paper's
source (not in the printed text) gives +-1 with probability 1/(2 sqrt n)
each and 0 otherwise.

Entries here come from Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011), written from that
paper's definition: a 4 x 32-bit counter and a 2 x 32-bit key; a round maps
(c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
lo(M0 c0)) with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is bumped by
(0x9E3779B9, 0xBB67AE85) before every round but the first; ten rounds.

Omega_ij for a 64-bit seed and density d in (0, 1]:
  u   = word (j mod 4) of Philox4x32-10(counter (i lo, i hi, j div 4, 0),
                                        key (seed lo, seed hi))
  t   = round(d * 2^31)                     (clamped to [1, 2^31])
  Omega_ij = 0 if (u >> 1) >= t, else (-1 if u & 1 else +1)
d = 1 gives the dense random sign matrix; d = 1/sqrt(n) the sparse one.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: (N, 4) uint32, key: (2,) uint32 -> (N, 4) uint32."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k0, k1 = np.uint32(key[0]), np.uint32(key[1])
    for rnd in range(10):
        if rnd > 0:
            k0 = np.uint32((int(k0) + int(W0)) & 0xFFFFFFFF)
            k1 = np.uint32((int(k1) + int(W1)) & 0xFFFFFFFF)
        p0 = c[:, 0].astype(np.uint64) * M0
        p1 = c[:, 2].astype(np.uint64) * M1
        hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
        lo0 = (p0 & _MASK).astype(np.uint32)
        hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
        lo1 = (p1 & _MASK).astype(np.uint32)
        c = np.stack([hi1 ^ c[:, 1] ^ k0, lo1, hi0 ^ c[:, 3] ^ k1, lo0], axis=1)
    return c


def threshold(density):
    t = int(round(float(density) * 2.0 ** 31))
    return min(max(t, 1), 1 << 31)


def omega_rows(i0, i1, r, seed, density):
    """Rows i0..i1-1 of Omega as an (i1 - i0, r) float64 array."""
    i = np.arange(i0, i1, dtype=np.uint64)
    nb = (r + 3) // 4
    ii = np.repeat(i, nb)
    jb = np.tile(np.arange(nb, dtype=np.uint64), i.size)
    ctr = np.stack([(ii & _MASK).astype(np.uint32), (ii >> np.uint64(32)).astype(np.uint32),
                    jb.astype(np.uint32), np.zeros(ii.size, dtype=np.uint32)], axis=1)
    seed = int(seed)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    u = philox4x32_10(ctr, key).reshape(i.size, nb * 4)[:, :r]
    t = np.uint32(threshold(density)) if threshold(density) < (1 << 31) else None
    keep = np.ones(u.shape, dtype=bool) if t is None else (u >> np.uint32(1)) < t
    sign = np.where((u & np.uint32(1)) != 0, -1.0, 1.0)
    return np.where(keep, sign, 0.0)


def omega_column(n, j, seed, density, chunk=1 << 20):
    """Column j of Omega (all n rows) as float64, without the other columns."""
    out = np.zeros(n)
    seed = int(seed)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    t = threshold(density)
    for i0 in range(0, n, chunk):
        i = np.arange(i0, min(n, i0 + chunk), dtype=np.uint64)
        ctr = np.stack([(i & _MASK).astype(np.uint32), (i >> np.uint64(32)).astype(np.uint32),
                        np.full(i.size, j // 4, dtype=np.uint32),
                        np.zeros(i.size, dtype=np.uint32)], axis=1)
        u = philox4x32_10(ctr, key)[:, j % 4]
        keep = np.ones(u.shape, dtype=bool) if t >= (1 << 31) else (u >> np.uint32(1)) < np.uint32(t)
        out[i0:i0 + i.size] = np.where(keep, np.where((u & np.uint32(1)) != 0, -1.0, 1.0), 0.0)
    return out


def project_sign(A, seed, density, r, chunk=65536):
    """B = A Omega (Section 5.1's concise target), A dense m x n, FP64."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    B = np.zeros((m, r))
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        B += A[:, i0:i1] @ omega_rows(i0, i1, r, seed, density)
    return B
