"""FP64 definitions for inputs too large for the C oracle's plain loops --
TEST INFRASTRUCTURE.

Each function is a definition from the paper written with library
primitives (numpy matrix products and QR), no blocking or reordering beyond
the library's own:

* ``project(A_cs, m, Omega)``: the concise target B = A Omega (Section 5.1),
  summed over column chunks.
* ``error(A_S, B)``: ||B - P_S B||_F^2 (Problems 1/5) with P_S = Q Q^T from
  a QR of A_S (Section 3.1's projection without the explicit inverse).
* ``scores(A_S, A_cand, B)``: the greedy criterion of Problem 6 for each
  candidate column given the picks A_S: ||F^T E_i||^2 / ||E_i||^2 with
  E = (I - P_S) A, F = (I - P_S) B.

Column stores are (n, ld) arrays whose row i is column i.
"""
from __future__ import annotations

import numpy as np


def project(A_cs, m, Omega, chunk=65536):
    """B (m x r, float64) = sum over columns i of A_i Omega_i:."""
    n = A_cs.shape[0]
    r = Omega.shape[1]
    B = np.zeros((m, r))
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        B += np.asarray(A_cs[i0:i1, :m], dtype=np.float64).T @ np.asarray(Omega[i0:i1], dtype=np.float64)
    return B


def _basis(A_S):
    A_S = np.asarray(A_S, dtype=np.float64)
    if A_S.shape[1] == 0:
        return np.zeros((A_S.shape[0], 0))
    Q, R = np.linalg.qr(A_S)
    keep = np.abs(np.diag(R)) > 1e-13 * np.max(np.abs(np.diag(R)))
    return Q[:, keep]


def error(A_S, B, chunk=8192):
    """||B - Q Q^T B||_F^2, B given dense (m x r) or as a column store callback."""
    Q = _basis(A_S)
    B = np.asarray(B, dtype=np.float64)
    tot = 0.0
    for c0 in range(0, B.shape[1], chunk):
        Bc = B[:, c0:c0 + chunk]
        R = Bc - Q @ (Q.T @ Bc)
        tot += float(np.sum(R * R))
    return tot


def scores(A_S, A_cand, B):
    """Greedy criterion f_i / g_i of each candidate column (m x c) given picks A_S."""
    Q = _basis(A_S)
    E = np.asarray(A_cand, dtype=np.float64)
    E = E - Q @ (Q.T @ E)
    B = np.asarray(B, dtype=np.float64)
    F = B - Q @ (Q.T @ B)
    H = F.T @ E
    return np.sum(H * H, axis=0) / np.sum(E * E, axis=0)
