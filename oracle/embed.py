"""Outputs built on the selected columns -- TEST INFRASTRUCTURE (FP64, numpy).

Section 3 of the paper (Farahat et al., "Greedy Column Subset Selection for
Large-scale Data Sets"), after the selection:

* ``embedding(A, S)``: an orthonormal basis Q of A_S (QR of A_S, a library
  primitive) and the embedding W = Q^T A of every column (Eq. CSS_LowDim).
* ``rank_k(A, S, k)``: the rank-k approximation inside span(A_S) that the
  section attributes to Boutsidis et al.: the best rank-k approximation
  W_k = U_k Sigma_k V_k^T of W (SVD, a library primitive), then
  A_{S,k} = Q W_k.  Also the approximate leading singular triplets of A
  (Eq. ApproxSVD): U_A = Q U_k, Sigma_A = Sigma_k, V_A = V_k.

Sign convention (so that the triplets are unique for distinct singular
values): the entry of largest magnitude of each column of U_A is positive
(the first such entry on ties); V_A's column takes the same sign.
A is a dense m x n array here (columns are data points).
"""
from __future__ import annotations

import numpy as np


def embedding(A, S):
    """Q (m x l, orthonormal, span = span(A_S)) and W = Q^T A (l x n)."""
    A = np.asarray(A, dtype=np.float64)
    Q, _ = np.linalg.qr(A[:, list(S)])
    return Q, Q.T @ A


def sign_fix(U, V):
    """Flip column pairs so each column of U has its largest-magnitude entry positive."""
    U = np.array(U, dtype=np.float64)
    V = np.array(V, dtype=np.float64)
    for j in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, j])))     # first index of the maximum
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
            V[:, j] = -V[:, j]
    return U, V


def rank_k(A, S, k):
    """Boutsidis et al.'s rank-k approximation in span(A_S).

    Returns dict(U (m x k) = Q U_k, sigma (k), V (n x k), approx = Q W_k
    (m x n), err = ||A - Q W_k||_F^2).
    """
    A = np.asarray(A, dtype=np.float64)
    Q, W = embedding(A, S)
    Uw, sw, Vwt = np.linalg.svd(W, full_matrices=False)
    k = int(k)
    Uk, sk, Vk = Uw[:, :k], sw[:k], Vwt[:k].T
    UA, VA = sign_fix(Q @ Uk, Vk)
    approx = (UA * sk[None, :]) @ VA.T
    R = A - approx
    return dict(U=UA, sigma=sk, V=VA, approx=approx, err=float(np.sum(R * R)))
