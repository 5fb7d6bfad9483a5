"""Quality metric of the paper's experiments -- TEST INFRASTRUCTURE (FP64).

Section 7 of the paper (Farahat et al., "Greedy Column Subset Selection for
Large-scale Data Sets") compares column subsets by their relative accuracy

    (||A - A_U||_F - ||A - A_S||_F) / (||A - A_U||_F - ||A - A_l||_F) x 100%

with A_S the projection of A onto the span of the selected columns, A_U the
same for uniformly sampled columns (UniNoRep: without replacement; the
average of ||A - A_U||_F over several draws) and A_l the best rank-l
approximation (SVD).  Its DistApproxSVD baseline selects columns for the
target B = U_k Sigma_k (leading singular triplets of A).

* ``top_eig(A, k)``        leading eigenpairs of A A^T from an SVD of A
                           (library primitive), sign convention of
                           oracle.embed (largest-magnitude entry positive)
* ``best_rank_error(A, l)`` ||A - A_l||_F^2 = sum of sigma_j^2 for j > l
* ``relative_accuracy(err_s, errs_u, err_l)`` the formula above from
                           squared errors (Frobenius norms are their roots)
* ``svd_target(A, k)``     U_k Sigma_k
A is dense m x n.
"""
from __future__ import annotations

import numpy as np

from oracle import embed


def top_eig(A, k):
    """(lambda (k,), U (m x k)): eigenvalues of A A^T and left singular vectors."""
    A = np.asarray(A, dtype=np.float64)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    Uk, Vk = embed.sign_fix(U[:, :k], Vt[:k].T)
    return s[:k] ** 2, Uk


def best_rank_error(A, l):
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return float(np.sum(s[l:] ** 2))


def relative_accuracy(err_s, errs_u, err_l):
    """Percent; errors are squared Frobenius norms, the formula uses norms."""
    eu = float(np.mean(np.sqrt(np.asarray(errs_u, dtype=np.float64))))
    return (eu - np.sqrt(err_s)) / (eu - np.sqrt(err_l)) * 100.0


def svd_target(A, k):
    lam, U = top_eig(A, k)
    return U * np.sqrt(lam)[None, :]
