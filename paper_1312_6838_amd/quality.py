"""Relative accuracy of a column subset (Section 7 of the paper):

    (||A - A_U||_F - ||A - A_S||_F) / (||A - A_U||_F - ||A - A_l||_F) x 100%

A_S, A_U: projections of A onto the span of the selected / uniformly drawn
columns (UniNoRep; ||A - A_U||_F averaged over the draws); A_l: the best
rank-l approximation.  Every error comes from the library: the projection
errors from gcss_reconstruction_error under the target B = A, ||A||_F^2 as
the error of the empty set, and ||A - A_l||_F^2 = ||A||_F^2 - sum of the l
leading eigenvalues of A A^T from gcss_top_eig.  The uniform subsets are
inputs (drawn by the caller from a seeded generator).
"""
from __future__ import annotations

import math

import numpy as np


def relative_accuracy(sel, idx, uniform_subsets, l=None, s=None, max_iters=60, tol=1e-9, seed=1):
    """sel: a Selector whose current target is B = A.  Returns a dict with
    relative_accuracy (percent), err_s, errs_u, err_l, norm2 (||A||_F^2),
    eig_iters and eig_change."""
    idx = np.asarray(idx, dtype=np.int64)
    l = int(l if l is not None else idx.size)
    norm2 = sel.reconstruction_error(np.zeros(0, dtype=np.int64))
    err_s = sel.reconstruction_error(idx[:l])
    errs_u = [sel.reconstruction_error(np.asarray(u, dtype=np.int64)) for u in uniform_subsets]
    lam, _, it, ch = sel.top_eig(l, s=s, max_iters=max_iters, tol=tol, seed=seed, want_u=False)
    err_l = max(norm2 - float(np.sum(lam)), 0.0)
    eu = float(np.mean([math.sqrt(max(e, 0.0)) for e in errs_u]))
    ra = (eu - math.sqrt(err_s)) / (eu - math.sqrt(err_l)) * 100.0
    return dict(relative_accuracy=ra, err_s=err_s, errs_u=errs_u, err_l=err_l, norm2=norm2,
                eig_iters=it, eig_change=ch)
