"""Brute force for tiny inputs -- TEST INFRASTRUCTURE (numpy, float64).

Everything here is computed from the plain definitions, with no recursion:

* ``objective(A, B, S)`` is ||B - P_S B||_F^2 (Problem 1 / Problem 5), with
  P_S B obtained from the least-squares fit of B on the columns A_S
  (Section 3.1: T* = argmin ||B - A_S T||).
* ``greedy(A, B, k)`` is the greedy step of Section 4.2 taken literally:
  at every iteration, the objective of S + {i} is recomputed for every
  candidate i and the smallest is taken (ties to the lowest index).
* ``exhaustive(A, B, k)`` searches all k-subsets (the optimum the greedy
  method approximates).

A and B here are ordinary dense m x n / m x r float64 matrices.
"""
from __future__ import annotations

import itertools

import numpy as np


def objective(A, B, S):
    Bt = A if B is None else B
    S = list(S)
    if not S:
        return float(np.sum(Bt * Bt))
    X, *_ = np.linalg.lstsq(A[:, S], Bt, rcond=None)
    R = Bt - A[:, S] @ X
    return float(np.sum(R * R))


def greedy(A, B, k, zero_tol=0.0):
    """Returns (picks, F_after_each_pick, decrements) where decrements[t][i] is
    F(S) - F(S + {i}) for every candidate i at step t (nan for selected)."""
    n = A.shape[1]
    S = []
    F = [objective(A, B, S)]
    decs = []
    for _ in range(k):
        Fs = F[-1]
        d = np.full(n, np.nan)
        best, pbest = None, -1
        for i in range(n):
            if i in S:
                continue
            if np.sum(A[:, i] ** 2) <= zero_tol:
                continue
            Fi = objective(A, B, S + [i])
            d[i] = Fs - Fi
            if best is None or Fi < best:
                best, pbest = Fi, i
        decs.append(d)
        S.append(pbest)
        F.append(best)
    return S, np.array(F), decs


def exhaustive(A, B, k):
    n = A.shape[1]
    best, bestS = None, None
    for S in itertools.combinations(range(n), k):
        F = objective(A, B, S)
        if best is None or F < best:
            best, bestS = F, S
    return list(bestS), best
