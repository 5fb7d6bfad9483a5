"""Naive distributed CSS (Section 5's first approach) -- TEST INFRASTRUCTURE.

Each block of columns selects against itself (Algorithm 1 on A_(b), the C
oracle's select with B = A_(b)); the picks are pooled; an optional second
selection runs Algorithm 1 on the pooled columns A_{:L}.  Budgets: uniform
l/c or adaptive l ||A_(b)||^2 / ||A||^2, both rounded by largest remainders
within the block widths.
A is a dense m x n array.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import budgets as budget_rules


def budgets(A, col_off, l, policy):
    """Budgets of the naive approach: "uniform" is l / c and "adaptive" is
    l ||A_(b)||^2 / ||A||^2, both rounded by largest remainders within the
    block widths (oracle/budgets.py)."""
    widths = [col_off[b + 1] - col_off[b] for b in range(len(col_off) - 1)]
    norms = [float(np.sum(A[:, col_off[b]:col_off[b + 1]] ** 2)) for b in range(len(widths))]
    return budget_rules.budgets(norms, widths, l, {"uniform": "even", "adaptive": "norm"}[policy])


def naive_select(A, col_off, l, k_merge=0, policy="uniform"):
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    bud = budgets(A, col_off, l, policy)
    idx_block, obj_block = [], []
    for b in range(len(col_off) - 1):
        Ab = A[:, col_off[b]:col_off[b + 1]]
        if bud[b] == 0:
            idx_block.append(np.zeros(0, dtype=np.int64))
            obj_block.append(float(np.sum(Ab * Ab)))
            continue
        cs = np.ascontiguousarray(Ab.T)
        r = oracle.select(cs, m, bud[b])
        ns = r["n_selected"]
        idx_block.append(r["idx"][:ns] + col_off[b])
        obj_block.append(float(r["obj"][ns]))
    pool = np.concatenate(idx_block)
    out = dict(budgets=bud, idx_block=idx_block, pool=pool, obj_block=obj_block,
               idx_merge=None, obj_merge=None)
    if k_merge:
        km = min(k_merge, pool.size)
        r = oracle.select(np.ascontiguousarray(A[:, pool].T), m, km)
        ns = r["n_selected"]
        out["idx_merge"] = pool[r["idx"][:ns]]
        out["obj_merge"] = r["obj"]
    return out
