"""Naive distributed column subset selection (Section 5, the approach the
paper sets out to improve on): every block of columns selects against its
own data (B_(b) = A_(b), Algorithm 1 on the block), the union L of the picks
is the result, optionally reduced by a selection over the pooled columns
A_{:L} against themselves.  Per-block budgets l_(b): uniform (l / c, the
remainder to the first blocks) or adaptive (l ||A_(b)||_F^2 / ||A||_F^2,
rounded by largest remainders; a note in the paper's source names both).

Every selection, norm and gather runs in the library: one context per block
over the block's columns (a view into A), one over the gathered pool.
"""
from __future__ import annotations

import numpy as np


def block_budgets(norms2, widths, l, policy="uniform"):
    """Integer budgets summing to min(l, sum of widths), each <= its block
    width: the library's largest-remainder rounding of l / c ('uniform') or
    of the norm shares ('adaptive')."""
    from . import _abi
    widths = np.asarray(widths, dtype=np.int64)
    col_off = np.concatenate([[0], np.cumsum(widths)]).astype(np.int64)
    pol = {"uniform": "even", "adaptive": "norm"}[policy]
    return _abi.block_budgets(None, col_off, int(l), pol, norms2).astype(np.int64)


def naive_select(A, m, col_off, l, k_merge=0, policy="uniform", scales=None, tau=0.0):
    """A: (n, lda) column store on the GPU; col_off: c+1 block offsets.
    Returns dict(budgets, idx_block (list of arrays, global indices),
    pool, obj_block (final per-block objectives), idx_merge, obj_merge)."""
    from . import Selector
    col_off = [int(x) for x in col_off]
    c = len(col_off) - 1
    widths = [col_off[b + 1] - col_off[b] for b in range(c)]
    sels = []
    norms2 = []
    for b in range(c):
        o0, o1 = col_off[b], col_off[b + 1]
        sc = scales[o0:o1] if scales is not None else None
        s = Selector(A[o0:o1], m, k_max=max(1, min(widths[b], int(l))), self_target=True,
                     scales=sc, tau=tau)
        s.set_target(None)
        sels.append(s)
        norms2.append(s.reconstruction_error(np.zeros(0, dtype=np.int64)))
    budgets = block_budgets(norms2, widths, l, policy)
    idx_block, obj_block = [], []
    for b, s in enumerate(sels):
        if budgets[b] == 0:
            idx_block.append(np.zeros(0, dtype=np.int64))
            obj_block.append(norms2[b])
            continue
        idx, obj, ns, st = s.select(int(budgets[b]))
        idx_block.append(idx[:ns] + col_off[b])
        obj_block.append(float(obj[ns]))
        s.close()
    pool = np.concatenate(idx_block) if idx_block else np.zeros(0, dtype=np.int64)
    out = dict(budgets=budgets, idx_block=idx_block, pool=pool, obj_block=obj_block,
               norms2=norms2, idx_merge=None, obj_merge=None)
    if k_merge and pool.size:
        km = int(min(k_merge, pool.size))
        full = Selector(A, m, k_max=1, r_max=0, self_target=True, scales=scales)
        P, Ps = full.gather(pool)
        full.close()
        sp = Selector(P, m, k_max=km, self_target=True, scales=Ps, tau=tau)
        sp.set_target(None)
        loc, obj, ns, st = sp.select(km)
        out["idx_merge"] = pool[loc[:ns]]
        out["obj_merge"] = obj
        sp.close()
    return out
