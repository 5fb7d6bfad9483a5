"""Per-block budgets l_(b) of Algorithm 4 -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU baseline use this
module; the GPU library computes its budgets itself (gcss_block_budgets).

Section 5.2 (the paragraph after Algorithm 4) leaves the budgets open and
uses l_(b) = floor(l / c) for every one of the c blocks; the naive approach
of Section 5 names l / c and the norm-proportional l ||A_(b)||_F^2 /
||A||_F^2 (a note in the paper's source).  Written from those definitions:

  uniform  floor(l / c), at most the block's width;
  even     l / c,                       rounded by largest remainders;
  norm     l ||A_(b)||^2 / ||A||^2,     rounded by largest remainders
           (l / c for every block when A is zero).

"Rounded by largest remainders": every share is rounded down and capped at
the block's width, then the columns still missing to min(l, n) go one at a
time to the block with the largest (share - budget) among the blocks with
room, the lower block first on equal remainders.
"""
from __future__ import annotations

import math


def budgets(norms2, widths, l, policy):
    """norms2: ||A_(b)||_F^2 per block (floats); widths: columns per block."""
    c = len(widths)
    if c < 1 or l < 0:
        raise ValueError("need at least one block and l >= 0")
    if policy == "uniform":
        return [min(l // c, int(w)) for w in widths]
    total_cols = sum(int(w) for w in widths)
    target = min(int(l), total_cols)
    if policy == "even":
        share = [l / c for _ in range(c)]
    elif policy == "norm":
        tot = float(sum(norms2))
        share = [l * float(x) / tot for x in norms2] if tot > 0 else [l / c for _ in range(c)]
    else:
        raise ValueError(policy)
    out = [min(int(math.floor(s)), int(w)) for s, w in zip(share, widths)]
    while sum(out) < target:
        best, bi = None, -1
        for b in range(c):
            if out[b] < widths[b] and (best is None or share[b] - out[b] > best):
                best, bi = share[b] - out[b], b
        out[bi] += 1
    return out
