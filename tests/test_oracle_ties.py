"""Pins of the oracle's argmax tie rule and a mutation check of the pins.

The paper leaves ties in the argmax of Algorithms 1 and 3 open; the reading
taken here is that the lowest column index wins.  Exact ties are built so
that both candidates' scores are bitwise equal in FP64: orthogonal columns
with equal integer squared norms (closed form of Theorem 2, golden file) and
exact duplicate columns, for B = A and for an explicit target.

The mutation check compiles altered copies of the C oracle (a planted
mistake each: ties to the highest index, the residual Gram column without
the earlier picks' share, a flipped sign in the f update, a dropped g
update) and requires that every one of them fails at least one pin while
the real oracle passes them all.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def cs(M):
    return synth.to_colstore(M, lda=M.shape[0], dtype=np.float64)


def _tie_golden():
    return json.load(open(os.path.join(GOLD, "orthogonal_columns_ties.json")))


def _dup_matrix(seed):
    """Random 12 x 30 matrix whose columns 4 and 17 are one dominant column."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((12, 30))
    v = 5.0 * rng.standard_normal(12)
    A[:, 4] = v
    A[:, 17] = v
    return A


# ---- pin checks (each returns a failure message or None) ---------------------
def check_orthogonal_ties():
    gold = _tie_golden()
    A = synth.orthogonal_columns_dense(gold["sq_norms"])
    m, n = A.shape
    for B in (None, cs(A.copy())):
        res = oracle.select(cs(A), m, n, B=B, tau=1e-12)
        if list(res["idx"]) != gold["order"]:
            return f"order {list(res['idx'])} != {gold['order']}"
        if np.max(np.abs(res["obj"] - np.array(gold["objective"]))) > 1e-12:
            return "objective off the closed form"
    return None


def check_duplicate_winners():
    for seed in range(3):
        A = _dup_matrix(seed)
        m = A.shape[0]
        rng = np.random.default_rng(50 + seed)
        for B in (None, A @ rng.standard_normal((A.shape[1], 5))):
            res = oracle.select(cs(A), m, 3, B=None if B is None else cs(B))
            # the duplicate pair holds the largest score by construction
            Bv = A if B is None else B
            sc = np.sum((Bv.T @ A) ** 2, axis=0) / np.sum(A * A, axis=0)
            if np.delete(sc, [4, 17]).max() >= 0.9 * min(sc[4], sc[17]):
                return "construction: duplicates are not the best candidates"
            if res["idx"][0] != 4:
                return f"seed {seed}: first pick {res['idx'][0]}, want 4 (lowest duplicate)"
            if 17 in list(res["idx"]):
                return f"seed {seed}: the second copy was picked"
    return None


def check_bruteforce_steps():
    for seed in range(3):
        rng = np.random.default_rng(200 + seed)
        m, n = 8, 11
        A = rng.standard_normal((m, n))
        for B in (None, rng.standard_normal((m, 3))):
            k = 4
            res = oracle.select(cs(A), m, k, B=None if B is None else cs(B), trace=True)
            S, F, decs = brute.greedy(A, B, k)
            F0 = F[0]
            for t in range(k):
                f, g = res["fg"][t]
                cand = ~np.isnan(decs[t])
                if np.max(np.abs(f[cand] / g[cand] - decs[t][cand])) > 1e-9 * F0:
                    return f"seed {seed} step {t}: scores differ from brute force"
                if abs(res["obj"][t + 1] - F[t + 1]) > 1e-9 * F0 and list(res["idx"][:t + 1]) == S[:t + 1]:
                    return f"seed {seed} step {t}: objective differs from brute force"
    return None


PINS = [check_orthogonal_ties, check_duplicate_winners, check_bruteforce_steps]


# ---- the pins on the real oracle --------------------------------------------
def test_tie_golden_orthogonal_columns():
    assert check_orthogonal_ties() is None


def test_duplicate_columns_lowest_index_wins():
    assert check_duplicate_winners() is None


def test_bruteforce_checks_hold():
    assert check_bruteforce_steps() is None


# ---- planted mistakes --------------------------------------------------------
MUTANTS = {
    "ties_to_highest_index": ("if (s > s1) {", "if (s >= s1) {"),
    "gram_column_without_history": (
        "    for (int32_t s = 0; s < t; ++s) d -= wp[s] * W[(size_t)s * n + i];\n",
        ""),
    "f_update_sign": ("f[i] = f[i] - 2.0 * w * hu[i] + un * w * w;",
                      "f[i] = f[i] + 2.0 * w * hu[i] + un * w * w;"),
    "g_not_updated": ("g[i] = g[i] - w * w;", "g[i] = g[i];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_planted_mistake_fails_a_pin(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    text = oracle.source()
    assert text.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    lib = oracle.build_variant(text.replace(old, new), str(tmp_path), name)
    monkeypatch.setattr(oracle, "_lib", lib)
    failures = []
    for pin in PINS:
        try:
            msg = pin()
        except Exception as e:  # a mutant may also break an invariant loudly
            msg = f"raised {type(e).__name__}: {e}"
        if msg:
            failures.append(f"{pin.__name__}: {msg}")
    assert failures, f"mutant {name} passed every pin"
