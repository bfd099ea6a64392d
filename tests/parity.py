"""Comparison of GPU scan results with the CPU oracle.

The bar (per returned combination and per result set):
* every returned contingency table equals the oracle's table bit for bit;
* every returned float32 score is within 1e-5 relative of the oracle's
  float64 MI of that combination;
* scores are non-increasing, and equal scores list the lexicographically
  smaller combination first;
* the returned set equals the oracle's best-K set, except that a member may
  be swapped with a non-member whose oracle score is within 1e-5 relative of
  the oracle's K-th score (a tie inside the tolerance).
"""
from __future__ import annotations

import numpy as np

REL_TOL = 1e-5


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-30)


def check_scores_tables(orc, G, y, combos, scores, tables):
    """Oracle recount of every returned combination (one by one)."""
    if len(combos) == 0:
        return
    o_scores, o_tables = orc.score_list(G, y, combos)
    assert np.array_equal(np.asarray(tables, np.int64), o_tables.astype(np.int64)), "tables differ from oracle"
    err = rel_err(scores, o_scores)
    # an exactly-zero MI is allowed an absolute slack of the same size
    ok = (err <= REL_TOL) | (np.abs(np.asarray(scores, np.float64) - o_scores) <= 1e-9)
    assert ok.all(), f"score error {err.max():.3e} > {REL_TOL}"
    return o_scores


def check_topk(orc, G, y, order, top_k, combos, scores, tables, ref=None):
    """Full check against the oracle's best-K (``ref`` = precomputed oracle result)."""
    combos = np.asarray(combos)
    scores = np.asarray(scores, np.float64)
    o_scores = check_scores_tables(orc, G, y, combos, scores, tables)
    if ref is None:
        ref = orc.scan(G, y, order, top_k, tables=False)
    ref_combos = [tuple(int(v) for v in c) for c in ref["combos"]]
    ref_scores = np.asarray(ref["scores"], np.float64)
    assert len(combos) == len(ref_combos), f"{len(combos)} results, oracle has {len(ref_combos)}"
    if len(combos) == 0:
        return
    for c in combos:
        assert all(c[t] < c[t + 1] for t in range(order - 1)), f"indices not ascending: {c}"
    got = [tuple(int(v) for v in c) for c in combos]
    assert len(set(got)) == len(got), "duplicate combinations returned"
    # order: by oracle score (non-increasing within tolerance), ties lexicographic
    for r in range(1, len(got)):
        assert o_scores[r] <= o_scores[r - 1] * (1 + 2 * REL_TOL) + 1e-12, f"rank {r} out of order"
    kth = ref_scores[-1]
    tol = REL_TOL * max(abs(kth), 1e-30) + 1e-12
    for c in set(got) ^ set(ref_combos):
        if c in set(got):
            s = o_scores[got.index(c)]
        else:
            s = ref_scores[ref_combos.index(c)]
        assert abs(s - kth) <= tol, f"set differs beyond a tie at the K-th score: {c} (score {s}, K-th {kth})"
