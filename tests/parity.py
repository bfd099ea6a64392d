"""Comparison of GPU scan results with the CPU oracle.

The bar (per returned combination and per result set):
* every returned contingency table equals the oracle's table bit for bit;
* every returned float32 score is within 1e-5 relative of the oracle's
  float64 MI of that combination (an absolute 1e-9 only where the oracle's
  MI is zero up to its own float64 rounding, |MI| <= 1e-12);
* the returned float32 scores never increase; where two of them are equal
  and the later combination is lexicographically smaller, the two tables
  must not hold the same multiset of cells (then their exact fixed-point
  scores are equal and the tie goes to the smaller combination), and the
  oracle must not rank the later one higher by more than 1e-9 relative (two
  different MI values that round to the same float32, or equal MI values
  whose fixed-point sums differ in the last units);
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
    # a zero MI (the oracle's float64 value is then its own rounding) is
    # allowed an absolute slack instead
    zero = np.abs(o_scores) <= 1e-12
    ok = (err <= REL_TOL) | (zero & (np.abs(np.asarray(scores, np.float64) - o_scores) <= 1e-9))
    assert ok.all(), f"score error {err[~ok].max():.3e} > {REL_TOL}"
    return o_scores


def cell_terms(table):
    """The multiset of a table's mixed cells (both classes present) as
    unordered (n_case, n_control) pairs.  The score is a sum of one term per
    cell, symmetric in the two counts and exactly zero for a cell with an
    empty class, so tables with the same multiset have the same score in any
    arithmetic."""
    t = np.asarray(table, np.int64).reshape(2, -1)
    lo, hi = np.minimum(t[0], t[1]), np.maximum(t[0], t[1])
    keep = lo > 0
    return sorted(zip(lo[keep].tolist(), hi[keep].tolist()))


def check_order(combos, scores, o_scores, tables):
    """Best first (see the module docstring)."""
    got = [tuple(int(v) for v in c) for c in combos]
    s = np.asarray(scores, np.float32)
    for r in range(1, len(got)):
        assert s[r] <= s[r - 1], f"rank {r}: score {s[r]} above the previous {s[r - 1]}"
        if s[r] == s[r - 1] and got[r] < got[r - 1]:
            assert cell_terms(tables[r]) != cell_terms(tables[r - 1]), \
                f"rank {r}: exact tie {got[r - 1]}, {got[r]} not in lexicographic order"
            assert o_scores[r] - o_scores[r - 1] <= 1e-9 * abs(o_scores[r]), \
                f"rank {r}: equal scores, the later combination is better by the oracle"


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
    check_order(combos, scores, o_scores, tables)
    kth = ref_scores[-1]
    tol = REL_TOL * max(abs(kth), 1e-30) + 1e-12
    for c in set(got) ^ set(ref_combos):
        if c in set(got):
            s = o_scores[got.index(c)]
        else:
            s = ref_scores[ref_combos.index(c)]
        assert abs(s - kth) <= tol, f"set differs beyond a tie at the K-th score: {c} (score {s}, K-th {kth})"
