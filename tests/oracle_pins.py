"""Pins of the CPU oracle to facts fixed outside the oracle itself.

Each ``pin_*`` function takes an :class:`oracle.Oracle` and raises
``AssertionError`` when the oracle disagrees with:

* values printed in the paper (the worked bit example of Section 2.1, the
  combination counts of Table 'cells_per_order');
* library routines (scikit-learn's ``mutual_info_score``, SciPy's G-test);
* brute force on tiny inputs (numpy ``bincount`` over the mixed-radix cell
  index, and the paper's own bitset formulation: AND of genotype rows, then
  popcount);
* closed forms and invariants of mutual information and of the tables.

``tests/test_oracle_pins.py`` runs every pin on the real oracle;
``tests/test_oracle_mutants.py`` runs them on deliberately broken copies of the
oracle source and checks that each break is caught.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

from synth import random_genotypes

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---- independent brute-force helpers (not the oracle's code path) ---------

def bincount_table(G, y, combo):
    """2 x 3^k table via numpy bincount of the mixed-radix cell index."""
    k = len(combo)
    x = np.zeros(G.shape[1], np.int64)
    for c in combo:
        x = x * 3 + G[c].astype(np.int64)
    cases = np.bincount(x[y == 1], minlength=3**k)
    ctrls = np.bincount(x[y == 0], minlength=3**k)
    return np.stack([cases, ctrls]).astype(np.int64)


def bitset_table(G, y, combo):
    """2 x 3^k table the paper's way: per-class genotype rows as bitsets,
    AND across the SNPs of the combination, popcount (Sections 2.1-2.2)."""
    k = len(combo)
    out = np.zeros((2, 3**k), np.int64)
    for cls, sel in ((0, y == 1), (1, y == 0)):
        idx = np.nonzero(sel)[0]
        rows = []
        for c in combo:
            g = G[c, idx]
            rows.append([sum(1 << b for b in np.nonzero(g == v)[0].tolist()) for v in range(3)])
        for cell, gs in enumerate(itertools.product(range(3), repeat=k)):
            acc = (1 << len(idx)) - 1
            for t, v in enumerate(gs):
                acc &= rows[t][v]
            out[cls, cell] = bin(acc).count("1")
    return out


def sklearn_mi(G, y, combo):
    from sklearn.metrics import mutual_info_score

    x = np.zeros(G.shape[1], np.int64)
    for c in combo:
        x = x * 3 + G[c].astype(np.int64)
    return float(mutual_info_score(y, x))


def gtest_mi(table):
    """MI = G / (2 m) with G the log-likelihood-ratio statistic (SciPy)."""
    from scipy.stats import chi2_contingency

    t = np.asarray(table, np.float64)
    t = t[:, t.sum(axis=0) > 0]
    if t.shape[1] < 2 or (t.sum(axis=1) == 0).any():
        return 0.0
    g, _, _, _ = chi2_contingency(t, correction=False, lambda_="log-likelihood")
    return float(g) / (2.0 * t.sum())


def _bits(s):
    return [int(ch) for ch in s]


def fig_example_inputs():
    """Genotypes and phenotype rebuilt from the printed rows of Fig. gt_example:
    16 cases then 16 controls; an individual's genotype at a SNP is the index
    of the row whose bit is set for it."""
    with open(os.path.join(GOLDEN, "fig_gt_example.json")) as f:
        doc = json.load(f)
    G = np.zeros((2, 32), np.uint8)
    for s, key in enumerate(("snp_i", "snp_j")):
        for off, cls in ((0, "cases"), (16, "ctrls")):
            rows = [_bits(r) for r in doc[key][cls]]
            for b in range(16):
                hot = [r for r in range(3) if rows[r][b]]
                assert len(hot) == 1, "printed rows must be disjoint and cover every individual"
                G[s, off + b] = hot[0]
    y = np.array([1] * 16 + [0] * 16, np.uint8)
    return G, y, doc


# ---- pins -----------------------------------------------------------------

def pin_fig_gt_example(o):
    G, y, doc = fig_example_inputs()
    tab = o.count_table(G, y, [0, 1]).astype(np.int64)
    # Every printed combined row: its popcount is the cell count.
    for row in doc["combined_printed"]:
        cell = row["i"] * 3 + row["j"]
        assert tab[0, cell] == row["cases"].count("1"), ("cases", row)
        assert tab[1, cell] == row["ctrls"].count("1"), ("ctrls", row)
    # All nine cells: AND of the printed input rows, then popcount.
    for cls, key in ((0, "cases"), (1, "ctrls")):
        for a in range(3):
            for b in range(3):
                want = bin(int(doc["snp_i"][key][a], 2) & int(doc["snp_j"][key][b], 2)).count("1")
                assert tab[cls, a * 3 + b] == want, (key, a, b)
    mi = o.mi(tab)
    assert abs(mi - sklearn_mi(G, y, [0, 1])) < 1e-12
    assert abs(mi - gtest_mi(tab)) < 1e-12


def pin_tables_brute_force(o, seed=11):
    for M, N, k in ((5, 37, 1), (6, 64, 2), (6, 65, 3), (5, 29, 4), (5, 40, 5)):
        G, y = random_genotypes(M, N, seed=seed + M * 100 + N + k, case_fraction=0.4)
        for combo in itertools.combinations(range(M), k):
            tab = o.count_table(G, y, combo).astype(np.int64)
            assert np.array_equal(tab, bincount_table(G, y, combo)), (M, N, combo)
    for M, N, k in ((4, 33, 2), (4, 31, 3)):
        G, y = random_genotypes(M, N, seed=seed + 7 * N + k, case_fraction=0.5)
        for combo in itertools.combinations(range(M), k):
            assert np.array_equal(o.count_table(G, y, combo).astype(np.int64), bitset_table(G, y, combo))


def pin_table_invariants(o, seed=12):
    G, y = random_genotypes(7, 91, seed=seed, case_fraction=0.3)
    n_case, n_ctrl = int(y.sum()), int((1 - y).sum())
    for k in (2, 3, 4):
        for combo in itertools.islice(itertools.combinations(range(7), k), 12):
            tab = o.count_table(G, y, combo).astype(np.int64).reshape((2,) + (3,) * k)
            assert tab[0].sum() == n_case and tab[1].sum() == n_ctrl
            # summing out the last SNP gives the table of the prefix
            pref = o.count_table(G, y, combo[:-1]).astype(np.int64).reshape((2,) + (3,) * (k - 1))
            assert np.array_equal(tab.sum(axis=-1), pref)
            # summing out all but SNP t gives that SNP's per-class genotype counts
            for t, c in enumerate(combo):
                axes = tuple(1 + u for u in range(k) if u != t)
                single = o.count_table(G, y, [c]).astype(np.int64)
                assert np.array_equal(tab.sum(axis=axes), single)
            # permuting the SNPs permutes the table axes
            perm = list(reversed(range(k)))
            tab_p = o.count_table(G, y, [combo[p] for p in perm]).astype(np.int64).reshape((2,) + (3,) * k)
            assert np.array_equal(tab_p, np.transpose(tab, [0] + [1 + p for p in perm]))


def pin_mi_library(o, seed=13):
    for M, N, k, frac in ((6, 50, 2, 0.5), (6, 301, 3, 0.25), (5, 1000, 4, 0.7), (6, 77, 5, 0.45)):
        G, y = random_genotypes(M, N, seed=seed + N, case_fraction=frac)
        for combo in itertools.islice(itertools.combinations(range(M), k), 6):
            tab = o.count_table(G, y, combo)
            mi = o.mi(tab)
            ref = sklearn_mi(G, y, combo)
            assert abs(mi - ref) <= 1e-12 + 1e-10 * abs(ref), (combo, mi, ref)
            ref2 = gtest_mi(tab)
            assert abs(mi - ref2) <= 1e-12 + 1e-10 * abs(ref2), (combo, mi, ref2)


def pin_mi_closed_forms(o, seed=14):
    rng = np.random.default_rng(seed)
    # Independence: every genotype cell holds equal counts in both classes.
    half = rng.integers(0, 3, size=(3, 40)).astype(np.uint8)
    G = np.concatenate([half, half], axis=1)
    y = np.array([1] * 40 + [0] * 40, np.uint8)
    for combo in ((0, 1), (0, 1, 2)):
        assert abs(o.mi(o.count_table(G, y, combo))) < 1e-15
    # Pure cells: the class is a function of the genotypes -> MI = H(Y).
    G = rng.integers(0, 3, size=(3, 120)).astype(np.uint8)
    y = ((G[0].astype(int) + 2 * G[1]) % 3 == 0).astype(np.uint8)
    p = y.mean()
    h_y = -(p * math.log(p) + (1 - p) * math.log(1 - p))
    assert abs(o.mi(o.count_table(G, y, (0, 1))) - h_y) < 1e-12
    # Bounds 0 <= MI <= H(Y) <= ln 2, on random data.
    G, y = random_genotypes(5, 200, seed=seed + 1, case_fraction=0.35)
    p = y.mean()
    h_y = -(p * math.log(p) + (1 - p) * math.log(1 - p))
    for k in (1, 2, 3):
        for combo in itertools.combinations(range(5), k):
            mi = o.mi(o.count_table(G, y, combo))
            assert -1e-15 <= mi <= h_y + 1e-15 <= math.log(2) + 1e-15


def pin_mi_invariances(o, seed=15):
    G, y = random_genotypes(4, 150, seed=seed, case_fraction=0.4)
    rng = np.random.default_rng(seed)
    combo = (0, 2, 3)
    base = o.mi(o.count_table(G, y, combo))
    # swapping the class labels
    assert abs(o.mi(o.count_table(G, 1 - y, combo)) - base) < 1e-14
    # permuting individuals
    perm = rng.permutation(G.shape[1])
    assert abs(o.mi(o.count_table(G[:, perm], y[perm], combo)) - base) < 1e-14
    # relabelling one SNP's genotypes
    G2 = G.copy()
    G2[2] = np.array([2, 0, 1], np.uint8)[G[2]]
    assert abs(o.mi(o.count_table(G2, y, combo)) - base) < 1e-14


def pin_enumeration(o):
    for M in range(1, 12):
        for k in range(1, min(M, 8) + 1):
            assert o.enumerate_count(M, k) == math.comb(M, k) == o.binomial(M, k)
    with open(os.path.join(GOLDEN, "table2_cells_per_order.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        assert r["combinations"] * 3 ** r["size"] == r["total_cells"]
    assert o.enumerate_count(25000, 2) == rows[0]["combinations"]
    assert o.enumerate_count(23, 8) == rows[2]["combinations"]
    # the order-4 row is C(171,4): the printed SNP count 242 is a misprint
    assert o.binomial(171, 4) == rows[1]["combinations"] != o.binomial(242, 4)


def _brute_topk(G, y, k, K):
    rows = []
    for combo in itertools.combinations(range(G.shape[0]), k):
        rows.append((-sklearn_mi(G, y, combo), combo))
    rows.sort()
    return rows[:K]


def pin_topk_brute_force(o, seed=16):
    for M, N, k, K, threads in ((9, 64, 2, 10, 3), (9, 50, 3, 15, 4), (8, 40, 4, 7, 2), (7, 33, 1, 3, 2)):
        G, y = random_genotypes(M, N, seed=seed + M + N + k, case_fraction=0.5)
        ref = _brute_topk(G, y, k, K)
        got = o.scan(G, y, k, K, nthreads=threads)
        assert len(got["combos"]) == len(ref)
        for (neg, combo), gc, gs in zip(ref, got["combos"], got["scores"]):
            assert abs(gs + neg) < 1e-12
            if tuple(gc) != combo:
                # only an exact-score tie may reorder
                assert abs(o.mi(o.count_table(G, y, combo)) - gs) < 1e-14, (combo, tuple(gc))
        # the returned tables are the tables of the returned combinations
        for gc, tab in zip(got["combos"], got["tables"]):
            assert np.array_equal(tab.astype(np.int64), bincount_table(G, y, gc))


def pin_topk_lex_ties(o):
    # identical SNPs -> every combination has the same table and MI;
    # the order must then be lexicographic
    G0, y = random_genotypes(1, 60, seed=17, case_fraction=0.5)
    G = np.repeat(G0, 7, axis=0)
    for k in (2, 3):
        got = o.scan(G, y, k, math.comb(7, k), nthreads=3)
        assert [tuple(c) for c in got["combos"]] == list(itertools.combinations(range(7), k))


def pin_planted_recovery(o, seed=18):
    # case iff the number of heterozygous loci in the planted set is odd
    rng = np.random.default_rng(seed)
    for k, planted in ((2, (3, 11)), (3, (1, 6, 12))):
        G = rng.choice(3, size=(14, 400), p=[0.25, 0.5, 0.25]).astype(np.uint8)
        y = (sum((G[p] == 1).astype(int) for p in planted) % 2).astype(np.uint8)
        got = o.scan(G, y, k, 3)
        assert tuple(got["combos"][0]) == planted


def pin_rank_ranges(o, seed=19):
    # the union of the best lists of a split of the rank space is the whole
    G, y = random_genotypes(10, 80, seed=seed, case_fraction=0.5)
    whole = o.scan(G, y, 3, 20, nthreads=1)
    n = math.comb(10, 3)
    parts = [o.scan(G, y, 3, 20, rank_begin=b, rank_end=e, nthreads=2)
             for b, e in ((0, 37), (37, 80), (80, n))]
    rows = []
    for p in parts:
        rows += [(-s, tuple(c)) for s, c in zip(p["scores"], p["combos"])]
    rows.sort()
    assert [c for _, c in rows[:20]] == [tuple(c) for c in whole["combos"]]


def pin_score_list(o, seed=21):
    """Tables and MI of an explicit list of combinations, row by row (every
    row, not only the first, so a wrong per-row offset of the combinations,
    tables or scores fails): numpy bincount and scikit-learn, also for lists
    in non-lexicographic order and with repeated combinations."""
    rng = np.random.default_rng(seed)
    for M, N, k, frac in ((9, 70, 2, 0.5), (8, 133, 3, 0.3), (7, 64, 4, 0.55), (6, 41, 5, 0.4)):
        G, y = random_genotypes(M, N, seed=seed + 10 * M + k, case_fraction=frac)
        combos = [tuple(sorted(rng.choice(M, k, replace=False).tolist())) for _ in range(9)]
        combos.append(combos[2])
        scores, tables = o.score_list(G, y, np.asarray(combos, np.int32))
        assert scores.shape == (len(combos),) and tables.shape == (len(combos), 2, 3**k)
        for r, c in enumerate(combos):
            assert np.array_equal(tables[r].astype(np.int64), bincount_table(G, y, c)), (r, c)
            ref = sklearn_mi(G, y, c)
            assert abs(scores[r] - ref) <= 1e-12 + 1e-10 * abs(ref), (r, c, scores[r], ref)
        assert np.array_equal(tables[2], tables[-1]) and scores[2] == scores[-1]


_MASK64 = (1 << 64) - 1


def _splitmix_out(z):
    """SplitMix64's output function (Steele, Lea and Flood, 2014), in Python
    integers reduced modulo 2^64."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def brute_digest(G, y, k):
    """(count, digest) of all k-combinations, written out from the definition:
    h folds the indices, s weighs the table's counts (numpy bincount), the
    contribution is mix(h ^ s), summed modulo 2^64."""
    count, total = 0, 0
    for combo in itertools.combinations(range(G.shape[0]), k):
        h = 0
        for c in combo:
            h = _splitmix_out((h + c + 1) & _MASK64)
        tab = bincount_table(G, y, combo)
        s = 0
        for cls in (0, 1):
            for x in range(3**k):
                s = (s + int(tab[cls, x]) * _splitmix_out(2 * x + cls + 1)) & _MASK64
        total = (total + _splitmix_out(h ^ s)) & _MASK64
        count += 1
    return count, total


def pin_digest(o, seed=22):
    """The completeness digest against its definition written out in Python
    (count = C(M,k)), over rank splits that must add up, for every order."""
    for M, N, k, frac in ((9, 50, 2, 0.5), (8, 67, 3, 0.3), (7, 40, 4, 0.6), (7, 33, 5, 0.45), (9, 20, 8, 0.5)):
        G, y = random_genotypes(M, N, seed=seed + M + k, case_fraction=frac)
        want = brute_digest(G, y, k)
        assert want[0] == math.comb(M, k)
        assert o.digest(G, y, k, nthreads=3) == want, (M, N, k)
        n = math.comb(M, k)
        parts = [o.digest(G, y, k, b, e, nthreads=2) for b, e in ((0, n // 3), (n // 3, n - 1), (n - 1, n))]
        assert sum(p[0] for p in parts) == want[0]
        assert sum(p[1] for p in parts) & _MASK64 == want[1]
    # one count moved between the classes changes the digest
    G, y = random_genotypes(6, 30, seed=seed, case_fraction=0.5)
    y2 = y.copy()
    y2[np.nonzero(y)[0][0]] = 0
    y2[np.nonzero(y == 0)[0][0]] = 1
    assert o.digest(G, y, 3) != o.digest(G, y2, 3)


def _row_bits(word_list, n):
    """First n bits of a row (bit b of word w = individual 32 w + b) as a 0/1 string."""
    return "".join(str((int(word_list[b // 32]) >> (b % 32)) & 1) for b in range(n))


def pin_genotype_rows_fig_example(o):
    """The combined genotype table of Fig. gt_example: the printed rows, bit for
    bit (the misprinted control row by the AND of its printed inputs)."""
    G, y, doc = fig_example_inputs()
    rows = o.genotype_rows(G, y, [0, 1], 1, 1)
    assert rows.shape == (9, 2)
    bad = {(m["i"], m["j"], m["class"]) for m in doc["misprinted_rows"]}
    for row in doc["combined_printed"]:
        x = row["i"] * 3 + row["j"]
        for col, key in ((0, "cases"), (1, "ctrls")):
            if (row["i"], row["j"], key) in bad:
                want = int(doc["snp_i"][key][row["i"]], 2) & int(doc["snp_j"][key][row["j"]], 2)
                want = format(want, "016b")
            else:
                want = row[key]
            assert _row_bits(rows[x, col:col + 1], 16) == want, (row, key)
    # single-SNP tables are the printed input rows themselves
    for s, key in enumerate(("snp_i", "snp_j")):
        r1 = o.genotype_rows(G, y, [s], 1, 1)
        for g in range(3):
            assert _row_bits(r1[g, 0:1], 16) == doc[key]["cases"][g]
            assert _row_bits(r1[g, 1:2], 16) == doc[key]["ctrls"][g]


def pin_genotype_rows_invariants(o, seed=20):
    """Rows of a class partition its individuals, hold nothing past its size,
    and their popcounts are the contingency table; a row is the AND of the
    rows of its SNPs (the combine step of Algorithm 1)."""
    G, y = random_genotypes(6, 150, seed=seed, case_fraction=0.35)
    n = (int(y.sum()), int((1 - y).sum()))
    words = (4 * ((n[0] + 127) // 128), 4 * ((n[1] + 127) // 128))
    for k in (1, 2, 3, 4):
        for combo in itertools.islice(itertools.combinations(range(6), k), 6):
            rows = o.genotype_rows(G, y, combo, *words).astype(np.uint64)
            tab = o.count_table(G, y, combo).astype(np.int64)
            for cls in (0, 1):
                part = rows[:, (0 if cls == 0 else words[0]):(words[0] if cls == 0 else words[0] + words[1])]
                bits = np.unpackbits(part.astype("<u4").view(np.uint8), bitorder="little").reshape(len(part), -1)
                assert np.array_equal(bits.sum(axis=1), tab[cls])
                assert np.array_equal(bits.sum(axis=0)[: n[cls]], np.ones(n[cls], np.int64))
                assert bits[:, n[cls]:].sum() == 0
            if k > 1:
                pref = o.genotype_rows(G, y, combo[:-1], *words)
                last = o.genotype_rows(G, y, combo[-1:], *words)
                for x in range(3**k):
                    assert np.array_equal(rows[x].astype(np.uint32), pref[x // 3] & last[x % 3])


ALL_PINS = [
    pin_fig_gt_example,
    pin_genotype_rows_fig_example,
    pin_genotype_rows_invariants,
    pin_tables_brute_force,
    pin_table_invariants,
    pin_mi_library,
    pin_mi_closed_forms,
    pin_mi_invariances,
    pin_enumeration,
    pin_topk_brute_force,
    pin_topk_lex_ties,
    pin_planted_recovery,
    pin_rank_ranges,
    pin_score_list,
    pin_digest,
]


def run_battery(o):
    """Run every pin; return the names of those that fail (any exception)."""
    failed = []
    for pin in ALL_PINS:
        try:
            pin(o)
        except Exception:  # noqa: BLE001 - a crash of a broken oracle is a failure too
            failed.append(pin.__name__)
    return failed
