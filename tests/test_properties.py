"""Property tests over random shapes (hypothesis).

CPU: the oracle against independent brute force on arbitrary small inputs,
including class sizes at the 32/64/128-individual word edges, identical SNPs
and SNPs with a single genotype.  GPU: the HIP scan against the oracle on the
same kind of inputs, end to end through the C ABI.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle_pins import bincount_table, sklearn_mi


@st.composite
def datasets(draw, max_m=9, orders=(1, 2, 3, 4)):
    """(G, y, k): genotypes with some identical and some single-genotype SNPs,
    class sizes drawn near multiples of 32, 64 and 128."""
    k = draw(st.sampled_from(orders))
    M = draw(st.integers(min_value=max(k, 2), max_value=max_m))
    edge = draw(st.sampled_from([0, 1, 31, 32, 33, 63, 64, 65, 127, 128, 129]))
    n_case = max(1, edge + draw(st.integers(min_value=0, max_value=2)))
    n_ctrl = max(1, draw(st.sampled_from([1, 2, 63, 64, 65, 100, 128, 150])))
    seed = draw(st.integers(min_value=0, max_value=2**31 - 1))
    rng = np.random.default_rng(seed)
    N = n_case + n_ctrl
    p = rng.dirichlet(np.ones(3))
    G = rng.choice(3, size=(M, N), p=p).astype(np.uint8)
    if draw(st.booleans()):
        G[M - 1] = G[0]  # an identical pair of SNPs
    if draw(st.booleans()):
        G[M // 2] = draw(st.integers(min_value=0, max_value=2))  # a single-genotype SNP
    y = np.zeros(N, np.uint8)
    y[rng.permutation(N)[:n_case]] = 1
    return G, y, k


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(datasets())
def test_oracle_tables_rows_and_mi(orc, data):
    G, y, k = data
    n = (int(y.sum()), int((1 - y).sum()))
    words = (4 * ((n[0] + 127) // 128), 4 * ((n[1] + 127) // 128))
    for combo in itertools.islice(itertools.combinations(range(G.shape[0]), k), 6):
        tab = orc.count_table(G, y, combo).astype(np.int64)
        assert np.array_equal(tab, bincount_table(G, y, combo))
        rows = orc.genotype_rows(G, y, combo, *words)
        pop = np.unpackbits(rows.astype("<u4").view(np.uint8), bitorder="little").reshape(3**k, 2, -1)
        pop = pop.reshape(3**k, -1)
        assert np.array_equal(pop[:, : 32 * words[0]].sum(axis=1), tab[0])
        assert np.array_equal(pop[:, 32 * words[0]:].sum(axis=1), tab[1])
        mi = orc.mi(tab)
        hy = -sum(c / sum(n) * math.log(c / sum(n)) for c in n)
        assert -1e-12 <= mi <= hy + 1e-12
        assert abs(mi - sklearn_mi(G, y, combo)) < 1e-10


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(datasets(orders=(2, 3, 4)), st.integers(min_value=1, max_value=20))
def test_oracle_rank_ranges_compose(orc, data, K):
    G, y, k = data
    total = math.comb(G.shape[0], k)
    cut = total // 2
    full = orc.scan(G, y, k, K, tables=False)
    a = orc.scan(G, y, k, K, rank_end=cut, tables=False)
    b = orc.scan(G, y, k, K, rank_begin=cut, tables=False)
    merged = sorted([(-s, tuple(c)) for part in (a, b) for c, s in zip(part["combos"], part["scores"])])[:K]
    assert [c for _, c in merged] == [tuple(c) for c in full["combos"]]


@pytest.mark.gpu
@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow,
                                                                 HealthCheck.function_scoped_fixture])
@given(datasets(max_m=12, orders=(2, 3, 4, 5)), st.integers(min_value=1, max_value=30))
def test_gpu_scan_matches_oracle(orc, data, K):
    from parity import check_topk

    from paper_2201_02460_amd import epi

    G, y, k = data
    print("property case M", G.shape[0], "N", G.shape[1], "cases", int(y.sum()), "order", k, "K", K, flush=True)
    with epi.Context(0) as cx:
        ds = cx.load(G, y)
        try:
            res = cx.scan(ds, k, K)
        finally:
            epi.epi_unload(cx.ctx, ds)
    check_topk(orc, G, y, k, K, res["combos"], res["scores"], res["tables"])
