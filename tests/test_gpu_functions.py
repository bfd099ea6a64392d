"""The steps of the method as separate passes (genotype tables, contingency
tables, mutual information) through the C ABI, against the oracle (needs an
MI355X)."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from synth import random_genotypes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def cx():
    from paper_2201_02460_amd import epi

    with epi.Context(0) as c:
        yield c


def _combos(M, k, n, seed):
    """n combinations of k indices in [0, M): the first few in lexicographic
    order, then random ones (unsorted, repeats allowed)."""
    rng = np.random.default_rng(seed)
    head = list(itertools.islice(itertools.combinations(range(M), k), n // 2))
    tail = [rng.integers(0, M, size=k).tolist() for _ in range(n - len(head))]
    return np.asarray(head + tail, np.int32).reshape(n, k)


def _words(y):
    n_case = int(y.sum())
    return 4 * ((n_case + 127) // 128), 4 * ((len(y) - n_case + 127) // 128)


# orders 1..8; class sizes spanning several 128-individual groups with ragged tails
GT_CASES = [(1, 9, 300, 129), (2, 12, 257, 128), (3, 10, 700, 300), (4, 9, 130, 1), (5, 8, 385, 200),
            (6, 8, 64, 32), (7, 9, 129, 64), (8, 10, 200, 70)]


@pytest.mark.parametrize("order,M,N,nc", GT_CASES, ids=lambda v: str(v))
def test_genotype_tables_vs_oracle(cx, orc, order, M, N, nc):
    import torch

    from paper_2201_02460_amd import epi

    say("gt case", order, M, N, nc)
    G, y = random_genotypes(M, N, seed=900 + order, case_fraction=nc / N)
    ds = cx.load(G, y)
    try:
        n = 12
        combos = _combos(M, order, n, seed=order)
        W0, W1 = _words(y)
        rows = torch.full((n, 3**order, W0 + W1), 0xABCD, dtype=torch.int32, device="cuda")
        ms = epi.epi_genotype_tables(cx.ctx, ds, torch.from_numpy(combos).cuda(), rows)
        got = rows.cpu().numpy().view(np.uint32)
        for i, c in enumerate(combos):
            want = orc.genotype_rows(G, y, c, W0, W1)
            assert np.array_equal(got[i], want), (i, c)
        assert ms >= 0
    finally:
        epi.epi_unload(cx.ctx, ds)


@pytest.mark.parametrize("N,nc", [(129, 64), (256, 128), (300, 1), (1000, 999), (4097, 2048)])
def test_packing_round_trip(cx, N, nc):
    """unpack(pack(G)) = G: the order-1 genotype tables of every SNP are the
    packed rows; in each class every individual is in exactly one of them
    (its genotype), and bits past the class are zero."""
    import torch

    from paper_2201_02460_amd import epi

    M = 37
    G, y = random_genotypes(M, N, seed=N + nc, case_fraction=nc / N)
    G[5] = 2  # a SNP with one genotype only
    ds = cx.load(G, y)
    try:
        W0, W1 = _words(y)
        combos = torch.arange(M, dtype=torch.int32, device="cuda").reshape(M, 1)
        rows = torch.zeros((M, 3, W0 + W1), dtype=torch.int32, device="cuda")
        epi.epi_genotype_tables(cx.ctx, ds, combos, rows)
        r = rows.cpu().numpy().view(np.uint32)
        bits = np.unpackbits(r.astype("<u4").view(np.uint8), bitorder="little").reshape(M, 3, -1)
        for cls, idx, lo, words in ((0, np.flatnonzero(y == 1), 0, W0), (1, np.flatnonzero(y == 0), W0, W1)):
            b = bits[:, :, 32 * lo: 32 * (lo + words)]
            n = len(idx)
            assert (b.sum(axis=1)[:, :n] == 1).all(), "every individual in exactly one genotype row"
            assert b[:, :, n:].sum() == 0, "pad bits are zero"
            assert np.array_equal(b[:, :, :n].argmax(axis=1), G[:, idx]), "rows decode to the genotypes"
    finally:
        epi.epi_unload(cx.ctx, ds)


CT_CASES = [(2, 40, 1000, 450), (3, 20, 257, 100), (4, 12, 640, 511), (5, 10, 129, 64), (6, 9, 300, 150),
            (7, 9, 200, 80), (8, 10, 385, 129)]


@pytest.mark.parametrize("order,M,N,nc", CT_CASES, ids=lambda v: str(v))
def test_tables_and_mi_vs_oracle(cx, orc, order, M, N, nc):
    import torch

    from paper_2201_02460_amd import epi

    say("ct/mi case", order, M, N, nc)
    G, y = random_genotypes(M, N, seed=950 + order, case_fraction=nc / N)
    ds = cx.load(G, y)
    try:
        n = 300
        combos = _combos(M, order, n, seed=50 + order)
        tabs = torch.zeros((n, 2, 3**order), dtype=torch.int32, device="cuda")
        epi.epi_contingency_tables(cx.ctx, ds, torch.from_numpy(combos).cuda(), tabs)
        got = tabs.cpu().numpy().view(np.uint32).astype(np.int64)
        mi = torch.zeros(n, dtype=torch.float64, device="cuda")
        epi.epi_mutual_information(cx.ctx, ds, order, tabs, mi)
        mi = mi.cpu().numpy()
        # exact fixed-point sum: 3^k + 1 cell terms of 3 table entries, each
        # rounded to 2^-shift with shift >= 35 for N below about 2 million
        tol = (3 * 3**order + 3) * 2.0**-35 / N + 1e-12
        for i, c in enumerate(combos):
            want = orc.count_table(G, y, c).astype(np.int64)
            assert np.array_equal(got[i], want), (i, c)
            assert abs(mi[i] - orc.mi(want)) <= tol, (i, c, mi[i], orc.mi(want))
    finally:
        epi.epi_unload(cx.ctx, ds)


def test_mi_equals_scan_scores(cx, orc):
    """MI of the tables of a scan's results is the scan's score (float)."""
    import torch

    from paper_2201_02460_amd import epi

    G, y = random_genotypes(60, 777, seed=31, case_fraction=0.4)
    ds = cx.load(G, y)
    try:
        for order in (2, 3, 4, 5):
            res = cx.scan(ds, order, 20)
            combos = torch.from_numpy(np.ascontiguousarray(res["combos"], np.int32)).cuda()
            tabs = torch.zeros((len(res["combos"]), 2, 3**order), dtype=torch.int32, device="cuda")
            epi.epi_contingency_tables(cx.ctx, ds, combos, tabs)
            assert np.array_equal(tabs.cpu().numpy().view(np.uint32), res["tables"])
            mi = torch.zeros(len(res["combos"]), dtype=torch.float64, device="cuda")
            epi.epi_mutual_information(cx.ctx, ds, order, tabs, mi)
            assert np.array_equal(mi.cpu().numpy().astype(np.float32), res["scores"])
    finally:
        epi.epi_unload(cx.ctx, ds)


def test_function_errors(cx):
    import torch

    from paper_2201_02460_amd import epi

    G, y = random_genotypes(10, 100, seed=3)
    ds = cx.load(G, y)
    try:
        W0, W1 = _words(y)
        bad = torch.tensor([[0, 1], [3, 10]], dtype=torch.int32, device="cuda")  # index 10 == M
        rows = torch.zeros((2, 9, W0 + W1), dtype=torch.int32, device="cuda")
        with pytest.raises(epi.EpiError) as e:
            epi.epi_genotype_tables(cx.ctx, ds, bad, rows)
        assert e.value.code == epi.EPI_EINVAL
        tabs = torch.zeros((2, 2, 9), dtype=torch.int32, device="cuda")
        with pytest.raises(epi.EpiError) as e:
            epi.epi_contingency_tables(cx.ctx, ds, bad, tabs)
        assert e.value.code == epi.EPI_EINVAL
        # the valid combination's table is still written
        good = torch.tensor([[0, 1]], dtype=torch.int32, device="cuda")
        t1 = torch.zeros((1, 2, 9), dtype=torch.int32, device="cuda")
        epi.epi_contingency_tables(cx.ctx, ds, good, t1)
        assert torch.equal(tabs[0], t1[0])
        # a table whose class sums are not the dataset's
        t1[0, 0, 0] += 1
        mi = torch.zeros(1, dtype=torch.float64, device="cuda")
        with pytest.raises(epi.EpiError) as e:
            epi.epi_mutual_information(cx.ctx, ds, 2, t1, mi)
        assert e.value.code == epi.EPI_EINVAL and torch.isnan(mi[0])
        # order 1 has genotype tables but no contingency tables here
        with pytest.raises(epi.EpiError) as e:
            epi.epi_contingency_tables(cx.ctx, ds, good[:, :1].contiguous(), t1)
        assert e.value.code == epi.EPI_EINVAL
        # buffers the binding can see are too small, or of the wrong type, never reach the library
        with pytest.raises(epi.EpiError):
            epi.epi_contingency_tables(cx.ctx, ds, good, torch.zeros((1, 2, 8), dtype=torch.int32, device="cuda"))
        with pytest.raises(epi.EpiError):
            epi.epi_genotype_tables(cx.ctx, ds, good.long(), rows)
        with pytest.raises(epi.EpiError):
            epi.epi_mutual_information(cx.ctx, ds, 2, t1, torch.zeros(1, dtype=torch.float32, device="cuda"))
        # nothing to do
        empty = torch.zeros((0, 3), dtype=torch.int32, device="cuda")
        assert epi.epi_contingency_tables(cx.ctx, ds, empty, t1) == 0.0
    finally:
        epi.epi_unload(cx.ctx, ds)
