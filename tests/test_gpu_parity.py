"""GPU scan vs CPU oracle, through the C ABI (needs an MI355X)."""
from __future__ import annotations

import itertools
import json
import math
import os
import time

import numpy as np
import pytest

from parity import check_scores_tables, check_topk
from synth import WORKLOADS, make_case_control, make_workload, random_genotypes

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def cx():
    from paper_2201_02460_amd import epi

    with epi.Context(0) as c:
        yield c


def run_scan(cx, G, y, order, K):
    from paper_2201_02460_amd import epi

    ds = cx.load(G, y)
    try:
        return cx.scan(ds, order, K)
    finally:
        epi.epi_unload(cx.ctx, ds)


# Several 64-SNP blocks and 128-individual groups with ragged tails, every
# order, unbalanced and balanced classes.
CASES = [
    # order, M, N, n_cases, K
    (2, 3, 2, 1, 5),
    (2, 130, 257, 128, 20),
    (2, 200, 1000, 500, 10),
    (2, 65, 129, 1, 7),
    (3, 3, 5, 2, 2),
    (3, 70, 300, 100, 25),
    (3, 131, 385, 257, 40),
    (3, 66, 640, 511, 9),
    (4, 4, 40, 19, 3),
    (4, 30, 260, 90, 30),
    (4, 41, 129, 64, 17),
    (5, 5, 33, 16, 1),
    (5, 22, 200, 60, 50),
    (5, 26, 130, 65, 8),
    (6, 6, 40, 20, 1),
    (6, 14, 200, 70, 20),
    (7, 15, 129, 64, 9),
    (7, 11, 300, 150, 40),
    (8, 8, 33, 16, 1),
    (8, 13, 260, 100, 30),
    (8, 16, 129, 1, 5),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "k%d_M%d_N%d_c%d_K%d" % c)
def test_small_random_vs_oracle(cx, orc, case):
    order, M, N, n_cases, K = case
    say("case", case)
    G, y = random_genotypes(M, N, seed=M * 31 + N + order, case_fraction=n_cases / N)
    res = run_scan(cx, G, y, order, K)
    check_topk(orc, G, y, order, K, res["combos"], res["scores"], res["tables"])


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_planted_vs_oracle(cx, orc, order):
    M = {2: 150, 3: 90, 4: 34, 5: 40}[order]
    planted = tuple(range(3, 3 + 7 * order, 7))
    G, y, info = make_case_control(M, 600, 240, planted, seed=40 + order)
    say("planted", order, planted, info["h2"])
    res = run_scan(cx, G, y, order, 15)
    check_topk(orc, G, y, order, 15, res["combos"], res["scores"], res["tables"])


def test_deterministic_planted_ranks_first(cx):
    rng = np.random.default_rng(5)
    for order, planted in ((2, (10, 77)), (3, (4, 30, 61)), (4, (2, 9, 17, 25))):
        M = {2: 100, 3: 70, 4: 30}[order]
        G = rng.choice(3, size=(M, 700), p=[0.25, 0.5, 0.25]).astype(np.uint8)
        y = (sum((G[p] == 1).astype(int) for p in planted) % 2).astype(np.uint8)
        res = run_scan(cx, G, y, order, 3)
        assert tuple(res["combos"][0]) == planted


def test_more_results_than_combinations(cx, orc):
    G, y = random_genotypes(9, 90, seed=3)
    for order in (2, 3, 4, 5, 6, 7, 8):
        n = math.comb(9, order)
        res = run_scan(cx, G, y, order, n + 7)
        assert len(res["combos"]) == n
        check_topk(orc, G, y, order, n + 7, res["combos"], res["scores"], res["tables"])


def test_exact_ties_are_lexicographic(cx):
    G0, y = random_genotypes(1, 77, seed=9)
    G = np.repeat(G0, 9, axis=0)
    for order in (2, 3, 4):
        n = math.comb(9, order)
        res = run_scan(cx, G, y, order, n)
        assert [tuple(c) for c in res["combos"]] == list(itertools.combinations(range(9), order))
        assert len(set(res["scores"].tolist())) == 1


def test_invalid_inputs_are_rejected(cx):
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(5, 40, seed=1)
    bad = G.copy()
    bad[2, 7] = 3
    with pytest.raises(epi.EpiError) as e:
        cx.load(bad, y)
    assert e.value.code == epi.EPI_EINVAL
    yb = y.copy()
    yb[0] = 2
    with pytest.raises(epi.EpiError):
        cx.load(G, yb)
    with pytest.raises(epi.EpiError):
        cx.load(G, np.ones_like(y))
    ds = cx.load(G, y)
    for order, K, code in ((1, 5, epi.EPI_EINVAL), (6, 5, epi.EPI_EINVAL), (3, 0, epi.EPI_EINVAL),
                           (3, 257, epi.EPI_EUNSUPPORTED)):
        with pytest.raises(epi.EpiError) as e:
            epi.epi_scan(cx.ctx, ds, order, K)
        assert e.value.code == code
    epi.epi_unload(cx.ctx, ds)
    # an order beyond the largest supported one; order 8 keys a SNP in 8 bits (M <= 256)
    G, y = random_genotypes(300, 40, seed=2)
    ds = cx.load(G, y)
    for order, K, code in ((9, 5, epi.EPI_EUNSUPPORTED), (8, 5, epi.EPI_EUNSUPPORTED)):
        with pytest.raises(epi.EpiError) as e:
            epi.epi_scan(cx.ctx, ds, order, K)
        assert e.value.code == code
    with pytest.raises(epi.EpiError) as e:
        epi.epi_scan(cx.ctx, ds + 999, 2, 5)
    assert e.value.code == epi.EPI_ENOTFOUND
    epi.epi_unload(cx.ctx, ds)


def test_device_load_and_repack(cx, orc):
    import torch

    from paper_2201_02460_amd import epi

    G, y = random_genotypes(80, 333, seed=12, case_fraction=0.4)
    dG = torch.from_numpy(G).cuda()
    dy = torch.from_numpy(y).cuda()
    ds = epi.epi_load_genotypes_device(cx.ctx, dG, dy)
    res = cx.scan(ds, 3, 10)
    check_topk(orc, G, y, 3, 10, res["combos"], res["scores"], res["tables"])
    # new genotypes with the same class sizes, repacked asynchronously
    G2, _ = random_genotypes(80, 333, seed=13)
    y2 = np.random.default_rng(2).permutation(y)
    epi.epi_repack_device(cx.ctx, ds, torch.from_numpy(G2).cuda(), torch.from_numpy(y2).cuda())
    res2 = cx.scan(ds, 3, 10)
    check_topk(orc, G2, y2, 3, 10, res2["combos"], res2["scores"], res2["tables"])
    epi.epi_unload(cx.ctx, ds)


def test_repack_input_checks(cx, orc):
    """A repack with invalid values or other class sizes is reported by the
    results of the scans that follow it (the device checks the values while
    packing); a repack with valid input clears it.  The binding refuses
    tensors of the wrong shape, dtype or layout before any call."""
    import torch

    from paper_2201_02460_amd import epi

    G, y = random_genotypes(60, 300, seed=14, case_fraction=0.4)
    dG, dy = torch.from_numpy(G).cuda(), torch.from_numpy(y).cuda()
    ds = epi.epi_load_genotypes_device(cx.ctx, dG, dy)
    try:
        y_more = y.copy()
        y_more[np.nonzero(y == 0)[0][0]] = 1  # one more case than the dataset has
        G_bad = G.copy()
        G_bad[7, 100] = 3
        y_bad = y.copy()
        y_bad[5] = 2
        for gg, yy, what in ((G, y_more, "class sizes"), (G_bad, y, "genotype"), (G, y_bad, "phenotype")):
            say("invalid repack:", what)
            epi.epi_repack_device(cx.ctx, ds, torch.from_numpy(gg).cuda(), torch.from_numpy(yy).cuda())
            sid = epi.epi_scan(cx.ctx, ds, 3, 5)
            epi.epi_wait(cx.ctx, sid)
            with pytest.raises(epi.EpiError) as e:
                epi.epi_results(cx.ctx, sid, 5, 3)
            assert e.value.code == epi.EPI_EINVAL
            epi.epi_release(cx.ctx, sid)
        epi.epi_repack_device(cx.ctx, ds, dG, dy)
        res = cx.scan(ds, 3, 10)
        check_topk(orc, G, y, 3, 10, res["combos"], res["scores"], res["tables"])
        for bad_g, bad_y in ((dG[:, :299], dy[:299]), (dG.to(torch.int32), dy), (dG.t().contiguous().t(), dy),
                             (dG, dy.to(torch.int64)), (torch.from_numpy(G), dy)):
            with pytest.raises(epi.EpiError) as e:
                epi.epi_repack_device(cx.ctx, ds, bad_g, bad_y)
            assert e.value.code == epi.EPI_EINVAL
        with pytest.raises(epi.EpiError):
            epi.epi_load_genotypes(cx.ctx, G.astype(np.int64), y)
        with pytest.raises(epi.EpiError):
            epi.epi_load_genotypes(cx.ctx, G, y[:-1])
    finally:
        epi.epi_unload(cx.ctx, ds)


def _golden_names():
    return [n for n in WORKLOADS if os.path.exists(os.path.join(GOLDEN, n + ".json"))]


@pytest.mark.parametrize("name", _golden_names())
def test_full_size_workload_vs_stored_oracle(cx, orc, name):
    """The named workloads at full size, in the plain launch the benchmark
    times, against the oracle's full scan stored in tests/golden."""
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        gold = json.load(f)
    G, y, spec, info = make_workload(name)
    say("workload", name, spec)
    res = run_scan(cx, G, y, spec["order"], spec["top_k"])
    ref = {"combos": np.asarray(gold["combos"], np.int32), "scores": np.asarray(gold["scores"])}
    check_topk(orc, G, y, spec["order"], spec["top_k"], res["combos"], res["scores"], res["tables"], ref=ref)
    gold_tab = {tuple(c): np.asarray(t, np.int64) for c, t in zip(gold["combos"], gold["tables"])}
    for c, t in zip(res["combos"], res["tables"]):
        if tuple(c) in gold_tab:
            assert np.array_equal(t.astype(np.int64), gold_tab[tuple(c)])
    say("top-1", tuple(res["combos"][0]), float(res["scores"][0]), "planted", spec["planted"], "ms", res["ms"])


def test_batch_matches_single_scans(cx, orc):
    from paper_2201_02460_amd import epi

    specs = [(2, 140, 700, 300), (3, 75, 410, 150), (4, 28, 300, 100), (3, 120, 260, 60), (2, 33, 97, 40)]
    data, dss = [], []
    for i, (order, M, N, nc) in enumerate(specs):
        G, y = random_genotypes(M, N, seed=100 + i, case_fraction=nc / N)
        data.append((G, y))
        dss.append(cx.load(G, y))
    K = 12
    descs = [(dss[i], specs[i][0], K) for i in range(len(specs))]
    singles = [cx.scan(dss[i], specs[i][0], K) for i in range(len(specs))]
    bid = epi.epi_batch_create(cx.ctx, descs, persistent=True, use_graph=True)
    for rep in range(3):
        say("batch replay", rep)
        epi.epi_batch_run(cx.ctx, bid)
        epi.epi_batch_wait(cx.ctx, bid)
        for i, (order, M, N, nc) in enumerate(specs):
            c, s, t = epi.epi_batch_results(cx.ctx, bid, i, K, order)
            assert np.array_equal(c, singles[i]["combos"])
            assert np.array_equal(s, singles[i]["scores"])
            assert np.array_equal(t, singles[i]["tables"])
            if rep == 0:
                G, y = data[i]
                check_topk(orc, G, y, order, K, c, s, t)
    epi.epi_batch_destroy(cx.ctx, bid)
    # one-shot persistent batch through epi_scan_batch
    ids = epi.epi_scan_batch(cx.ctx, descs)
    for i, sid in enumerate(ids):
        epi.epi_wait(cx.ctx, sid)
        c, s, t = epi.epi_results(cx.ctx, sid, K, specs[i][0])
        assert np.array_equal(c, singles[i]["combos"]) and np.array_equal(s, singles[i]["scores"])
        epi.epi_release(cx.ctx, sid)
    for d in dss:
        epi.epi_unload(cx.ctx, d)


@pytest.mark.parametrize("order,M,N,nc,K", [(2, 130, 300, 100, 20), (3, 70, 257, 128, 25), (4, 30, 200, 77, 30),
                                            (5, 21, 385, 200, 12), (6, 14, 130, 40, 9), (7, 12, 96, 48, 5),
                                            (8, 13, 260, 100, 30)])
def test_segmented_matches_fused(cx, orc, order, M, N, nc, K):
    """The segmented variant (tables of a block counted first, then scored)
    gives the fused kernels' results exactly, and the oracle's."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(M, N, seed=700 + order, case_fraction=nc / N)
    ds = cx.load(G, y)
    try:
        fused = cx.scan(ds, order, K)
        epi.epi_set_prefix_block(cx.ctx, ds, order, epi.EPI_BLOCK_SEGMENTED)
        try:
            seg = cx.scan(ds, order, K)
        finally:
            epi.epi_set_prefix_block(cx.ctx, ds, order, 0)
        say("order", order, "fused variant", fused["variant"], "segmented variant", seg["variant"])
        assert seg["variant"] == 6 and fused["variant"] != 6
        assert np.array_equal(seg["combos"], fused["combos"]) and np.array_equal(seg["scores"], fused["scores"])
        assert np.array_equal(seg["tables"], fused["tables"])
        check_topk(orc, G, y, order, K, seg["combos"], seg["scores"], seg["tables"])
        with pytest.raises(epi.EpiError) as e:
            epi.epi_set_prefix_block(cx.ctx, ds, max(order, 4), 4)
        assert e.value.code == epi.EPI_EINVAL
    finally:
        epi.epi_unload(cx.ctx, ds)


def test_segmented_in_graph_batch(cx, orc):
    """Segmented scans inside a persistent graph-captured batch (their table
    buffers shared by a launch's tasks wave slot by wave slot) equal the
    fused single scans, over several replays."""
    from paper_2201_02460_amd import epi

    data = [random_genotypes(16, 300, seed=810 + i, case_fraction=0.4) for i in range(2)]
    dss = [cx.load(G, y) for G, y in data]
    try:
        K = 15
        fused = [cx.scan(ds, 5, K) for ds in dss] + [cx.scan(dss[0], 4, K)]
        for order in (4, 5):
            epi.epi_set_prefix_block(cx.ctx, dss[0], order, epi.EPI_BLOCK_SEGMENTED)
        try:
            descs = [(dss[0], 5, K), (dss[1], 5, K), (dss[0], 4, K)]
            bid = epi.epi_batch_create(cx.ctx, descs, persistent=True, use_graph=True)
            for rep in range(3):
                say("segmented batch replay", rep)
                epi.epi_batch_run(cx.ctx, bid)
                epi.epi_batch_wait(cx.ctx, bid)
                for i, (ds, order, _) in enumerate(descs):
                    c, sc, t = epi.epi_batch_results(cx.ctx, bid, i, K, order)
                    assert np.array_equal(c, fused[i]["combos"]) and np.array_equal(sc, fused[i]["scores"])
                    assert np.array_equal(t, fused[i]["tables"])
            epi.epi_batch_destroy(cx.ctx, bid)
        finally:
            for order in (4, 5):
                epi.epi_set_prefix_block(cx.ctx, dss[0], order, 0)
        check_topk(orc, data[1][0], data[1][1], 5, K, fused[1]["combos"], fused[1]["scores"], fused[1]["tables"])
    finally:
        for ds in dss:
            epi.epi_unload(cx.ctx, ds)


def test_scan_orders_one_pass(cx, orc):
    """Every order 2 .. max_order in one pass equals the separate scans; the
    order-2 scan is scored by the higher orders' pair sub-table pass."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(40, 500, seed=77, case_fraction=0.4)
    ds = cx.load(G, y)
    G2, y2 = random_genotypes(50, 300, seed=78, case_fraction=0.5)
    ds2 = cx.load(G2, y2)
    try:
        K = 25
        single = {o: cx.scan(ds, o, K) for o in range(2, 6)}
        ids = epi.epi_scan_orders(cx.ctx, ds, 5, K)
        assert len(ids) == 4
        for o, sid in zip(range(2, 6), ids):
            epi.epi_wait(cx.ctx, sid)
            c, sc, t = epi.epi_results(cx.ctx, sid, K, o)
            info = epi.epi_scan_info(cx.ctx, sid)
            say("order", o, "variant", info["variant"])
            if o == 2:
                assert info["variant"] == 7  # scored by the pair sub-table pass
            assert np.array_equal(c, single[o]["combos"]) and np.array_equal(sc, single[o]["scores"])
            assert np.array_equal(t, single[o]["tables"])
            epi.epi_release(cx.ctx, sid)
        check_topk(orc, G, y, 2, K, single[2]["combos"], single[2]["scores"], single[2]["tables"])
        # order 2 folded into an order-4 pass only, and not across datasets
        for descs, want in (([(ds, 2, K), (ds, 4, K)], 7), ([(ds2, 2, K), (ds, 3, K)], 1)):
            ids = epi.epi_scan_batch(cx.ctx, descs)
            epi.epi_wait(cx.ctx, ids[0])
            assert epi.epi_scan_info(cx.ctx, ids[0])["variant"] == want
            c, sc, t = epi.epi_results(cx.ctx, ids[0], K, 2)
            ref = single[2] if descs[0][0] == ds else cx.scan(ds2, 2, K)
            assert np.array_equal(c, ref["combos"]) and np.array_equal(sc, ref["scores"])
            for sid in ids:
                epi.epi_wait(cx.ctx, sid)
                epi.epi_release(cx.ctx, sid)
        with pytest.raises(epi.EpiError) as e:
            epi.epi_scan_orders(cx.ctx, ds, 9, K)
        assert e.value.code == epi.EPI_EUNSUPPORTED
    finally:
        epi.epi_unload(cx.ctx, ds)
        epi.epi_unload(cx.ctx, ds2)
    # up to order 8 on a small dataset
    G, y = random_genotypes(10, 260, seed=79, case_fraction=0.45)
    ds = cx.load(G, y)
    try:
        ids = epi.epi_scan_orders(cx.ctx, ds, 8, 12)
        for o, sid in zip(range(2, 9), ids):
            epi.epi_wait(cx.ctx, sid)
            c, sc, t = epi.epi_results(cx.ctx, sid, 12, o)
            epi.epi_release(cx.ctx, sid)
            check_topk(orc, G, y, o, 12, c, sc, t)
    finally:
        epi.epi_unload(cx.ctx, ds)


def test_autotune_keeps_results(cx, orc):
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(160, 700, seed=21, case_fraction=0.3)
    ds = cx.load(G, y)
    before = cx.scan(ds, 3, 20)
    choice = epi.epi_autotune(cx.ctx, ds, 3)
    assert choice in (1, 2, 4, 8, 16, 48)  # 16, 48: the matrix-core kernels
    after = cx.scan(ds, 3, 20)
    assert np.array_equal(before["combos"], after["combos"]) and np.array_equal(before["scores"], after["scores"])
    check_topk(orc, G, y, 3, 20, after["combos"], after["scores"], after["tables"])
    epi.epi_unload(cx.ctx, ds)


def test_autotune_every_order(cx, orc):
    """The tuner times every counting kernel of orders 2-5 on slices spread
    over the scan, reports ns per scored combination for each, and its
    choice (which persistent batches use too, order 2 included) keeps the
    results."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(60, 900, seed=23, case_fraction=0.4)
    ds = cx.load(G, y)
    try:
        K = 15
        plain = {o: cx.scan(ds, o, K) for o in (2, 3, 4, 5)}
        want = {2: [2, 4, 8, 16], 3: [1, 2, 4, 8, 16, 48], 4: [0, epi.EPI_BLOCK_ALL_CELLS, epi.EPI_BLOCK_SEGMENTED],
                5: [epi.EPI_BLOCK_ALL_CELLS, epi.EPI_BLOCK_SEGMENTED]}
        for o in (2, 3, 4, 5):
            choice = epi.epi_autotune(cx.ctx, ds, o)
            rep = epi.epi_autotune_report(cx.ctx, ds, o)
            say("order", o, "choice", choice, "report", rep)
            assert [b for b, _ in rep] == want[o]
            assert all(t > 0 for _, t in rep)
            assert choice == min(rep, key=lambda r: r[1])[0]
            res = cx.scan(ds, o, K)
            assert np.array_equal(res["combos"], plain[o]["combos"]) and np.array_equal(res["scores"], plain[o]["scores"])
        ids = epi.epi_scan_batch(cx.ctx, [(ds, 2, K), (ds, 3, K)])
        for o, sid in zip((2, 3), ids):
            epi.epi_wait(cx.ctx, sid)
            c, sc, t = epi.epi_results(cx.ctx, sid, K, o)
            assert np.array_equal(c, plain[o]["combos"]) and np.array_equal(t, plain[o]["tables"])
            epi.epi_release(cx.ctx, sid)
        check_topk(orc, G, y, 4, K, plain[4]["combos"], plain[4]["scores"], plain[4]["tables"])
    finally:
        for o in (2, 3, 4, 5):
            epi.epi_set_prefix_block(cx.ctx, ds, o, 0)
        epi.epi_unload(cx.ctx, ds)


@pytest.mark.parametrize("N", [9000, 17000])
def test_large_n_screening_paths(cx, orc, N):
    """Orders 2-4 where the screening table's two halves do not fit in LDS
    together (N = 9000: the first half only) and where neither does (N =
    17000: every combination takes the exact score)."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(40, N, seed=N, case_fraction=0.45)
    ds = cx.load(G, y)
    try:
        for order, K in ((2, 15), (3, 20), (4, 10)):
            say("N", N, "order", order)
            res = cx.scan(ds, order, K)
            check_topk(orc, G, y, order, K, res["combos"], res["scores"], res["tables"])
    finally:
        epi.epi_unload(cx.ctx, ds)


@pytest.mark.parametrize("N,nc", [(9000, 4000), (132000, 66000)])
def test_per_combination_paths(cx, orc, N, nc):
    """Orders 5-6 by the per-combination kernel where the n ln n table does
    not fit in LDS (N = 9000) and where class 0 exceeds 65535 individuals
    (N = 132000: the 27-cell form instead of the packed 81-cell one), fused
    and segmented."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(8, N, seed=N + 5, case_fraction=nc / N)
    ds = cx.load(G, y)
    try:
        for order, K in ((5, 12), (6, 9)):
            say("N", N, "order", order)
            res = cx.scan(ds, order, K)
            check_topk(orc, G, y, order, K, res["combos"], res["scores"], res["tables"])
            epi.epi_set_prefix_block(cx.ctx, ds, order, epi.EPI_BLOCK_SEGMENTED)
            try:
                seg = cx.scan(ds, order, K)
            finally:
                epi.epi_set_prefix_block(cx.ctx, ds, order, 0)
            assert np.array_equal(seg["combos"], res["combos"]) and np.array_equal(seg["tables"], res["tables"])
            assert np.array_equal(seg["scores"], res["scores"])
    finally:
        epi.epi_unload(cx.ctx, ds)


def test_counting_kernels_agree(cx, orc):
    """Every order-3 counting kernel (popcount prefix blocks, 4-bit float and
    8-bit integer matrix-core products) gives the same results."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(150, 1100, seed=31, case_fraction=0.35)
    ds = cx.load(G, y)
    ref = None
    for block in (1, 2, 4, 8, epi.EPI_BLOCK_MFMA_FP4, epi.EPI_BLOCK_MFMA_FP4_2J, epi.EPI_BLOCK_MFMA_I8):
        say("prefix block", block)
        epi.epi_set_prefix_block(cx.ctx, ds, 3, block)
        res = cx.scan(ds, 3, 30)
        assert res["prefix_block"] == block
        if ref is None:
            check_topk(orc, G, y, 3, 30, res["combos"], res["scores"], res["tables"])
            ref = res
        else:
            assert np.array_equal(res["combos"], ref["combos"])
            assert np.array_equal(res["scores"], ref["scores"])
            assert np.array_equal(res["tables"], ref["tables"])
    for bad in (3, 5, 128, -1):
        with pytest.raises(epi.EpiError) as e:
            epi.epi_set_prefix_block(cx.ctx, ds, 3, bad)
        assert e.value.code == epi.EPI_EINVAL
    for bad2 in (epi.EPI_BLOCK_MFMA_FP4_2J, epi.EPI_BLOCK_MFMA_I8):  # order-3 only blocks
        with pytest.raises(epi.EpiError):
            epi.epi_set_prefix_block(cx.ctx, ds, 2, bad2)
    # the choice holds for every dataset of the same size bucket: block 0
    # restores the built-in default (the 4-bit matrix-core kernel here)
    epi.epi_set_prefix_block(cx.ctx, ds, 3, 0)
    assert cx.scan(ds, 3, 30)["prefix_block"] == epi.EPI_BLOCK_MFMA_FP4
    epi.epi_unload(cx.ctx, ds)


def test_two_middle_kernel_class_size_limit(cx, orc):
    """The two-middle-SNP 4-bit kernel holds both classes of a cell in one
    float accumulator, 4 n(cases) + 2^T n(controls) with T = 2 + the bit width
    of the case count: at 2047 cases and 2047 controls a cell that holds every
    individual reaches 2^24 - 4, the largest such sum; one control more does
    not fit and the block is refused for that dataset."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(37, 4094, seed=47, case_fraction=0.5)
    y = np.zeros(4094, np.uint8)
    y[:2047] = 1
    G[[0, 5, 17, 36]] = 0  # monomorphic SNPs: cells that hold every individual
    G[9, ::3] = 2
    ds = cx.load(G, y)
    try:
        epi.epi_set_prefix_block(cx.ctx, ds, 3, epi.EPI_BLOCK_MFMA_FP4_2J)
        res = cx.scan(ds, 3, 40)
        assert res["prefix_block"] == epi.EPI_BLOCK_MFMA_FP4_2J
        check_topk(orc, G, y, 3, 40, res["combos"], res["scores"], res["tables"])
        epi.epi_set_prefix_block(cx.ctx, ds, 3, epi.EPI_BLOCK_MFMA_FP4)
        ref = cx.scan(ds, 3, 40)
        for k in ("combos", "scores", "tables"):
            assert np.array_equal(res[k], ref[k])
    finally:
        epi.epi_set_prefix_block(cx.ctx, ds, 3, 0)
        epi.epi_unload(cx.ctx, ds)
    G2 = np.concatenate([G, G[:, :1]], axis=1)
    y2 = np.concatenate([y, np.zeros(1, np.uint8)])
    ds = cx.load(G2, y2)
    try:
        with pytest.raises(epi.EpiError) as e:
            epi.epi_set_prefix_block(cx.ctx, ds, 3, epi.EPI_BLOCK_MFMA_FP4_2J)
        assert e.value.code == epi.EPI_EUNSUPPORTED
    finally:
        epi.epi_unload(cx.ctx, ds)


def test_full_size_order3_every_matrix_core_block(cx, orc):
    """The order-3 workload (M = 1000, N = 4000) on each matrix-core kernel:
    these launches run the pilot pass first (one item per wave counted into
    the histogram for a first bound), so a bound above the K-th best would
    drop results; every block must give the stored oracle top K exactly."""
    from paper_2201_02460_amd import epi

    name = "order3_M1000_N4000"
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        gold = json.load(f)
    G, y, spec, _ = make_workload(name)
    K = spec["top_k"]
    ref = {"combos": np.asarray(gold["combos"], np.int32), "scores": np.asarray(gold["scores"])}
    gold_tab = {tuple(c): np.asarray(t, np.int64) for c, t in zip(gold["combos"], gold["tables"])}
    ds = cx.load(G, y)
    first = None
    try:
        for block in (epi.EPI_BLOCK_MFMA_FP4, epi.EPI_BLOCK_MFMA_I8, epi.EPI_BLOCK_MFMA_FP4_2J):
            say("prefix block", block)
            epi.epi_set_prefix_block(cx.ctx, ds, 3, block)
            res = cx.scan(ds, 3, K)
            assert res["prefix_block"] == block
            if first is None:
                check_topk(orc, G, y, 3, K, res["combos"], res["scores"], res["tables"], ref=ref)
                for c, t in zip(res["combos"], res["tables"]):
                    if tuple(c) in gold_tab:
                        assert np.array_equal(t.astype(np.int64), gold_tab[tuple(c)])
                first = res
            else:
                for k in ("combos", "scores", "tables"):
                    assert np.array_equal(res[k], first[k])
    finally:
        epi.epi_set_prefix_block(cx.ctx, ds, 3, 0)
        epi.epi_unload(cx.ctx, ds)


@pytest.mark.parametrize("M,N,nc", [(2, 40, 17), (17, 300, 120), (33, 129, 64), (70, 1100, 700), (131, 385, 100)])
def test_order2_matrix_core_kernel(cx, orc, M, N, nc):
    """Order 2 on the matrix cores (prefix block EPI_BLOCK_MFMA_FP4 at order
    2: the order-3 products without the middle SNP's mask) against the
    oracle, on SNP counts that leave partial 16- and 32-SNP blocks and class
    sizes that leave partial 64-individual steps, and equal to the popcount
    kernel."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(M, N, seed=M + N, case_fraction=nc / N)
    ds = cx.load(G, y)
    K = min(25, M * (M - 1) // 2)
    try:
        epi.epi_set_prefix_block(cx.ctx, ds, 2, epi.EPI_BLOCK_MFMA_FP4)
        res = cx.scan(ds, 2, K)
        assert res["prefix_block"] == epi.EPI_BLOCK_MFMA_FP4
        check_topk(orc, G, y, 2, K, res["combos"], res["scores"], res["tables"])
        epi.epi_set_prefix_block(cx.ctx, ds, 2, 4)
        ref = cx.scan(ds, 2, K)
        for k in ("combos", "scores", "tables"):
            assert np.array_equal(res[k], ref[k])
    finally:
        epi.epi_set_prefix_block(cx.ctx, ds, 2, 0)
        epi.epi_unload(cx.ctx, ds)


def test_order2_pilot_pass_keeps_results(cx, orc):
    """An order-2 scan large enough for the pilot pass (at least 32 items per
    pilot item and 2K pilot items), on the popcount and the matrix-core
    kernel: the bound the pilot publishes must not drop any of the oracle's
    best K."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(720, 600, seed=71, case_fraction=0.45)
    ds = cx.load(G, y)
    K = 10
    try:
        first = None
        for block in (4, epi.EPI_BLOCK_MFMA_FP4):
            epi.epi_set_prefix_block(cx.ctx, ds, 2, block)
            res = cx.scan(ds, 2, K)
            assert res["prefix_block"] == block
            if first is None:
                check_topk(orc, G, y, 2, K, res["combos"], res["scores"], res["tables"])
                first = res
            else:
                for k in ("combos", "scores", "tables"):
                    assert np.array_equal(res[k], first[k])
    finally:
        epi.epi_set_prefix_block(cx.ctx, ds, 2, 0)
        epi.epi_unload(cx.ctx, ds)


def test_pinned_blocks_in_batches_and_server(cx, orc):
    """Every order-2 and order-3 block pinned for a dataset's size bucket is
    the kernel its scans run in a persistent batch and in served requests
    too (the launch group takes the scan's own block, the matrix-core order-2
    block included): results equal the plain scan's, which the oracle
    checks."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(150, 700, seed=83, case_fraction=0.4)
    ds = cx.load(G, y)
    K = 12
    try:
        for order, blocks in ((2, (2, 4, 8, epi.EPI_BLOCK_MFMA_FP4)), (3, (1, 8, epi.EPI_BLOCK_MFMA_FP4))):
            for block in blocks:
                say("order", order, "block", block)
                epi.epi_set_prefix_block(cx.ctx, ds, order, block)
                plain = cx.scan(ds, order, K)
                assert plain["prefix_block"] == block
                check_topk(orc, G, y, order, K, plain["combos"], plain["scores"], plain["tables"])
                bid = epi.epi_batch_create(cx.ctx, [(ds, order, K), (ds, order, K + 3)], persistent=True,
                                           use_graph=False)
                epi.epi_batch_run(cx.ctx, bid)
                epi.epi_batch_wait(cx.ctx, bid)
                c, s, t = epi.epi_batch_results(cx.ctx, bid, 0, K, order)
                epi.epi_batch_destroy(cx.ctx, bid)
                assert np.array_equal(c, plain["combos"]) and np.array_equal(s, plain["scores"])
                assert np.array_equal(t, plain["tables"])
                sid = epi.epi_server_start(cx.ctx, max_active=4)
                rid = epi.epi_server_submit(cx.ctx, sid, ds, order, K)
                while epi.epi_server_poll(cx.ctx, sid, rid) != 2:
                    time.sleep(0.001)
                c, s, t, _ = epi.epi_server_results(cx.ctx, sid, rid, K, order)
                epi.epi_server_stop(cx.ctx, sid)
                assert np.array_equal(c, plain["combos"]) and np.array_equal(s, plain["scores"])
                assert np.array_equal(t, plain["tables"])
            epi.epi_set_prefix_block(cx.ctx, ds, order, 0)
    finally:
        epi.epi_unload(cx.ctx, ds)
