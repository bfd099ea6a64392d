"""The batched and served workloads at their stated sizes (Section 2.4: the
best K of every scan), through the C ABI (needs an MI355X).

* 64 uneven scans of orders 2-3 (M ~ U[100, 2000], N ~ U[500, 8000], case
  fraction ~ U[0.2, 0.5]) as one persistent graph-captured launch, replayed,
  against the same 64 scans as back-to-back plain launches: all K results of
  every scan identical (combinations, float scores, tables), and every
  returned table and score recounted by the oracle.
* The first 100 requests of the serving stream (orders 2-4 over a pool of 32
  resident datasets, M in [50, 1500], N in [500, 16000]) submitted at once to
  the continuous-batching server, against the same requests as plain scans:
  all K results identical, each recounted by the oracle.

The oracle's own best-K of these scans would take days of CPU time (4.8e13
combination x individual steps for the batch); that every combination of a
scan is scored, each with its table, is what tests/test_gpu_digest.py shows
for the same kernels.
"""
from __future__ import annotations

import time

import numpy as np
import pytest

from parity import check_order, check_scores_tables
from synth import batched_specs, make_case_control, served_pool_specs, served_requests

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def cx():
    from paper_2201_02460_amd import epi

    with epi.Context(0) as c:
        yield c


def recount(orc, G, y, combos, scores, tables):
    """Every returned table bit for bit and every score within 1e-5 relative
    of the oracle, in best-first order."""
    o_scores = check_scores_tables(orc, G, y, combos, scores, tables)
    check_order(combos, scores, o_scores, tables)
    for c in combos:
        assert all(c[t] < c[t + 1] for t in range(len(c) - 1))
    assert len({tuple(c) for c in combos}) == len(combos)


def test_batched_64_scans_full_size(cx, orc):
    from paper_2201_02460_amd import epi

    specs = batched_specs(64)
    data, dss = [], []
    for s in specs:
        G, y, _ = make_case_control(s["M"], s["N"], s["n_cases"], s["planted"], s["seed"])
        data.append((G, y))
        dss.append(cx.load(G, y))
    try:
        descs = [(dss[i], s["order"], s["top_k"]) for i, s in enumerate(specs)]
        out = {}
        for name, persistent, graph in (("batched", True, True), ("back_to_back", False, False)):
            bid = epi.epi_batch_create(cx.ctx, descs, persistent=persistent, use_graph=graph)
            reps = []
            for rep in range(2):
                t0 = time.perf_counter()
                epi.epi_batch_run(cx.ctx, bid)
                epi.epi_batch_wait(cx.ctx, bid)
                say(name, "run", rep, f"{time.perf_counter() - t0:.3f}s")
                reps.append([epi.epi_batch_results(cx.ctx, bid, i, s["top_k"], s["order"])
                             for i, s in enumerate(specs)])
            epi.epi_batch_destroy(cx.ctx, bid)
            for a, b in zip(reps[0], reps[1]):  # replays agree
                assert all(np.array_equal(u, v) for u, v in zip(a, b))
            out[name] = reps[0]
        for i, s in enumerate(specs):
            a, b = out["batched"][i], out["back_to_back"][i]
            assert len(a[0]) == s["top_k"]
            assert all(np.array_equal(u, v) for u, v in zip(a, b)), f"scan {i} differs"
            recount(orc, data[i][0], data[i][1], *a)
        say("64 scans: all K identical batched and back to back; oracle recount of",
            sum(s["top_k"] for s in specs), "tables")
    finally:
        for d in dss:
            epi.epi_unload(cx.ctx, d)


def test_served_burst_full_size(cx, orc):
    from paper_2201_02460_amd import epi

    pool = served_pool_specs(32)
    data, dss = [], []
    for s in pool:
        G, y, _ = make_case_control(s["M"], s["N"], s["n_cases"], s["planted"], s["seed"])
        data.append((G, y))
        dss.append(cx.load(G, y))
    K = 100
    reqs, _ = served_requests(pool, 100)
    try:
        sid = epi.epi_server_start(cx.ctx, max_active=64)
        ids = [(epi.epi_server_submit(cx.ctx, sid, dss[d], o, K), d, o) for d, o in reqs]
        served = []
        t0 = time.perf_counter()
        for rid, d, o in ids:
            while epi.epi_server_poll(cx.ctx, sid, rid) != 2:
                assert time.perf_counter() - t0 < 240, f"request {rid} did not finish"
                time.sleep(0.001)
            served.append(epi.epi_server_results(cx.ctx, sid, rid, K, o)[:3])
        stats = epi.epi_server_stats(cx.ctx, sid)
        epi.epi_server_stop(cx.ctx, sid)
        say("served", len(reqs), "requests:", stats)
        assert stats["peak_active"] > 1
        for (rid, d, o), got in zip(ids, served):
            alone = cx.scan(dss[d], o, K)
            assert all(np.array_equal(u, alone[k]) for u, k in zip(got, ("combos", "scores", "tables"))), \
                f"request on dataset {d} order {o} differs from the plain scan"
            recount(orc, data[d][0], data[d][1], *got)
    finally:
        for d in dss:
            epi.epi_unload(cx.ctx, d)
