"""Continuous-batching server through the C ABI (needs an MI355X).

Each request's result must equal the plain scan of the same dataset, order
and K exactly (same combinations, float scores and tables), whatever else
shared its launch rounds; a sample is also checked against the oracle.
"""
from __future__ import annotations

import math
import threading
import time

import numpy as np
import pytest

from parity import check_topk
from synth import random_genotypes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def cx():
    from paper_2201_02460_amd import epi

    with epi.Context(0) as c:
        yield c


def _datasets(cx):
    shapes = [(90, 700, 0.3), (40, 1500, 0.5), (150, 300, 0.2), (25, 2600, 0.4), (70, 129, 0.5)]
    out = []
    for i, (M, N, f) in enumerate(shapes):
        G, y = random_genotypes(M, N, seed=300 + i, case_fraction=f)
        out.append((cx.load(G, y), G, y))
    return out


def _wait(epi, cx, sid, rid, timeout=120.0):
    t0 = time.time()
    while epi.epi_server_poll(cx.ctx, sid, rid) != 2:
        assert time.time() - t0 < timeout, f"request {rid} did not finish"
        time.sleep(0.002)


@pytest.mark.parametrize("depth", [0, 1, 2])
def test_served_equals_alone(cx, orc, depth):
    """Same results with one round in flight, two, or the adaptive choice."""
    from paper_2201_02460_amd import epi

    say("rounds in flight", depth)
    data = _datasets(cx)
    reqs = [(0, 3, 20), (1, 2, 15), (2, 3, 40), (3, 4, 12), (4, 2, 9), (0, 2, 30), (1, 4, 7), (2, 2, 50),
            (3, 3, 25), (4, 3, 11), (4, 5, 6), (3, 5, 8)]
    alone = {}
    for di, order, K in reqs:
        ds = data[di][0]
        alone[(di, order, K)] = cx.scan(ds, order, K)
    sid = epi.epi_server_start(cx.ctx, max_active=4, rounds_in_flight=depth)
    ids = []

    def submitter():
        for n, (di, order, K) in enumerate(reqs):
            ids.append((epi.epi_server_submit(cx.ctx, sid, data[di][0], order, K), (di, order, K)))
            time.sleep(0.003 * (n % 3))  # staggered arrivals while rounds run

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    for rid, key in ids:
        _wait(epi, cx, sid, rid)
        di, order, K = key
        c, s, t, lat = epi.epi_server_results(cx.ctx, sid, rid, K, order)
        a = alone[key]
        assert np.array_equal(c, a["combos"]) and np.array_equal(s, a["scores"]) and np.array_equal(t, a["tables"])
        assert lat > 0
    stats = epi.epi_server_stats(cx.ctx, sid)
    say("server stats", stats)
    assert stats["requests_done"] == len(reqs) and stats["peak_active"] <= 4
    # every combination of every request counted once
    want = sum(math.comb(data[di][1].shape[0], order) * data[di][1].shape[1] for di, order, _ in reqs)
    assert stats["combo_samples"] == want
    # orders above the served maximum are refused at submission (plain scans take them)
    with pytest.raises(epi.EpiError) as e:
        epi.epi_server_submit(cx.ctx, sid, data[4][0], epi.EPI_SERVE_MAX_ORDER + 1, 5)
    assert e.value.code == epi.EPI_EUNSUPPORTED
    epi.epi_server_stop(cx.ctx, sid)
    # a depth outside 0..2 is refused
    for bad in (-1, 3):
        with pytest.raises(epi.EpiError) as e:
            epi.epi_server_start(cx.ctx, max_active=4, rounds_in_flight=bad)
        assert e.value.code == epi.EPI_EINVAL
    # one served result against the oracle as well
    di, order, K = reqs[2]
    a = alone[reqs[2]]
    check_topk(orc, data[di][1], data[di][2], order, K, a["combos"], a["scores"], a["tables"])
    for d in data:
        epi.epi_unload(cx.ctx, d[0])


def test_admission_by_memory_budget(cx):
    from paper_2201_02460_amd import epi

    data = _datasets(cx)
    # room for about one order-3 request's buffers at a time
    sid = epi.epi_server_start(cx.ctx, max_active=8, request_budget=1_200_000)
    ids = [(epi.epi_server_submit(cx.ctx, sid, data[i % 4][0], 3, 10), i % 4) for i in range(8)]
    for rid, di in ids:
        _wait(epi, cx, sid, rid)
        c, s, t, _ = epi.epi_server_results(cx.ctx, sid, rid, 10, 3)
        a = cx.scan(data[di][0], 3, 10)
        assert np.array_equal(c, a["combos"]) and np.array_equal(s, a["scores"])
    stats = epi.epi_server_stats(cx.ctx, sid)
    say("budgeted server stats", stats)
    assert stats["peak_request_bytes"] <= 1_200_000
    epi.epi_server_stop(cx.ctx, sid)
    with pytest.raises(epi.EpiError):
        epi.epi_server_submit(cx.ctx, sid, data[0][0], 2, 5)
    for d in data:
        epi.epi_unload(cx.ctx, d[0])


def test_unload_refused_while_requests_use_dataset(cx, orc):
    """A dataset named by a queued or running request cannot be unloaded; the
    requests still finish with the plain scans' results, and the dataset can
    be unloaded once they are done.  Other datasets unload meanwhile."""
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(150, 300, seed=330, case_fraction=0.4)
    ds = cx.load(G, y)
    G2, y2 = random_genotypes(30, 200, seed=331, case_fraction=0.5)
    other = cx.load(G2, y2)
    reqs = [(4, 10), (3, 20), (2, 15), (3, 7)]
    alone = {r: cx.scan(ds, r[0], r[1]) for r in reqs}
    sid = epi.epi_server_start(cx.ctx, max_active=1)
    ids = [(epi.epi_server_submit(cx.ctx, sid, ds, o, K), (o, K)) for o, K in reqs]
    with pytest.raises(epi.EpiError) as e:
        epi.epi_unload(cx.ctx, ds)
    assert e.value.code == epi.EPI_EINVAL
    say("unload refused:", e.value)
    epi.epi_unload(cx.ctx, other)
    for rid, (o, K) in ids:
        _wait(epi, cx, sid, rid)
        c, s, t, _ = epi.epi_server_results(cx.ctx, sid, rid, K, o)
        a = alone[(o, K)]
        assert np.array_equal(c, a["combos"]) and np.array_equal(s, a["scores"]) and np.array_equal(t, a["tables"])
    epi.epi_server_stop(cx.ctx, sid)
    check_topk(orc, G, y, 3, 20, alone[(3, 20)]["combos"], alone[(3, 20)]["scores"], alone[(3, 20)]["tables"])
    epi.epi_unload(cx.ctx, ds)
    with pytest.raises(epi.EpiError) as e:
        cx.scan(ds, 2, 5)
    assert e.value.code == epi.EPI_ENOTFOUND
