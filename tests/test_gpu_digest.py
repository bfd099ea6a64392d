"""Every combination scored exactly once, each with its table (Algorithm 1,
Section 2.2), on every counting kernel: the checking build of a scan counts
the combinations it scores and sums a hash of each with its table; the
count must be C(M, k) and the digest the oracle's (needs an MI355X).

The oracle computes the same digest by walking the combinations in
lexicographic order and counting each table one individual at a time; the
full-size values are stored in tests/golden/digest_<workload>.json by
tests/golden/make_golden.py --digest.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from synth import WORKLOADS, make_workload, random_genotypes

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def cx():
    from paper_2201_02460_amd import epi

    with epi.Context(0) as c:
        yield c


def kernels_of(order):
    """Every counting kernel of an order, as the block that pins it."""
    from paper_2201_02460_amd import epi

    if order == 2:
        return [2, 4, 8, epi.EPI_BLOCK_MFMA_FP4, epi.EPI_BLOCK_SEGMENTED]
    if order == 3:
        return [1, 2, 4, 8, epi.EPI_BLOCK_MFMA_FP4, epi.EPI_BLOCK_MFMA_FP4_2J, epi.EPI_BLOCK_MFMA_I8,
                epi.EPI_BLOCK_SEGMENTED]
    if order == 4:
        return [0, epi.EPI_BLOCK_ALL_CELLS, epi.EPI_BLOCK_SEGMENTED]  # 0: reduced cells
    return [0, epi.EPI_BLOCK_SEGMENTED]  # 0: all cells


def checked_scan(cx, ds, order, K, block):
    """Scan with the kernel `block` pins, in the checking build; returns the
    digest pair, the results and the kernel variant."""
    from paper_2201_02460_amd import epi

    epi.epi_set_prefix_block(cx.ctx, ds, order, block)
    try:
        sid = epi.epi_scan_check(cx.ctx, ds, order, K)
        try:
            epi.epi_wait(cx.ctx, sid)
            dig = epi.epi_scan_digest(cx.ctx, sid)
            res = epi.epi_results(cx.ctx, sid, K, order)
            info = epi.epi_scan_info(cx.ctx, sid)
        finally:
            epi.epi_release(cx.ctx, sid)
        plain = cx.scan(ds, order, K)
    finally:
        epi.epi_set_prefix_block(cx.ctx, ds, order, 0)
    # the checking build returns the plain scan's results
    for a, b in zip(res, (plain["combos"], plain["scores"], plain["tables"])):
        assert np.array_equal(a, b)
    return dig, info


SMALL = [  # order, M, N, n_cases
    (2, 131, 300, 120), (2, 66, 129, 1),
    (3, 70, 257, 128), (3, 97, 200, 61),
    (4, 37, 260, 90), (4, 30, 129, 64),
    (5, 22, 200, 60), (6, 14, 130, 40), (7, 12, 96, 48), (8, 13, 260, 100),
]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "k%d_M%d_N%d_c%d" % c)
def test_small_digest_every_kernel(cx, orc, case):
    from paper_2201_02460_amd import epi

    order, M, N, nc = case
    G, y = random_genotypes(M, N, seed=900 + M + order, case_fraction=nc / N)
    want = orc.digest(G, y, order)
    assert want[0] == math.comb(M, order)
    ds = cx.load(G, y)
    try:
        for block in kernels_of(order):
            say("case", case, "block", block)
            got, info = checked_scan(cx, ds, order, 10, block)
            assert got == want, f"block {block} (variant {info['variant']}): {got} != oracle {want}"
    finally:
        epi.epi_unload(cx.ctx, ds)


def _digest_names():
    return [n for n in WORKLOADS if os.path.exists(os.path.join(GOLDEN, "digest_" + n + ".json"))]


@pytest.mark.parametrize("name", _digest_names())
def test_full_size_digest_every_kernel(cx, name):
    """The named workloads at full size: every counting kernel of the order
    scores C(M, k) combinations with the oracle's digest."""
    from paper_2201_02460_amd import epi

    with open(os.path.join(GOLDEN, "digest_" + name + ".json")) as f:
        gold = json.load(f)
    G, y, spec, _ = make_workload(name)
    order = spec["order"]
    want = (gold["n_combinations"], gold["digest"])
    assert want[0] == math.comb(spec["M"], order)
    ds = cx.load(G, y)
    try:
        for block in kernels_of(order):
            say("workload", name, "block", block)
            got, info = checked_scan(cx, ds, order, spec["top_k"], block)
            say("  variant", info["variant"], "prefix block", info["prefix_block"], "count", got[0])
            assert got == want, f"block {block} (variant {info['variant']}): {got} != oracle {want}"
    finally:
        epi.epi_unload(cx.ctx, ds)


def test_digest_needs_a_checking_scan(cx):
    from paper_2201_02460_amd import epi

    G, y = random_genotypes(20, 100, seed=3)
    ds = cx.load(G, y)
    try:
        sid = epi.epi_scan(cx.ctx, ds, 3, 5)
        epi.epi_wait(cx.ctx, sid)
        with pytest.raises(epi.EpiError) as e:
            epi.epi_scan_digest(cx.ctx, sid)
        assert e.value.code == epi.EPI_EINVAL
        epi.epi_release(cx.ctx, sid)
        with pytest.raises(epi.EpiError) as e:
            epi.epi_set_prefix_block(cx.ctx, ds, 3, epi.EPI_BLOCK_ALL_CELLS)
        assert e.value.code == epi.EPI_EINVAL
    finally:
        epi.epi_unload(cx.ctx, ds)
