"""The allocation-free scan (epi_scan_noalloc) through the C ABI, against the
plain scan of the same dataset (needs an MI355X).

Two calls in a row share the device's scratch array, the second on a smaller
input; neither may allocate (the context's allocator and torch's device
memory are unchanged across them), and both must return the plain scan's
results exactly.
"""
from __future__ import annotations

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


def out_buffers(torch, order, K):
    return (torch.full((K, order), -7, dtype=torch.int32, device="cuda"),
            torch.full((K,), -1.0, dtype=torch.float32, device="cuda"),
            torch.full((K, 2, 3**order), -5, dtype=torch.int32, device="cuda"),
            torch.full((1,), -9, dtype=torch.int32, device="cuda"))


def read(bufs):
    c, s, t, n = (b.cpu().numpy() for b in bufs)
    k = int(n[0])
    return k, c[:k], s[:k], t[:k].view(np.uint32)


def same(got, ref):
    k, c, s, t = got
    return (k == len(ref["combos"]) and np.array_equal(c, ref["combos"]) and np.array_equal(s, ref["scores"])
            and np.array_equal(t, ref["tables"]))


def test_noalloc_equals_plain_scan(cx, orc):
    import torch

    from paper_2201_02460_amd import epi

    stream = torch.cuda.Stream()
    G1, y1 = random_genotypes(300, 1500, seed=61, case_fraction=0.4)
    G2, y2 = random_genotypes(90, 400, seed=62, case_fraction=0.3)
    ds1, ds2 = cx.load(G1, y1), cx.load(G2, y2)
    try:
        K1, K2 = 40, 25
        b1, b2 = out_buffers(torch, 3, K1), out_buffers(torch, 3, K2)
        torch.cuda.synchronize()
        used0 = epi.epi_memory(cx.ctx)[0]
        torch0 = torch.cuda.memory_allocated()
        # first call: shapes the context has not cached (descriptor tables
        # built into the scratch); second: a smaller input on the same array
        say("noalloc order 3, M 300, N 1500")
        epi.epi_scan_noalloc(cx.ctx, ds1, 3, K1, *b1, stream=stream)
        say("noalloc order 3, M 90, N 400")
        epi.epi_scan_noalloc(cx.ctx, ds2, 3, K2, *b2, stream=stream)
        stream.synchronize()
        assert epi.epi_memory(cx.ctx)[0] == used0, "the library's allocator was used"
        assert torch.cuda.memory_allocated() == torch0
        r1, r2 = cx.scan(ds1, 3, K1), cx.scan(ds2, 3, K2)
        assert same(read(b1), r1) and same(read(b2), r2)
        k, c, s, t = read(b2)
        check_topk(orc, G2, y2, 3, K2, c, s, t)
        # other orders, now with the context's cached descriptor tables; the
        # same scratch again, larger then smaller
        for ds, order, K in ((ds1, 2, 30), (ds2, 4, 20), (ds2, 2, 12), (ds2, 5, 9)):
            say("noalloc order", order, "dataset", ds)
            b = out_buffers(torch, order, K)
            torch.cuda.synchronize()
            used0 = epi.epi_memory(cx.ctx)[0]
            epi.epi_scan_noalloc(cx.ctx, ds, order, K, *b, stream=stream)
            stream.synchronize()
            assert epi.epi_memory(cx.ctx)[0] == used0
            assert same(read(b), cx.scan(ds, order, K)), f"order {order}"
        # the tables are optional
        b = out_buffers(torch, 3, K2)
        epi.epi_scan_noalloc(cx.ctx, ds2, 3, K2, b[0], b[1], None, b[3], stream=stream)
        stream.synchronize()
        k, c, s, _ = read(b)
        assert k == K2 and np.array_equal(c, r2["combos"]) and np.array_equal(s, r2["scores"])
        assert (b[2].cpu().numpy() == -5).all()
    finally:
        epi.epi_unload(cx.ctx, ds1)
        epi.epi_unload(cx.ctx, ds2)


def test_noalloc_limits(cx):
    import torch

    from paper_2201_02460_amd import epi

    # order 3 on 3000 SNPs: the pair sub-table alone (144 MB) exceeds the array
    G, y = random_genotypes(3000, 70, seed=63, case_fraction=0.5)
    ds = cx.load(G, y)
    try:
        b = out_buffers(torch, 3, 10)
        used0 = epi.epi_memory(cx.ctx)[0]
        with pytest.raises(epi.EpiError) as e:
            epi.epi_scan_noalloc(cx.ctx, ds, 3, 10, *b)
        assert e.value.code == epi.EPI_EUNSUPPORTED
        say("refused:", e.value)
        assert epi.epi_memory(cx.ctx)[0] == used0
        assert (b[3].cpu().numpy() == -9).all()  # nothing was written
        # order 2 on the same dataset fits
        epi.epi_scan_noalloc(cx.ctx, ds, 2, 10, *out_buffers(torch, 2, 10))
        with pytest.raises(epi.EpiError) as e:
            epi.epi_scan_noalloc(cx.ctx, ds, 1, 10, *out_buffers(torch, 1, 10))
        assert e.value.code == epi.EPI_EINVAL
    finally:
        torch.cuda.synchronize()
        epi.epi_unload(cx.ctx, ds)
