"""Benchmark of the exhaustive epistasis scan on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-batched] [--no-served] [--cpu-seconds S]

A step is one pass of the whole hot path over one synthetic dataset that is
already resident in HBM (uint8 genotypes + phenotype as torch tensors):
device packing into genotype masks, enumeration, contingency tables, mutual
information, best-K selection, result tables and their copy to the host.

Prints ONE JSON line.  ``value`` is tera combos x individuals per second of
the plain single-scan path on the named workload; ``roofline`` reports the
main counting kernel against the integer-VALU peak (HIP events on the scan's
stream); ``cpu_baseline`` is the CPU oracle timed on a bounded slice of the
same workload; ``batched`` compares one persistent, graph-captured launch of
64 uneven scans (kernels picked by the autotuner per order and size bucket)
with 64 back-to-back plain launches, all K results of every scan compared;
``served`` runs the continuous-batching server on a burst of requests at once
against back-to-back plain scans (capacity, all K results compared), then on
Poisson arrivals at the stated rate and near the measured capacity;
``pcie_inclusive_value`` is the same step with the genotypes handed over from
host memory; ``orders`` times the other named workloads (orders 2, 4, 5).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tera combos×samples/s at order k, batched vs plain, counts bit-exact vs oracle"
UNIT = "tera combos×samples/s"
# Integer VALU peak of MI355X: 256 CUs x 4 SIMD x 16 lanes per clock x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Dense 4-bit-float matrix-core peak of MI355X (published), TFLOP/s.
MFMA_FP4_PEAK_TFLOPS = 10.1e3
# Dense 8-bit integer matrix-core peak of MI355X (published), TOP/s.
MFMA_I8_PEAK_TOPS = 5.0e3
BLOCK_MFMA_FP4 = 16
BLOCK_MFMA_I8 = 32
BLOCK_MFMA_FP4_2J = 48
MFMA_KERNELS = {
    BLOCK_MFMA_FP4: ("scan_persistent<0,16,0> (order-3 reduced cells as fp4 0/1 matrix products)", "scan_mfma"),
    BLOCK_MFMA_FP4_2J: ("scan_persistent<0,48,0> (fp4 0/1 matrix products, two middle SNPs per item, both classes "
                        "in one accumulator)", "scan_mfma2"),
}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2201_02460_amd", "csrc", "kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ops_per_unit(order):
    """Algorithmic integer ops per combination x individual of the counting
    kernels: 2^order directly counted cells (all genotypes in {0,1}), one
    three-input AND and one popcount-accumulate per cell per 32 individuals."""
    return 2.0 * 2**order / 32.0


def mfma_flops_per_unit(order):
    """Algorithmic matrix-core work per combination x individual of the
    matrix-core kernel: one multiply-add (2 flops) per counted cell."""
    return 2.0 * 2**order


def ops_per_unit_3k(order):
    """Same for counting every one of the 3^order cells (the paper's fused
    last-level AND + popcount over all cells)."""
    return 2.0 * 3**order / 32.0


def kernel_hash():
    """Hash of the kernel source with comments and blank lines removed, so a
    comment edit does not invalidate counters taken on the same code."""
    code = []
    for line in open(KERNEL_SOURCE).read().splitlines():
        line = line.split("//", 1)[0].rstrip()
        if line:
            code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()[:16]


def load_traffic(kernel_tag, workload):
    """HBM bytes per launch from the committed counter summary of this kernel
    and workload, or None if there is none or the kernel code has changed."""
    try:
        doc = json.load(open(os.path.join(PROFILES, f"traffic_{kernel_tag}_{workload}.json")))
    except (OSError, ValueError):
        return None
    if doc.get("kernel_sha") != kernel_hash():
        return None
    return doc.get("hbm_bytes_per_launch")


def plain_bench(epi, torch, spec, G, y, steps, warmup, block=None, extra=None):
    """Timed steps of repack + scan + results on one resident dataset; the
    counting kernel is the autotuner's choice unless `block` pins one.  With
    `extra` (a dict), the device packing alone is timed after the steps
    (events on the stream it runs on) into extra["pack_ms"]."""
    dG = torch.from_numpy(G).cuda()
    dy = torch.from_numpy(y).cuda()
    stream = torch.cuda.current_stream()
    ctx = epi.epi_create(0)
    ds = epi.epi_load_genotypes_device(ctx, dG, dy, stream)
    if block is None:
        tuned = epi.epi_autotune(ctx, ds, spec["order"])
    else:
        epi.epi_set_prefix_block(ctx, ds, spec["order"], block)
        tuned = block
    order, K = spec["order"], spec["top_k"]
    mains, alls = [], []
    res = None

    def step():
        epi.epi_repack_device(ctx, ds, dG, dy, stream)
        sid = epi.epi_scan(ctx, ds, order, K, stream)
        epi.epi_wait(ctx, sid)
        r = epi.epi_results(ctx, sid, K, order)
        ms = epi.epi_scan_timing(ctx, sid)
        info = epi.epi_scan_info(ctx, sid)
        epi.epi_release(ctx, sid)
        return r, ms, info

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res, ms, info = step()
        mains.append(ms[2])
        alls.append(ms[0])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if extra is not None:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            epi.epi_repack_device(ctx, ds, dG, dy, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        extra["pack_ms"] = e0.elapsed_time(e1) / reps
    epi.epi_unload(ctx, ds)
    epi.epi_destroy(ctx)
    return dt, mains, alls, res, info, tuned


def host_cores():
    """Host cores for the CPU baseline: every core this process may run on,
    within the per-GPU CPU share the host states in OMP_NUM_THREADS (a
    one-GPU share of a larger machine)."""
    affinity = len(os.sched_getaffinity(0))
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return (min(affinity, share) if share > 0 else affinity), affinity, share or None


def cpu_baseline(spec, G, y, seconds):
    """The oracle as it stands, on a bounded rank range of the workload."""
    import oracle

    o = oracle.default()
    order, N = spec["order"], spec["N"]
    threads, affinity, share = host_cores()
    total = o.binomial(spec["M"], order)
    # a probe of about half a second sizes the sample; a sample that still
    # ran short of half the requested time is sized again from its own rate
    n = min(total, max(1000, int(4e9 / N)))
    for _ in range(3):
        t0 = time.perf_counter()
        r = o.scan(G, y, order, spec["top_k"], 0, n, nthreads=threads, tables=False)
        dt = time.perf_counter() - t0
        want = min(total, max(n, int(n * seconds / max(dt, 1e-3))))
        if dt >= 0.5 * seconds or n == total:
            break
        n = want
    return {
        "value": n * N / dt / 1e12,
        "unit": UNIT,
        "cores": r["threads"],
        "nproc": os.cpu_count(),
        "affinity_cores": affinity,
        "host_share_cores": share,
        "kind": "oracle",
        "sample": f"first {n} of {o.binomial(spec['M'], order)} combinations (lexicographic) of the same "
                  f"workload, all {N} individuals, {dt:.1f} s",
    }


def pcie_bench(epi, spec, G, y, steps):
    """Same steps with the genotypes handed over from host memory: load
    (host-to-device copy + packing) + scan + results + unload."""
    order, K = spec["order"], spec["top_k"]
    ctx = epi.epi_create(0)
    times = []
    for i in range(steps + 1):
        t0 = time.perf_counter()
        ds = epi.epi_load_genotypes(ctx, G, y)
        sid = epi.epi_scan(ctx, ds, order, K)
        epi.epi_wait(ctx, sid)
        epi.epi_results(ctx, sid, K, order)
        epi.epi_release(ctx, sid)
        epi.epi_unload(ctx, ds)
        if i:
            times.append(time.perf_counter() - t0)
    epi.epi_destroy(ctx)
    return math.comb(spec["M"], order) * spec["N"] * len(times) / sum(times) / 1e12


def orders_bench(epi, torch, names, steps):
    """Plain scans of the other named workloads (one per order), for the
    per-order rate and roofline fraction of their counting kernels."""
    from synth import make_workload

    out = {}
    ctx = epi.epi_create(0)
    for name in names:
        G, y, spec, _ = make_workload(name)
        order, K = spec["order"], spec["top_k"]
        work = math.comb(spec["M"], order) * spec["N"]
        ds = epi.epi_load_genotypes(ctx, G, y)
        epi.epi_autotune(ctx, ds, order)
        walls, mains = [], []
        for i in range(steps + 2):
            t0 = time.perf_counter()
            sid = epi.epi_scan(ctx, ds, order, K)
            epi.epi_wait(ctx, sid)
            epi.epi_results(ctx, sid, K, order)
            ms = epi.epi_scan_timing(ctx, sid)
            info = epi.epi_scan_info(ctx, sid)
            epi.epi_release(ctx, sid)
            if i >= 2:
                walls.append(time.perf_counter() - t0)
                mains.append(ms[2])
        epi.epi_unload(ctx, ds)
        kms = sorted(mains)[len(mains) // 2]
        # reduced-cell variants count 2^k cells, the generic one all 3^k;
        # order 2 may run on the matrix cores (2 x 2^2 flops per unit)
        mfma2 = order == 2 and info["prefix_block"] == BLOCK_MFMA_FP4
        opu = ops_per_unit(order) if info["variant"] in (1, 2, 5) else ops_per_unit_3k(order)
        out[name] = {"value": work * len(walls) / sum(walls) / 1e12, "kernel_ms": kms,
                     "kernel_value": work / (kms * 1e-3) / 1e12, "variant": info["variant"],
                     "prefix_block": info["prefix_block"],
                     "ops_per_unit": mfma_flops_per_unit(2) if mfma2 else opu,
                     "bound": "mfma" if mfma2 else "alu",
                     "frac": (work * mfma_flops_per_unit(2) / (kms * 1e-3) / 1e12 / MFMA_FP4_PEAK_TFLOPS if mfma2
                              else work * opu / (kms * 1e-3) / 1e12 / VALU_PEAK_TOPS),
                     "frac_3k_cells": work * ops_per_unit_3k(order) / (kms * 1e-3) / 1e12 / VALU_PEAK_TOPS}
        log(f"{name}: kernel {kms:.3f} ms, {out[name]['kernel_value']:.2f} T, frac {out[name]['frac']:.3f}")
    epi.epi_destroy(ctx)
    return out


def pairs_bench(epi, steps, M=4000, N=4000, K=100):
    """Order 2 at a size where the counting matters (M = 4000 SNPs, N = 4000
    individuals, the workloads' generator with one planted pair): the
    popcount prefix blocks against the pair counts as fp4 0/1 matrix
    products, kernel time and identical results."""
    import numpy as np
    from synth import make_case_control

    G, y, _ = make_case_control(M, N, N // 2, [17, 113], seed=5)
    work = math.comb(M, 2) * N
    ctx = epi.epi_create(0)
    ds = epi.epi_load_genotypes(ctx, G, y)
    out, ref = {"workload": f"order 2, M={M}, N={N}, top-{K}"}, None
    for block in (2, 4, 8, BLOCK_MFMA_FP4):
        epi.epi_set_prefix_block(ctx, ds, 2, block)
        mains, res = [], None
        for i in range(steps + 1):
            sid = epi.epi_scan(ctx, ds, 2, K)
            epi.epi_wait(ctx, sid)
            res = epi.epi_results(ctx, sid, K, 2)
            ms = epi.epi_scan_timing(ctx, sid)
            epi.epi_release(ctx, sid)
            if i:
                mains.append(ms[2])
        kms = sorted(mains)[len(mains) // 2]
        ref = res if ref is None else ref
        mf = block == BLOCK_MFMA_FP4
        opu = mfma_flops_per_unit(2) if mf else ops_per_unit(2)
        peak = MFMA_FP4_PEAK_TFLOPS if mf else VALU_PEAK_TOPS
        out[f"block_{block}"] = {"kernel_ms": round(kms, 4), "kernel_value": round(work / (kms * 1e-3) / 1e12, 3),
                                 "bound": "mfma" if mf else "alu", "frac": round(work * opu / (kms * 1e-3) / 1e12 / peak, 4),
                                 "identical_results": bool(all(np.array_equal(u, v) for u, v in zip(res, ref)))}
        log(f"pairs M={M}: block {block} kernel {kms:.3f} ms")
    epi.epi_unload(ctx, ds)
    epi.epi_destroy(ctx)
    return out


def segmented_bench(epi, names, steps):
    """The segmented variant (a wave's 64 tables counted into a buffer, then
    scored: the paper's Algorithm 2) against the fused kernel of each named
    workload: median kernel times and whether the results are identical."""
    import numpy as np

    from synth import make_workload

    out = {}
    ctx = epi.epi_create(0)
    for name in names:
        G, y, spec, _ = make_workload(name)
        order, K = spec["order"], spec["top_k"]
        work = math.comb(spec["M"], order) * spec["N"]
        ds = epi.epi_load_genotypes(ctx, G, y)
        row = {}
        for form in ("fused", "segmented"):
            epi.epi_set_prefix_block(ctx, ds, order, epi.EPI_BLOCK_SEGMENTED if form == "segmented" else 0)
            mains, res = [], None
            for i in range(steps + 1):
                sid = epi.epi_scan(ctx, ds, order, K)
                epi.epi_wait(ctx, sid)
                r = epi.epi_results(ctx, sid, K, order)
                ms = epi.epi_scan_timing(ctx, sid)
                variant = epi.epi_scan_info(ctx, sid)["variant"]
                epi.epi_release(ctx, sid)
                if i:
                    mains.append(ms[2])
                res = r
            kms = sorted(mains)[len(mains) // 2]
            row[form] = {"kernel_ms": kms, "kernel_value": work / (kms * 1e-3) / 1e12, "variant": variant,
                         "result": res}
        epi.epi_set_prefix_block(ctx, ds, order, 0)
        epi.epi_unload(ctx, ds)
        a, b = row["fused"].pop("result"), row["segmented"].pop("result")
        row["identical_results"] = bool(all(np.array_equal(u, v) for u, v in zip(a, b)))
        row["segmented_over_fused_time"] = row["segmented"]["kernel_ms"] / row["fused"]["kernel_ms"]
        out[name] = row
        log(f"{name}: fused {row['fused']['kernel_ms']:.3f} ms, segmented {row['segmented']['kernel_ms']:.3f} ms, "
            f"identical {row['identical_results']}")
    epi.epi_destroy(ctx)
    return out


def orders_pass_bench(epi, names, steps):
    """Every order 2 .. k of a named workload in one pass (epi_scan_orders)
    against the same scans one after another: end-to-end wall time (launch
    through results on the host), median of steps runs."""
    import numpy as np

    from synth import make_workload

    out = {}
    ctx = epi.epi_create(0)
    for name in names:
        G, y, spec, _ = make_workload(name)
        kmax, K = spec["order"], spec["top_k"]
        orders = list(range(2, kmax + 1))
        work = sum(math.comb(spec["M"], o) for o in orders) * spec["N"]
        ds = epi.epi_load_genotypes(ctx, G, y)
        t_one, t_sep, res_one, res_sep = [], [], None, None
        for i in range(steps + 1):
            t0 = time.perf_counter()
            ids = epi.epi_scan_orders(ctx, ds, kmax, K)
            res_one = []
            for o, sid in zip(orders, ids):
                epi.epi_wait(ctx, sid)
                res_one.append(epi.epi_results(ctx, sid, K, o))
                epi.epi_release(ctx, sid)
            t1 = time.perf_counter()
            res_sep = []
            for o in orders:
                sid = epi.epi_scan(ctx, ds, o, K)
                epi.epi_wait(ctx, sid)
                res_sep.append(epi.epi_results(ctx, sid, K, o))
                epi.epi_release(ctx, sid)
            t2 = time.perf_counter()
            if i:
                t_one.append(t1 - t0)
                t_sep.append(t2 - t1)
        epi.epi_unload(ctx, ds)
        one, sep = sorted(t_one)[len(t_one) // 2], sorted(t_sep)[len(t_sep) // 2]
        same = all(np.array_equal(u, v) for a, b in zip(res_one, res_sep) for u, v in zip(a, b))
        out[name] = {"orders": orders, "one_pass_ms": one * 1e3, "separate_ms": sep * 1e3,
                     "one_pass_value": work / one / 1e12, "separate_value": work / sep / 1e12,
                     "speedup": sep / one, "identical_results": bool(same)}
        log(f"{name} orders {orders}: one pass {one * 1e3:.3f} ms, separate {sep * 1e3:.3f} ms, identical {same}")
    epi.epi_destroy(ctx)
    return out


def functions_bench(epi, torch, reps=3, out_cap=1 << 30, table_cap=8 << 30):
    """The three steps as separate passes over a list of combinations, timed
    per genotype-table row (both classes), per contingency-table cell (both
    classes) and per MI cell: order 3 against the number of individuals, and
    orders 2, 4 and 8 at 2048 individuals (the paper's per-function
    figures).  Each pass covers the first n lexicographic combinations of M
    SNPs (1500 for order 2, 200 for order 3, else 64), at most 2^20, n bounded
    so that the genotype rows stay under out_cap bytes and the tables under
    table_cap bytes; the MI pass reads the tables repeated up to that many."""
    import itertools

    import numpy as np

    from synth import random_genotypes

    ctx = epi.epi_create(0)
    out = {"vs_individuals_order3": {}, "vs_order_N2048": {}}
    points = [(3, n_ind, "vs_individuals_order3") for n_ind in (128, 256, 512, 1024, 2048, 4096, 8192)]
    points += [(k, 2048, "vs_order_N2048") for k in (2, 4, 8)]
    for order, N, key in points:
        M = {2: 1500, 3: 200}.get(order, 64)
        G, y = random_genotypes(M, N, seed=4000 + N + order, case_fraction=0.5)
        ds = epi.epi_load_genotypes(ctx, G, y)
        n_case = int(y.sum())
        W = 4 * ((n_case + 127) // 128) + 4 * ((N - n_case + 127) // 128)
        P = 3**order
        n_gt = max(1, min(math.comb(M, order), out_cap // (P * W * 4), 1 << 20))
        n_ct = max(1, min(math.comb(M, order), table_cap // (P * 8), 1 << 20))
        n_mi = max(1, min(table_cap // (P * 8), 1 << 20))
        combos = np.asarray(list(itertools.islice(itertools.combinations(range(M), order), max(n_gt, n_ct))),
                            np.int32)
        dc = torch.from_numpy(combos).cuda()
        rows = torch.empty((n_gt, P, W), dtype=torch.int32, device="cuda")
        tabs = torch.empty((n_ct, 2, P), dtype=torch.int32, device="cuda")
        mi = torch.empty(n_mi, dtype=torch.float64, device="cuda")
        t_gt, t_ct, t_mi = [], [], []
        for _ in range(reps + 1):
            t_gt.append(epi.epi_genotype_tables(ctx, ds, dc[:n_gt], rows))
            t_ct.append(epi.epi_contingency_tables(ctx, ds, dc[:n_ct], tabs))
            if n_mi > n_ct:
                big = tabs.repeat(((n_mi + n_ct - 1) // n_ct, 1, 1))[:n_mi].contiguous()
                t_mi.append(epi.epi_mutual_information(ctx, ds, order, big, mi))
                del big
            else:
                t_mi.append(epi.epi_mutual_information(ctx, ds, order, tabs, mi))
        med = lambda v: sorted(v[1:])[len(v[1:]) // 2]  # noqa: E731
        gt_ms, ct_ms, mi_ms = med(t_gt), med(t_ct), med(t_mi)
        row = {"order": order, "individuals": N, "gt_combinations": n_gt, "ct_combinations": n_ct, "mi_tables": n_mi,
               "gt_ns_per_row": gt_ms * 1e6 / (n_gt * P), "gt_write_GBps": n_gt * P * W * 4 / (gt_ms * 1e-3) / 1e9,
               "ct_ns_per_cell": ct_ms * 1e6 / (n_ct * P), "mi_ns_per_cell": mi_ms * 1e6 / (n_mi * P),
               "mi_read_GBps": n_mi * P * 8 / (mi_ms * 1e-3) / 1e9}
        out[key][f"k{order}_N{N}"] = row
        log(f"functions k={order} N={N}: GT {row['gt_ns_per_row']:.4f} ns/row ({row['gt_write_GBps']:.0f} GB/s), "
            f"CT {row['ct_ns_per_cell']:.4f} ns/cell, MI {row['mi_ns_per_cell']:.4f} ns/cell "
            f"({row['mi_read_GBps']:.0f} GB/s)")
        del rows, tabs, mi, dc
        epi.epi_unload(ctx, ds)
    epi.epi_destroy(ctx)
    return out


def batched_bench(epi, torch, n_scans, reps):
    """One persistent graph-captured launch of n uneven scans vs n back-to-back plain launches."""
    import numpy as np

    from synth import batched_specs, make_case_control

    specs = batched_specs(n_scans)
    ctx = epi.epi_create(0)
    dss, work = [], 0
    t0 = time.perf_counter()
    for s in specs:
        G, y, _ = make_case_control(s["M"], s["N"], s["n_cases"], s["planted"], s["seed"])
        dss.append(epi.epi_load_genotypes(ctx, G, y))
        work += math.comb(s["M"], s["order"]) * s["N"]
    log(f"batched: {n_scans} datasets generated and loaded in {time.perf_counter() - t0:.1f}s, "
        f"{work:.3e} combos x individuals")
    descs = [(dss[i], specs[i]["order"], specs[i]["top_k"]) for i in range(n_scans)]
    # the tuner picks the counting kernel of every (order, size bucket) of
    # the mix, on one dataset of that bucket; the batch then uses the picks
    tuned, seen = [], set()
    for i, s in enumerate(specs):
        n_case = s["n_cases"]
        words = 4 * ((n_case + 127) // 128) + 4 * ((s["N"] - n_case + 127) // 128)
        key = (s["order"], max(0, (words - 1).bit_length()), max(0, (s["M"] - 1).bit_length()))
        if key in seen:
            continue
        seen.add(key)
        choice = epi.epi_autotune(ctx, dss[i], s["order"])
        rep = epi.epi_autotune_report(ctx, dss[i], s["order"])
        tuned.append({"order": s["order"], "words_bucket": key[1], "snp_bucket": key[2],
                      "tuned_on": {"M": s["M"], "N": s["N"]},
                      "choice": choice, "ns_per_combination": {str(b): round(t, 6) for b, t in rep}})
        log(f"batched tune order {s['order']} buckets {key[1]}/{key[2]} (M={s['M']}, N={s['N']}): pick {choice}, "
            + ", ".join(f"{b}: {t:.5f} ns" for b, t in rep))
    out = {}
    for name, persistent, graph in (("batched", True, True), ("back_to_back", False, False)):
        bid = epi.epi_batch_create(ctx, descs, persistent=persistent, use_graph=graph)
        epi.epi_batch_run(ctx, bid)
        epi.epi_batch_wait(ctx, bid)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            epi.epi_batch_run(ctx, bid)
            epi.epi_batch_wait(ctx, bid)
            times.append(time.perf_counter() - t0)
        res = [epi.epi_batch_results(ctx, bid, i, specs[i]["top_k"], specs[i]["order"]) for i in range(n_scans)]
        out[name] = {"seconds": min(times), "value": work / min(times) / 1e12, "results": res,
                     "top1": [tuple(int(v) for v in c[0]) for c, _, _ in res]}
        epi.epi_batch_destroy(ctx, bid)
        log(f"{name}: {min(times) * 1e3:.1f} ms -> {out[name]['value']:.2f} T")
    same = all(np.array_equal(u, v) for a, b in zip(out["batched"]["results"], out["back_to_back"]["results"])
               for u, v in zip(a, b))
    planted_hits = sum(1 for s, c in zip(specs, out["batched"]["top1"]) if tuple(s["planted"]) == c)
    for d in dss:
        epi.epi_unload(ctx, d)
    epi.epi_destroy(ctx)
    return {
        "config": {"workload": f"{n_scans} scans, order 2-3, M~U[100,2000], N~U[500,8000], cases U[0.2,0.5]",
                   "combos_x_samples": work},
        "value": out["batched"]["value"],
        "back_to_back_value": out["back_to_back"]["value"],
        "speedup": out["batched"]["value"] / out["back_to_back"]["value"],
        "seconds": out["batched"]["seconds"],
        "back_to_back_seconds": out["back_to_back"]["seconds"],
        "identical_results": bool(same),
        "planted_top1": planted_hits,
        "autotuned": tuned,
    }


def served_pool(epi, ctx):
    """Resident dataset pool of the serving workload (loaded once)."""
    from synth import make_case_control, served_pool_specs

    pool = served_pool_specs(32)
    t0 = time.perf_counter()
    dss = []
    for s in pool:
        G, y, _ = make_case_control(s["M"], s["N"], s["n_cases"], s["planted"], s["seed"])
        dss.append(epi.epi_load_genotypes(ctx, G, y))
    log(f"served: pool of {len(pool)} datasets loaded in {time.perf_counter() - t0:.1f}s")
    return pool, dss


def served_capacity(epi, ctx, pool, dss, cap, K=100, depth=0, reps=3):
    """The same requests submitted at once to a fresh server, against the same
    requests as back-to-back plain scans (scan, wait, results): aggregate
    rates (median of ``reps`` interleaved repetitions of each), and whether
    every request's K results (combinations, scores, tables) are the plain
    scan's in every repetition."""
    import numpy as np

    work = sum(math.comb(pool[d]["M"], o) * pool[d]["N"] for d, o in cap)
    burst, b2b, same, rounds, peak = [], [], True, 0, 0
    for _ in range(reps):
        sid = epi.epi_server_start(ctx, max_active=64, rounds_in_flight=depth)
        t0 = time.perf_counter()
        ids = [(epi.epi_server_submit(ctx, sid, dss[d], o, K), o) for d, o in cap]
        served = []
        for rid, o in ids:
            while epi.epi_server_poll(ctx, sid, rid) != 2:
                time.sleep(0.0005)
            served.append(epi.epi_server_results(ctx, sid, rid, K, o)[:3])
        burst.append(time.perf_counter() - t0)
        stats = epi.epi_server_stats(ctx, sid)
        rounds, peak = stats["rounds"], stats["peak_active"]
        epi.epi_server_stop(ctx, sid)
        t0 = time.perf_counter()
        plain = []
        for d, o in cap:
            q = epi.epi_scan(ctx, dss[d], o, K)
            epi.epi_wait(ctx, q)
            plain.append(epi.epi_results(ctx, q, K, o))
            epi.epi_release(ctx, q)
        b2b.append(time.perf_counter() - t0)
        same = same and all(np.array_equal(u, v) for a, b in zip(served, plain) for u, v in zip(a, b))
    burst_s, b2b_s = float(np.median(burst)), float(np.median(b2b))
    log(f"served capacity: {len(cap)} requests at once {burst_s:.3f}s ({rounds} rounds) "
        f"vs back-to-back plain {b2b_s:.3f}s (medians of {reps}), identical results {same}")
    return {"requests": len(cap), "combos_x_samples": int(work), "value": work / burst_s / 1e12,
            "back_to_back_value": work / b2b_s / 1e12, "speedup": b2b_s / burst_s, "rounds": rounds,
            "peak_active": peak, "repetitions": reps, "identical_results": bool(same)}


def served_leg(epi, ctx, pool, dss, reqs, gaps, K, depth=0):
    """Submit the requests at their Poisson arrival times to a fresh server
    and collect each one's latency (submission to results ready)."""
    import threading

    import numpy as np

    work = [math.comb(pool[d]["M"], o) * pool[d]["N"] for d, o in reqs]
    sid = epi.epi_server_start(ctx, max_active=64, rounds_in_flight=depth)
    pending, lat, done_at = {}, [], []
    lock = threading.Lock()
    start = time.perf_counter()

    def submit():
        t = start
        for (d, o), g in zip(reqs, gaps):
            t += g
            dt = t - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            rid = epi.epi_server_submit(ctx, sid, dss[d], o, K)
            with lock:
                pending[rid] = o

    th = threading.Thread(target=submit)
    th.start()
    finished, last_log = 0, start
    while finished < len(reqs):
        with lock:
            items = list(pending.items())
        for rid, o in items:
            if epi.epi_server_poll(ctx, sid, rid) == 2:
                _, _, _, ms = epi.epi_server_results(ctx, sid, rid, K, o, tables=False)
                lat.append(ms)
                done_at.append(time.perf_counter())
                with lock:
                    del pending[rid]
                finished += 1
        now = time.perf_counter()
        if now - last_log > 20:
            log(f"  served: {finished} of {len(reqs)} requests done after {now - start:.0f}s")
            last_log = now
        time.sleep(0.0005)
    th.join()
    wall = max(done_at) - start
    stats = epi.epi_server_stats(ctx, sid)
    epi.epi_server_stop(ctx, sid)
    lat = np.sort(np.asarray(lat))
    arrivals = float(np.sum(gaps))
    return {
        "requests": len(reqs),
        "rate_per_s": len(reqs) / arrivals,
        "value": sum(work) / wall / 1e12,
        "offered_T": sum(work) / arrivals / 1e12,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "wall_s": wall,
        "rounds": stats["rounds"],
        "peak_active": stats["peak_active"],
    }


def served_bench(epi, torch, n_requests, rate, burst, load_frac=0.8, seed=7):
    """The continuous-batching server on a resident dataset pool: capacity
    (a burst of requests at once, results compared with plain scans), then
    Poisson arrivals at the stated rate and at load_frac of the capacity
    measured on the same request sequence submitted at once (the order-4
    share of a sample sets its rate), p50/p99 latency from submission to
    results ready after a warm-up."""
    from synth import served_requests

    ctx = epi.epi_create(0)
    pool, dss = served_pool(epi, ctx)
    K = 100
    # warm-up: a short burst of every order, not counted
    warm, _ = served_requests(pool, 24, seed=seed + 100)
    served_capacity(epi, ctx, pool, dss, warm, K, reps=1)
    cap_reqs, _ = served_requests(pool, burst, seed=seed + 1)
    capacity = served_capacity(epi, ctx, pool, dss, cap_reqs, K)
    reqs, gaps = served_requests(pool, n_requests, seed=seed, rate=rate)
    mean_work = sum(math.comb(pool[d]["M"], o) * pool[d]["N"] for d, o in reqs) / len(reqs)
    log(f"served: {n_requests} requests at {rate}/s")
    stated = served_leg(epi, ctx, pool, dss, reqs, gaps, K)
    # the request sequence does not depend on the rate (only the gaps do)
    reqs2, _ = served_requests(pool, n_requests, seed=seed + 2)
    log(f"served: the {n_requests} requests of the near-capacity leg at once")
    mix_cap = served_capacity(epi, ctx, pool, dss, reqs2, K, reps=1)
    mean_work2 = mix_cap["combos_x_samples"] / len(reqs2)
    near_rate = load_frac * mix_cap["value"] * 1e12 / mean_work2
    reqs2, gaps2 = served_requests(pool, n_requests, seed=seed + 2, rate=near_rate)
    log(f"served: {n_requests} requests at {near_rate:.1f}/s ({load_frac:.0%} of their capacity)")
    near = served_leg(epi, ctx, pool, dss, reqs2, gaps2, K)
    for d in dss:
        epi.epi_unload(ctx, d)
    epi.epi_destroy(ctx)
    return {
        "config": {"workload": f"{n_requests} Poisson requests per leg after a warm-up, orders 2-4 (order 4 on "
                               f"M<=200), M in [50,1500], N in [500,16000], pool of {len(pool)} resident datasets, "
                               "top-100",
                   "mean_combos_x_samples_per_request": mean_work},
        "value": stated["value"],
        "p50_ms": stated["p50_ms"],
        "p99_ms": stated["p99_ms"],
        "offered_T": stated["offered_T"],
        "peak_active": stated["peak_active"],
        "stated_rate": stated,
        "near_capacity": near,
        "near_capacity_mix_at_once": mix_cap,
        "capacity": capacity,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="order3_M1000_N4000")
    ap.add_argument("--block", type=int, default=None,
                    help="pin the counting kernel of the main workload (a block of epi_set_prefix_block) "
                         "instead of running the autotuner")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--batched-scans", type=int, default=64)
    ap.add_argument("--batched-reps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--served-requests", type=int, default=2000, help="requests per Poisson leg")
    ap.add_argument("--served-rate", type=float, default=20.0)
    ap.add_argument("--served-burst", type=int, default=100,
                    help="requests of the served capacity comparison (all submitted at once)")
    ap.add_argument("--no-orders", action="store_true")
    ap.add_argument("--no-pairs", action="store_true")
    ap.add_argument("--no-segmented", action="store_true", help="skip the segmented-vs-fused comparison")
    ap.add_argument("--no-functions", action="store_true", help="skip the per-step (GT, CT, MI) timings")
    ap.add_argument("--no-orders-pass", action="store_true", help="skip the all-orders-in-one-pass comparison")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison with the other counting kernels")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-copy-mib", type=int, default=0,
                    help="also run an elementwise kernel over this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the scan is built and measured for a single MI355X; "
              "multi-GPU sharding is a design note, not a built path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch

    from paper_2201_02460_amd import epi
    from synth import make_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    G, y, spec, info = make_workload(args.workload)
    order, M, N = spec["order"], spec["M"], spec["N"]
    n_combos = math.comb(M, order)
    log(f"workload {args.workload}: C({M},{order}) = {n_combos} combinations x {N} individuals")

    if args.profile_copy_mib:
        # a plain elementwise kernel that reads and writes exactly this many
        # bytes: the reference for scaling the HBM byte counters
        a = torch.zeros(args.profile_copy_mib << 20, dtype=torch.uint8, device="cuda")
        for _ in range(3):
            b = a + 1
        torch.cuda.synchronize()
        del b

    extra = {}
    dt, mains, alls, res, sinfo, tuned = plain_bench(epi, torch, spec, G, y, args.steps, args.warmup, block=args.block,
                                                     extra=extra)
    combos, scores, tables = res
    value = n_combos * N * args.steps / dt / 1e12
    ms_main = sum(mains) / len(mains)
    ms_scan = sum(alls) / len(alls)
    work = n_combos * N
    mfma = sinfo["prefix_block"] in MFMA_KERNELS
    if mfma:
        kname, ktag = MFMA_KERNELS[sinfo["prefix_block"]]
        roofline = {
            "bound": "mfma",
            "achieved": round(work * mfma_flops_per_unit(order) / (ms_main * 1e-3) / 1e12, 3),
            "peak": MFMA_FP4_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "kernel": kname,
            "timed": "pilot pass + main launch (scan_pilot, then the kernel)",
            "flops_per_unit": mfma_flops_per_unit(order),
            "traffic": load_traffic(ktag, args.workload),
        }
    else:
        roofline = {
            "bound": "alu",
            "achieved": round(work * ops_per_unit(order) / (ms_main * 1e-3) / 1e12, 3),
            "peak": round(VALU_PEAK_TOPS, 3),
            "unit": "TOP/s",
            "kernel": "scan_persistent (reduced-cell popcount variant)",
            "ops_per_unit": ops_per_unit(order),
            "traffic": load_traffic("scan_popcount", args.workload),
        }
    roofline["frac"] = round(roofline["achieved"] / roofline["peak"], 4)
    roofline["kernel_ms"] = round(ms_main, 4)
    roofline["frac_valu_3k_cells"] = round(work * ops_per_unit_3k(order) / (ms_main * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4)
    planted_rank = next((i + 1 for i, c in enumerate(combos.tolist()) if tuple(c) == tuple(spec["planted"])), None)
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "order": order, "M": M, "N": N, "n_cases": spec["n_cases"],
                   "top_k": spec["top_k"], "n_combinations": n_combos, "parallelism": "single GPU",
                   "variant": sinfo["variant"], "prefix_block": sinfo["prefix_block"], "autotuned": tuned},
        "roofline": roofline,
        "scan_ms": round(ms_scan, 4),
        "pack_ms": round(extra["pack_ms"], 4),
        "top1": {"combo": [int(v) for v in combos[0]], "mi": float(scores[0]), "planted": list(spec["planted"]),
                 "planted_rank": planted_rank, "achieved_h2": info["h2"]},
    }
    if order == 3 and not args.no_compare:
        # the same step with the other counting kernels pinned: popcount
        # (prefix block 8), the 8-bit integer matrix-core products and the
        # 4-bit ones the main line did not take
        legs = [("popcount_kernel", 8, "alu", ops_per_unit(order), VALU_PEAK_TOPS, "TOP/s", "scan_popcount"),
                ("mfma_int8_kernel", BLOCK_MFMA_I8, "mfma", mfma_flops_per_unit(order), MFMA_I8_PEAK_TOPS, "TOP/s",
                 "scan_mfma_i8")]
        for blk, tag_name in ((BLOCK_MFMA_FP4, "mfma_fp4_kernel"), (BLOCK_MFMA_FP4_2J, "mfma_fp4_two_middle_kernel")):
            if blk != sinfo["prefix_block"]:
                legs.append((tag_name, blk, "mfma", mfma_flops_per_unit(order), MFMA_FP4_PEAK_TFLOPS, "TFLOP/s",
                             MFMA_KERNELS[blk][1]))
        for name, block, bound, opu, peak, unit, tag in legs:
            try:
                pdt, pm, _, pres, _, _ = plain_bench(epi, torch, spec, G, y, max(3, args.steps // 4), 2, block=block)
            except epi.EpiError as e:  # a kernel this dataset cannot run (class sizes)
                out[name] = {"skipped": str(e)}
                continue
            pk = sum(pm) / len(pm)
            achieved = work * opu / (pk * 1e-3) / 1e12
            out[name] = {
                "value": round(work * len(pm) / pdt / 1e12, 4), "kernel_ms": round(pk, 4), "bound": bound,
                "achieved": round(achieved, 3), "peak": round(peak, 3), "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": load_traffic(tag, args.workload),
                "identical_results": bool((pres[0] == combos).all() and (pres[1] == scores).all()),
            }
    out["pcie_inclusive_value"] = round(pcie_bench(epi, spec, G, y, 5), 4)
    if not args.no_orders:
        others = [n for n in ("order2_M200_N1000", "order4_M200_N2000", "order5_M60_N2000", "order8_M23_N2048")
                  if n != args.workload]
        out["orders"] = orders_bench(epi, torch, others, 5)
    if not args.no_pairs:
        out["pairs"] = pairs_bench(epi, 5)
    if not args.no_orders_pass:
        out["orders_one_pass"] = orders_pass_bench(
            epi, [args.workload, "order4_M200_N2000", "order5_M60_N2000"], 5)
    if not args.no_functions:
        out["functions"] = functions_bench(epi, torch)
    if not args.no_segmented:
        out["segmented"] = segmented_bench(
            epi, ["order2_M200_N1000", args.workload, "order4_M200_N2000", "order5_M60_N2000", "order8_M23_N2048"], 3)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, G, y, args.cpu_seconds)
    if not args.no_batched:
        out["batched"] = batched_bench(epi, torch, args.batched_scans, args.batched_reps)
    if not args.no_served:
        out["served"] = served_bench(epi, torch, args.served_requests, args.served_rate, args.served_burst)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
