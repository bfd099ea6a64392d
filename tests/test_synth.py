"""Generator properties (CPU): determinism, class sizes, HWE, no marginal effect."""
import itertools

import numpy as np

from synth import (WORKLOADS, batched_specs, hwe_probs, make_case_control, make_workload, planted_penetrance,
                   served_pool_specs)


def test_deterministic_and_sized():
    a = make_case_control(50, 300, 90, (3, 7), seed=5)
    b = make_case_control(50, 300, 90, (3, 7), seed=5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    G, y, info = a
    assert G.shape == (50, 300) and G.dtype == np.uint8 and set(np.unique(G)) <= {0, 1, 2}
    assert int(y.sum()) == 90 and y.shape == (300,)


def test_penetrance_has_no_marginal_effect():
    rng = np.random.default_rng(0)
    for k in (2, 3, 4):
        maf = rng.uniform(0.05, 0.5, k)
        f, h2 = planted_penetrance(maf, 0.1, 0.1)
        a = hwe_probs(maf)
        joint = np.ones((3,) * k)
        for t in range(k):
            shape = [1] * k
            shape[t] = 3
            joint = joint * a[t].reshape(shape)
        assert abs((joint * f).sum() - 0.1) < 1e-12
        # every proper subset of the planted SNPs has penetrance K in every cell
        for r in range(1, k):
            for sub in itertools.combinations(range(k), r):
                rest = tuple(t for t in range(k) if t not in sub)
                marg = (joint * f).sum(axis=rest) / joint.sum(axis=rest)
                assert np.allclose(marg, 0.1, atol=1e-12)
        assert 0 < h2 <= 0.1 + 1e-12 and (f >= 0).all() and (f <= 1).all()


def test_planted_maf_and_strength():
    # planted SNPs draw their MAF from [0.3, 0.5], which keeps the achieved
    # heritability of every named workload well above the cap that rare
    # planted alleles impose
    for name in WORKLOADS:
        G, y, spec, info = make_workload(name)
        pm = info["maf"][list(spec["planted"])]
        assert np.all((pm >= 0.3) & (pm <= 0.5)), name
        assert info["h2"] >= 0.02, (name, info["h2"])
        assert abs(info["h2"] - planted_penetrance(pm, 0.1, 0.1)[1]) < 1e-15


def test_hwe_frequencies():
    G, y, info = make_case_control(20, 20000, 10000, (), seed=3)
    a = hwe_probs(info["maf"])
    freq = np.stack([(G == g).mean(axis=1) for g in range(3)], axis=1)
    assert np.abs(freq - a).max() < 0.02


def test_specs():
    for spec in WORKLOADS.values():
        assert len(spec["planted"]) == spec["order"]
    specs = batched_specs()
    assert len(specs) == 64 and {s["order"] for s in specs} <= {2, 3}
    assert all(100 <= s["M"] <= 2000 and 500 <= s["N"] <= 8000 for s in specs)
    pool = served_pool_specs()
    assert all((4 in d["orders"]) == (d["M"] <= 200) or d["M"] <= 200 for d in pool)
