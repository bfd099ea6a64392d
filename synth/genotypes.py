"""Seeded synthetic genotype/phenotype generator.

Recipe (all draws from ``numpy.random.default_rng(seed)``, PCG64):

1. Per-SNP minor-allele frequency ``maf ~ U(0.05, 0.5)``.
2. Genotype ``g`` = minor-allele count in {0, 1, 2}, drawn under Hardy-Weinberg
   proportions ``((1-p)^2, 2p(1-p), p^2)``.  Value ``g`` is genotype-table row
   ``g`` (homozygous dominant, heterozygous, homozygous recessive), the three
   rows of a single-SNP genotype table in Section 2.1 of the paper.
3. One planted interaction of the scan's order with no marginal effect:
   penetrance ``f(g_S) = K + sigma * prod_t u_t[g_t]`` with
   ``u_t = (sqrt(w), -1/sqrt(w), sqrt(w))`` and ``w = a1 / (a0 + a2)`` under
   SNP t's HWE probabilities ``a``.  Each ``u_t`` has mean 0 and variance 1, so
   every proper subset of the planted SNPs has marginal penetrance exactly K
   (an "XOR-style" heterozygote-parity interaction), and the heritability is
   ``sigma^2 / (K (1 - K))``.  ``sigma`` is capped so that ``f`` stays in
   [0, 1]; the achieved heritability is returned.
4. Case-control ascertainment: candidate individuals' planted genotypes and
   Bernoulli(f) phenotypes are drawn in batches and accepted until exactly
   ``n_cases`` cases and ``N - n_cases`` controls are filled; the null SNPs of
   the accepted individuals are then drawn from HWE and the sample order is
   shuffled.

The paper gives only the sizes of its inputs (numbers of SNPs, individuals and
the interaction order, Section 4); these generators stand in for its data.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "hwe_probs",
    "planted_penetrance",
    "make_case_control",
    "random_genotypes",
    "WORKLOADS",
    "make_workload",
    "batched_specs",
    "served_pool_specs",
    "served_requests",
]


def hwe_probs(maf):
    """Hardy-Weinberg genotype probabilities, shape ``maf.shape + (3,)``."""
    p = np.asarray(maf, dtype=np.float64)
    return np.stack([(1.0 - p) ** 2, 2.0 * p * (1.0 - p), p**2], axis=-1)


def planted_penetrance(maf_planted, prevalence=0.1, h2=0.1):
    """Penetrance over the 3^k genotype cells of the planted SNPs.

    Returns ``(f, achieved_h2)``; ``f`` has shape ``(3,)*k`` with the first SNP
    on the first axis.
    """
    a = hwe_probs(maf_planted)  # (k, 3)
    k = a.shape[0]
    w = a[:, 1] / (a[:, 0] + a[:, 2])
    u = np.stack([np.sqrt(w), -1.0 / np.sqrt(w), np.sqrt(w)], axis=-1)  # (k, 3)
    prod = np.ones((3,) * k)
    for t in range(k):
        shape = [1] * k
        shape[t] = 3
        prod = prod * u[t].reshape(shape)
    K = float(prevalence)
    sigma = np.sqrt(h2 * K * (1.0 - K))
    pos = prod[prod > 0]
    neg = prod[prod < 0]
    cap = np.inf
    if pos.size:
        cap = min(cap, (1.0 - K) / pos.max())
    if neg.size:
        cap = min(cap, K / (-neg.min()))
    sigma = min(sigma, cap)
    f = np.clip(K + sigma * prod, 0.0, 1.0)
    return f, float(sigma**2 / (K * (1.0 - K)))


def _draw_genotypes(rng, probs, n):
    """Draw ``n`` genotypes per row of ``probs`` (rows, 3) -> uint8 (rows, n)."""
    u = rng.random((probs.shape[0], n))
    c0 = probs[:, 0:1]
    c1 = c0 + probs[:, 1:2]
    return ((u >= c0).astype(np.uint8) + (u >= c1).astype(np.uint8)).astype(np.uint8)


def make_case_control(M, N, n_cases, planted, seed, prevalence=0.1, h2=0.1, planted_maf=(0.3, 0.5)):
    """Genotypes ``G`` (uint8, M x N, SNP-major) and phenotype ``y`` (uint8, 1 = case).

    ``planted`` is a sequence of distinct SNP indices (may be empty for null
    data).  The planted SNPs draw their MAF from ``planted_maf`` (the other
    SNPs from U(0.05, 0.5)): a rare planted allele makes the penetrance
    table's extreme cells cap the interaction's effect far below ``h2``.
    Returns ``(G, y, info)`` with ``info`` holding the MAFs, the planted set
    and the achieved heritability.
    """
    M, N, n_cases = int(M), int(N), int(n_cases)
    if not (0 < n_cases < N):
        raise ValueError("need at least one case and one control")
    planted = [int(s) for s in planted]
    if len(set(planted)) != len(planted) or any(not 0 <= s < M for s in planted):
        raise ValueError("planted SNPs must be distinct indices in [0, M)")
    rng = np.random.default_rng(seed)
    maf = rng.uniform(0.05, 0.5, M)
    if planted:
        maf[planted] = rng.uniform(planted_maf[0], planted_maf[1], len(planted))
    probs = hwe_probs(maf)
    n_ctrl = N - n_cases
    info = {"maf": maf, "planted": tuple(planted), "h2": 0.0, "seed": seed}
    if planted:
        f, h2_ach = planted_penetrance(maf[planted], prevalence, h2)
        info["h2"] = h2_ach
        k = len(planted)
        cases, ctrls = [], []
        got_case = got_ctrl = 0
        batch = max(4096, 4 * int(N / max(prevalence, 1e-3)))
        while got_case < n_cases or got_ctrl < n_ctrl:
            gs = _draw_genotypes(rng, probs[planted], batch)  # (k, batch)
            cell = np.ravel_multi_index(tuple(gs[t] for t in range(k)), (3,) * k)
            pheno = rng.random(batch) < f.reshape(-1)[cell]
            if got_case < n_cases:
                take = gs[:, pheno][:, : n_cases - got_case]
                cases.append(take)
                got_case += take.shape[1]
            if got_ctrl < n_ctrl:
                take = gs[:, ~pheno][:, : n_ctrl - got_ctrl]
                ctrls.append(take)
                got_ctrl += take.shape[1]
        planted_g = np.concatenate(cases + ctrls, axis=1)  # cases first
    y = np.concatenate([np.ones(n_cases, np.uint8), np.zeros(n_ctrl, np.uint8)])
    G = _draw_genotypes(rng, probs, N)
    if planted:
        G[planted, :] = planted_g
    perm = rng.permutation(N)
    G = np.ascontiguousarray(G[:, perm])
    y = np.ascontiguousarray(y[perm])
    return G, y, info


def random_genotypes(M, N, seed, case_fraction=0.5, probs=None):
    """Unstructured test input: i.i.d. genotypes and a random class split.

    Every class keeps at least one sample.  ``probs`` (3,) overrides the
    genotype distribution (defaults to uniform over {0, 1, 2}).
    """
    rng = np.random.default_rng(seed)
    p = np.full(3, 1.0 / 3.0) if probs is None else np.asarray(probs, np.float64)
    G = rng.choice(3, size=(M, N), p=p).astype(np.uint8)
    n_cases = int(round(case_fraction * N))
    n_cases = min(max(n_cases, 1), N - 1)
    y = np.zeros(N, np.uint8)
    y[rng.choice(N, n_cases, replace=False)] = 1
    return G, y


# Named single-scan workloads: the sizes of the paper-shaped configurations.
WORKLOADS = {
    "order2_M200_N1000": dict(order=2, M=200, N=1000, n_cases=500, planted=(17, 113), seed=0, top_k=10),
    "order3_M1000_N4000": dict(order=3, M=1000, N=4000, n_cases=2000, planted=(17, 113, 617), seed=0, top_k=100),
    "order4_M200_N2000": dict(order=4, M=200, N=2000, n_cases=600, planted=(17, 59, 113, 171), seed=0, top_k=100),
    "order5_M60_N2000": dict(order=5, M=60, N=2000, n_cases=600, planted=(5, 17, 29, 41, 53), seed=0, top_k=100),
    # the order-8 row of the paper's Table 2 (23 SNPs, 2048 individuals)
    "order8_M23_N2048": dict(order=8, M=23, N=2048, n_cases=1024, planted=(1, 4, 7, 10, 13, 16, 19, 22), seed=0,
                             top_k=10),
}


def make_workload(name):
    """``(G, y, spec, info)`` for one of :data:`WORKLOADS`."""
    spec = dict(WORKLOADS[name])
    G, y, info = make_case_control(spec["M"], spec["N"], spec["n_cases"], spec["planted"], spec["seed"])
    return G, y, spec, info


def batched_specs(n=64, seed_base=1000, m_range=(100, 2000), n_range=(500, 8000), frac_range=(0.2, 0.5),
                  orders=(2, 3), top_k=100):
    """Specs of ``n`` independent scans of uneven size, each with its own planted set."""
    out = []
    for i in range(n):
        seed = seed_base + i
        rng = np.random.default_rng(seed)
        order = int(rng.integers(orders[0], orders[-1] + 1))
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        frac = float(rng.uniform(*frac_range))
        n_cases = min(max(int(round(frac * N)), 1), N - 1)
        planted = tuple(int(v) for v in sorted(rng.choice(M, order, replace=False)))
        out.append(dict(order=order, M=M, N=N, n_cases=n_cases, planted=planted, seed=seed + 10**6,
                        top_k=top_k))
    return out


def served_pool_specs(n=32, seed_base=2000, m_range=(50, 1500), n_range=(500, 16000), small_m=(50, 200),
                      frac_range=(0.2, 0.5)):
    """Dataset pool for the serving workload.

    A third of the pool is drawn with ``M`` in ``small_m``; only those datasets
    take order-4 requests.  Each entry lists the orders it accepts.
    """
    out = []
    for d in range(n):
        seed = seed_base + d
        rng = np.random.default_rng(seed)
        small = d % 3 == 0
        lo, hi = small_m if small else m_range
        M = int(rng.integers(lo, hi + 1))
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        frac = float(rng.uniform(*frac_range))
        n_cases = min(max(int(round(frac * N)), 1), N - 1)
        orders = (2, 3, 4) if small else (2, 3)
        planted = tuple(int(v) for v in sorted(rng.choice(M, 3, replace=False)))
        out.append(dict(M=M, N=N, n_cases=n_cases, planted=planted, seed=seed + 10**6, orders=orders))
    return out


def served_requests(pool, n, seed=7, rate=20.0):
    """Request stream of the serving workload: each request picks a dataset of
    the pool uniformly and one of the orders that dataset accepts; arrival
    gaps are exponential with mean 1 / rate (Poisson arrivals).  Returns
    ([(dataset index, order)] * n, gaps in seconds)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        d = int(rng.integers(len(pool)))
        reqs.append((d, int(rng.choice(pool[d]["orders"]))))
    gaps = rng.exponential(1.0 / rate, n)
    return reqs, gaps
