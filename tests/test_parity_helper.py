"""The GPU-vs-oracle comparison helper catches the mistakes it is meant to
catch (CPU only: the oracle's own best-K list, with planted mistakes, stands
in for a GPU result)."""
import itertools
import math

import numpy as np
import pytest

from parity import check_topk
from synth import random_genotypes


def _result(orc, G, y, order, K):
    r = orc.scan(G, y, order, K)
    return r["combos"].copy(), r["scores"].astype(np.float32), r["tables"].astype(np.uint32), r


def test_helper_accepts_the_oracle_and_rejects_planted_mistakes(orc):
    G, y = random_genotypes(14, 150, seed=5, case_fraction=0.4)
    order, K = 3, 12
    c, s, t, ref = _result(orc, G, y, order, K)
    check_topk(orc, G, y, order, K, c, s, t, ref=ref)
    mistakes = []
    c2 = c.copy()
    c2[[2, 3]] = c2[[3, 2]]
    s2 = s.copy()
    s2[[2, 3]] = s2[[3, 2]]
    t2 = t.copy()
    t2[[2, 3]] = t2[[3, 2]]
    mistakes.append(("two results swapped", c2, s2, t2))
    t3 = t.copy()
    t3[4, 0, 5] += 1
    t3[4, 1, 5] -= 1
    mistakes.append(("a cell moved between classes", c, s, t3))
    s4 = s.copy()
    s4[1] = np.float32(s4[1] * (1 + 3e-5))
    mistakes.append(("a score off by 3e-5", c, s4, t))
    worst = orc.scan(G, y, order, math.comb(14, order))
    c5, s5, t5 = c.copy(), s.copy(), t.copy()
    c5[-1], s5[-1], t5[-1] = worst["combos"][-1], np.float32(worst["scores"][-1]), worst["tables"][-1]
    mistakes.append(("a result outside the best K", c5, s5, t5))
    c6 = c.copy()
    c6[0] = c6[0][::-1]
    mistakes.append(("indices not ascending", c6, s, t))
    for what, cc, ss, tt in mistakes:
        with pytest.raises(AssertionError):
            check_topk(orc, G, y, order, K, cc, ss, tt, ref=ref)
        print("caught:", what)


def test_helper_checks_tie_order(orc):
    # identical SNPs: every combination has the same table and score, so the
    # order must be lexicographic
    G0, y = random_genotypes(1, 60, seed=17, case_fraction=0.5)
    G = np.repeat(G0, 6, axis=0)
    c, s, t, ref = _result(orc, G, y, 2, 15)
    assert [tuple(x) for x in c] == list(itertools.combinations(range(6), 2))
    check_topk(orc, G, y, 2, 15, c, s, t, ref=ref)
    with pytest.raises(AssertionError):
        check_topk(orc, G, y, 2, 15, c[::-1].copy(), s, t[::-1].copy(), ref=ref)
