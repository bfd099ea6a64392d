"""Host-side check of the signed cell form used by the matrix-core order-3
epilogue (inclusion-exclusion of Section 2.2's genotype tables with one
three-input add per step).

A cell whose index (9a + 3b + e, digit 2 = marginal over that SNP, genotype 2
after the step) has an odd number of digits 2 is held as B - 4n, the others as
4n, B = 8N + 4.  The marginal inputs are offset so that the steps land in that
form: pair cells B - 4n, single-SNP cells 4n - 4B, the class size 13B - 4n.
These tests recompute the steps in 32-bit modular arithmetic on random
genotype tables and compare with the counts taken directly, and check that
both forms address the mirrored screening table (t(n) at entry n and at entry
2N + 1 - n).  The device code is checked against the oracle by the GPU parity
tests; this pins the offsets themselves.
"""
import numpy as np

M32 = (1 << 32) - 1


def twos(x):
    return [x // 9, (x // 3) % 3, x % 3].count(2)


def marginal_form(cells):
    """F[x]: count of (a, b, e) with digit 2 meaning 'any genotype'."""
    F = []
    for x in range(27):
        d = [x // 9, (x // 3) % 3, x % 3]
        rng = [[v] if v < 2 else [0, 1, 2] for v in d]
        F.append(sum(cells[9 * a + 3 * b + e] for a in rng[0] for b in rng[1] for e in rng[2]))
    return F


def signed_steps(R):
    """The three passes, each step one sum of three (kernel: mobius3_signed)."""
    R = list(R)
    for r in range(9):
        R[18 + r] = (R[18 + r] + R[r] + R[9 + r]) & M32
    for a in range(3):
        for e in range(3):
            R[9 * a + 6 + e] = (R[9 * a + 6 + e] + R[9 * a + e] + R[9 * a + 3 + e]) & M32
    for ab in range(9):
        R[3 * ab + 2] = (R[3 * ab + 2] + R[3 * ab] + R[3 * ab + 1]) & M32
    return R


OFFSET = {0: (1, 0), 1: (-1, 1), 2: (1, -4), 3: (-1, 13)}  # (sign of 4n, multiple of B)


def test_signed_steps_give_counts():
    rng = np.random.default_rng(7)
    for _ in range(500):
        N = int(rng.integers(0, 5000))
        B = 8 * N + 4
        cells = [int(v) for v in rng.integers(0, 60, 27)]
        F = marginal_form(cells)
        start = [((OFFSET[twos(x)][0] * 4 * F[x]) + OFFSET[twos(x)][1] * B) & M32 for x in range(27)]
        out = signed_steps(start)
        for x in range(27):
            want = 4 * cells[x] if twos(x) % 2 == 0 else B - 4 * cells[x]
            assert out[x] == want & M32, (x, out[x], want)


def test_both_forms_address_the_mirrored_table():
    N = 37
    B = 8 * N + 4
    table = np.zeros(2 * N + 2, np.int64)
    t = np.array([0 if n < 2 else n * 1000 + 7 for n in range(N + 1)])
    table[: N + 1] = t
    table[N + 1:] = t[::-1]  # entry 2N + 1 - n holds t(n)
    for n0 in range(N + 1):
        for n1 in range(N + 1 - n0):
            assert table[(4 * n0) // 4] == t[n0]
            assert table[(B - 4 * n0) // 4] == t[n0]
            # the class-sum cell of an odd cell: a0 + a1 - B = B - 4 (n0 + n1)
            s = (B - 4 * n0) + (B - 4 * n1) - B
            assert table[s // 4] == t[n0 + n1]
