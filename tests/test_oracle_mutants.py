"""Plausible mistakes planted in a copy of the oracle source must fail a pin.

Each mutant is a textual edit of ``oracle/epi_oracle.c`` compiled into a
temporary library and checked in a child process (a broken oracle may crash
or loop).  The real oracle source is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "epi_oracle.c")

MUTANTS = {
    # cell index built with the operands of the mixed radix transposed
    "cell_index_transposed": ("x = x * 3 + g;", "x = g * 3 + x;"),
    # joint entropy accumulated with the wrong sign
    "hxy_sign": ("h_xy -= p * log(p);", "h_xy += p * log(p);"),
    # H(Y) dropped from Equation 1
    "drop_hy": ("return h_x + h_y - h_xy;", "return h_x - h_xy;"),
    # wrong denominator for p(x)
    "px_denominator": ("double p = n_x / m;", "double p = n_x / (m + 1.0);"),
    # cases and controls swapped in the table
    "class_swap": ("int cls = y[s] ? 0 : 1;", "int cls = y[s] ? 1 : 0;"),
    # enumeration stops one value early
    "enum_off_by_one": ("c[t] == M - k + t)", "c[t] == M - k + t - 1)"),
    # ties broken towards the larger combination
    "tie_break_reversed": ("return a[t] < b[t];", "return a[t] > b[t];"),
    # unranking off by one (splits of the rank space overlap)
    "unrank_off_by_one": ("if (rank < block)", "if (rank <= block)"),
    # top-K keeps the worse entry
    "topk_compare": ("return a->mi > b->mi;", "return a->mi < b->mi;"),
    # genotype-table bits numbered from the other end of the word
    "gt_bit_order": ("(uint32_t)1 << (b % 32)", "(uint32_t)1 << (31 - b % 32)"),
    # genotype-table classes in swapped word ranges
    "gt_class_words": ("(cl ? words0 : 0) + b / 32", "(cl ? 0 : words1) + b / 32"),
    # genotype-table row index with the SNPs in reverse significance
    "gt_row_radix": ("row = 3 * row + geno;", "row = row + geno * (t == 0 ? 1 : (t == 1 ? 3 : 9));"),
    # score list: per-row table offset of one class instead of two
    "score_list_table_offset": ("out_tables + (int64_t)i * 2 * P : table;", "out_tables + (int64_t)i * P : table;"),
    # score list: combinations read one index apart instead of k
    "score_list_combo_offset": ("combos + (int64_t)i * k, k, t)", "combos + (int64_t)i, k, t)"),
    # score list: every score written to the first slot
    "score_list_score_index": ("out_scores[i] = oracle_mi(t, k);", "out_scores[0] = oracle_mi(t, k);"),
    # digest: indices folded without their offset
    "digest_index_fold": ("h = splitmix_out(h + (uint64_t)c[t] + 1);", "h = splitmix_out(h + (uint64_t)c[t]);"),
    # digest: cell weights indexed by the cell alone (classes share weights)
    "digest_cell_weight": ("splitmix_out(2 * (uint64_t)x + (uint64_t)cls + 1)", "splitmix_out((uint64_t)x + 1)"),
    # digest: the last combination of every thread's range left out
    "digest_drop_last": ("j->sum += digest_term(c, j->k, j->table);",
                         "if (r + 1 < j->end) j->sum += digest_term(c, j->k, j->table);"),
}

CHILD = r"""
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle, oracle_pins
o = oracle.Oracle(oracle.load({lib!r}))
print(",".join(oracle_pins.run_battery(o)))
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    sys.path.insert(0, ROOT)
    import oracle

    lib = oracle.build(str(mut), str(tmp_path / "libmutant.so"))
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    try:
        proc = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    except subprocess.TimeoutExpired:
        return  # a mutant that never finishes is caught too
    if proc.returncode != 0:
        return  # crashed: caught
    failed = [f for f in proc.stdout.strip().splitlines()[-1].split(",") if f] if proc.stdout.strip() else []
    assert failed, f"mutant {name} passed every pin"
