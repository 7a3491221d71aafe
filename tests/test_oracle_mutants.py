"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/lcs_oracle.c``, plants one plausible mistake (a
dropped term, a wrong comparison, a wrong index or priority), compiles it to a
temporary library on the CPU and checks that at least one pin fails.
"""
import json
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import brute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "oracle", "lcs_oracle.c")).read()
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_example.json")))

MUTANTS = {
    # textbook recurrence: max replaced by min
    "dp_min_not_max": ("cur[j] = prev[j] > cur[j - 1] ? prev[j] : cur[j - 1];",
                       "cur[j] = prev[j] > cur[j - 1] ? cur[j - 1] : prev[j];"),
    # textbook recurrence: the +1 of a match dropped
    "dp_dropped_plus_one": ("cur[j] = prev[j - 1] + 1;", "cur[j] = prev[j - 1];"),
    # witness walk: DIAG tried before LEFT
    "walk_diag_first": ("if (CELL(i, j - 1) == c) {", "if (a[i - 1] != b[j - 1] && CELL(i, j - 1) == c) {"),
    # path listing: UP tried before LEFT (a path that leaves rows too early)
    "path_up_before_left": ("if (j > 0 && T[(size_t)i * W + (size_t)(j - 1)] == c) {",
                            "if (j > 0 && (i == 0 || T[(size_t)(i - 1) * W + (size_t)j] != c) && T[(size_t)i * W + (size_t)(j - 1)] == c) {"),
    # path listing: the exit column of a row recorded as its entry column
    "path_exit_is_entry": ("if (j > col_out[i]) col_out[i] = (int32_t)j;",
                           "if (j < col_out[i] || col_out[i] < 0) col_out[i] = (int32_t)j;"),
    # breakout definition: strict instead of >=
    "dist_strict": ("if (row[c] >= j) { d = i + c; break; }", "if (row[c] > j) { d = i + c; break; }"),
    # base case: the text's tail (from j_r + 2) instead of the example's (from j_r + 1)
    "base_tail_text": ("if (r == 0 || k > pos[r - 1] || c == n)", "if (r == 0 || k > pos[r - 1] + 1 || c == n)"),
    # base case: gap written one cell late
    "base_gap_index": ("cell[pos[k - 2] + 1] = pos[k - 1] - pos[k - 2];",
                       "cell[pos[k - 2] + (pos[k - 2] < n ? 1 : 0)] = pos[k - 1] - pos[k - 2] + 1;"),
    # combine: k starts at 1 as printed (drops the D_GL term)
    "combine_k_from_1": ("int64_t lo = j - hL > 0 ? j - hL : 0;", "int64_t lo = j - hL > 1 ? j - hL : 1;"),
    # combine: drops the k = j (D_GU) term
    "combine_no_upper_term": ("int64_t hi = j < hU ? j : hU;", "int64_t hi = j < hU ? j - 1 : hU;"),
}


def _build(tmp_path, name, src):
    c = tmp_path / (name + ".c")
    so = tmp_path / (name + ".so")
    c.write_text(src)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", str(so), str(c)])
    return oracle._bind(str(so))


def _pins(lib):
    """A compact run of the pins; returns the list of failures."""
    fails = []
    enc = lambda s: np.frombuffer(s.encode(), dtype=np.uint8).copy()
    a, b = GOLD["grid"]["a_rows"], GOLD["grid"]["b_cols"]
    n = len(b)
    if oracle.lcs_length("abccb", "abba", lib=lib) != 3:
        fails.append("three-string length")
    L, ai, bi = oracle.lcs_witness(enc("abccb"), enc("abba"), lib=lib)
    if L != 3 or list(ai) != [0, 1, 4] or list(bi) != [0, 1, 2]:
        fails.append("three-string witness")
    want = [n + 1 if v == "INF" else v - 1 for v in GOLD["base_row_t"]["final_1indexed"]] + [n + 1]
    if list(oracle.base_row(ord("t"), b, lib=lib)) != want:
        fails.append("base row example")
    D = oracle.dist_rows(a, 0, len(a), b, [0, 7], lib=lib)
    if list(D[0][:6]) != [0, 1, 2, 3, 4, 12] or D[1][5] != n + 1:
        fails.append("breakout example")
    r = np.random.default_rng(5)
    for _ in range(60):
        sig = int(r.integers(1, 4))
        x = r.integers(0, sig, int(r.integers(1, 9))).astype(np.uint8)
        y = r.integers(0, sig, int(r.integers(1, 9))).astype(np.uint8)
        if oracle.lcs_length(x, y, lib=lib) != brute.lcs_length(list(x), list(y)):
            fails.append("length vs brute force"); break
        Lw, wa, wb = oracle.lcs_witness(x, y, lib=lib)
        bl, ba, bb = brute.canonical_witness(list(x), list(y))
        if (Lw, list(wa), list(wb)) != (bl, ba, bb):
            fails.append("witness vs brute force"); break
    for _ in range(15):
        sig = int(r.integers(1, 4))
        h, nn = int(r.integers(2, 8)), int(r.integers(1, 14))
        x = r.integers(0, sig, h).astype(np.uint8)
        y = r.integers(0, sig, nn).astype(np.uint8)
        k = int(r.integers(1, h))
        DU = oracle.dist_rows(x, 0, k, y, lib=lib)
        DL = oracle.dist_rows(x, k, h, y, lib=lib)
        DG = oracle.dist_rows(x, 0, h, y, lib=lib)
        if not np.array_equal(oracle.combine(DU, DL, nn, lib=lib), DG):
            fails.append("combine vs definition"); break
        D1 = oracle.dist_rows(x[:1], 0, 1, y, lib=lib)
        if list(oracle.base_row(int(x[0]), y, lib=lib)) != list(D1[:, 1]):
            fails.append("base row vs definition"); break
        if int(np.sum(DG[0] <= nn)) - 1 != brute.lcs_length(list(x), list(y)):
            fails.append("top row vs brute force"); break
    for _ in range(40):
        sig = int(r.integers(1, 4))
        x = r.integers(0, sig, int(r.integers(0, 6))).astype(np.uint8)
        y = r.integers(0, sig, int(r.integers(0, 6))).astype(np.uint8)
        _, ci, co = brute.leftmost_path_rows(x, y)
        oi, oo = oracle.path_rows(x, y, lib=lib)
        if list(oi) != ci or list(oo) != co:
            fails.append("path rows vs brute force"); break
    return fails


def test_unmutated_oracle_passes(tmp_path):
    assert _pins(_build(tmp_path, "clean", SRC)) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert SRC.count(old) >= 1, "mutation anchor not found: " + old
    lib = _build(tmp_path, name, SRC.replace(old, new))
    assert _pins(lib), "planted mistake %s was not caught by any pin" % name
