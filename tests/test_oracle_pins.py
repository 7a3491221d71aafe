"""Pins for the CPU oracle: paper values, brute force, closed forms, invariants.

None of these compares the oracle with itself: each check comes from the
paper's printed example, from subsequence enumeration, from a closed form, or
from a property the mathematics fixes.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute, paper_search

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")))


def enc(s):
    return np.frombuffer(s.encode(), dtype=np.uint8).copy()


def dec(arr):
    return bytes(np.asarray(arr, dtype=np.uint8)).decode()


# ---------------------------------------------------------------- paper values


def test_three_string_example():
    """Section I: LCS(abccb, abba, acbb) = abb; pairwise LCS(abccb, abba) = 3."""
    s1, s2, s3 = GOLD["three_strings"]["strings"]
    want = GOLD["three_strings"]["lcs"]
    assert oracle.lcs_length(s1, s2) == 3
    L, ai, bi = oracle.lcs_witness(enc(s1), enc(s2))
    assert L == 3 and dec(enc(s1)[ai]) == want
    assert list(ai) == [0, 1, 4] and list(bi) == [0, 1, 2]
    # the three-string answer itself, by enumeration
    common = brute.common_subsequences_of_length(s1, s2, 3)
    common = {c for c in common if brute.is_subsequence(c, s3)}
    assert common == {tuple(want)}
    assert not any(brute.is_subsequence(c, s3) for c in brute.common_subsequences_of_length(s1, s2, 4))


def test_base_row_worked_example():
    """Section II-B-3: D_{G_1} for a_1 = t against gatttatgcagg."""
    g = GOLD["base_row_t"]
    b = GOLD["grid"]["b_cols"]
    n = len(b)
    got = oracle.base_row(ord(g["symbol"]), b)
    want = [n + 1 if v == "INF" else v - 1 for v in g["final_1indexed"]] + [n + 1]
    assert list(got) == want
    pos = [j + 1 for j, ch in enumerate(b) if ch == g["symbol"]]
    assert pos == g["positions_1indexed"]


def test_breakouts_of_vertex_1_1():
    """Section II-B-1: breakouts of vertex (1,1) are (9,2),(9,3),(9,4),(9,5),(9,13)."""
    a, b = GOLD["grid"]["a_rows"], GOLD["grid"]["b_cols"]
    n = len(b)
    D = oracle.dist_rows(a, 0, len(a), b, [GOLD["breakouts_vertex_1_1"]["vertex_0indexed"]])[0]
    cols = [c - 1 for c in GOLD["breakouts_vertex_1_1"]["columns_1indexed"]]
    assert list(D[: len(cols) + 1]) == [0] + cols
    assert all(v == n + 1 for v in D[len(cols) + 1:])
    # Fig. 2's cell D_G(1,3): third breakout of (1,1) is column 4 (1-indexed)
    f = GOLD["fig2_cell"]
    assert D[f["weight"]] == f["column_1indexed"] - 1
    # the LCS of the Fig. 1 strings is the largest reachable weight
    assert oracle.lcs_length(a, b) == len(cols)


def test_no_fifth_breakout_of_vertex_1_8():
    a, b = GOLD["grid"]["a_rows"], GOLD["grid"]["b_cols"]
    g = GOLD["no_fifth_breakout_vertex_1_8"]
    D = oracle.dist_rows(a, 0, len(a), b, [g["vertex_0indexed"]])[0]
    assert D[g["weight"]] == len(b) + 1
    assert D[g["weight"] - 1] <= len(b)


# ---------------------------------------------------------------- brute force


def _rand_pair(r, maxlen=10, maxsig=4):
    sig = int(r.integers(1, maxsig + 1))
    m, n = int(r.integers(0, maxlen + 1)), int(r.integers(0, maxlen + 1))
    return r.integers(0, sig, m).astype(np.uint8), r.integers(0, sig, n).astype(np.uint8), sig


def test_length_and_witness_vs_brute_force():
    r = np.random.default_rng(11)
    for _ in range(300):
        a, b, _ = _rand_pair(r)
        L = brute.lcs_length(list(a), list(b))
        assert oracle.lcs_length(a, b) == L
        Lw, ai, bi = oracle.lcs_witness(a, b)
        bl, bai, bbi = brute.canonical_witness(list(a), list(b))
        assert Lw == L == bl
        assert list(ai) == bai and list(bi) == bbi


def test_path_rows_vs_brute_force():
    """Section II-E path listing: the oracle's per-row entry/exit columns are the
    row-wise minimum over every heaviest path, enumerated move by move (which is
    itself a heaviest path: the leftmost one), and its diagonal steps are the
    brute-force canonical witness."""
    r = np.random.default_rng(20)
    for _ in range(250):
        sig = int(r.integers(1, 4))
        m, n = int(r.integers(0, 7)), int(r.integers(0, 7))
        a = r.integers(0, sig, m).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        L, cin, cout = brute.leftmost_path_rows(a, b)
        oi, oo = oracle.path_rows(a, b)
        assert list(oi) == cin and list(oo) == cout, (a, b)
        assert oi[0] == 0 and oo[m] == n
        # diagonal steps (row r leaves at c, row r + 1 enters at c + 1) = the witness
        diag = [(rr, int(oo[rr])) for rr in range(m) if oi[rr + 1] == oo[rr] + 1]
        bl, ba, bb = brute.canonical_witness(list(a), list(b))
        assert diag == list(zip(ba, bb)) and len(diag) == L == bl


def test_path_rows_closed_forms():
    """Unary alphabet: the leftmost path goes straight down to row m - n (m >= n)
    and then diagonally; with m < n it goes diagonally first and then right
    along row m.  Disjoint alphabets: straight down column 0, then along row m."""
    for m, n in [(6, 3), (3, 6), (5, 5), (0, 4), (4, 0)]:
        cin, cout = oracle.path_rows(np.zeros(m, np.uint8), np.zeros(n, np.uint8))
        if m >= n:
            want_in = [max(0, r - (m - n)) for r in range(m + 1)]
            want_out = list(want_in)
        else:
            want_in = list(range(m + 1))
            want_out = list(range(m)) + [n]
        assert list(cin) == want_in and list(cout) == want_out, (m, n)
    cin, cout = oracle.path_rows(np.zeros(5, np.uint8), np.ones(7, np.uint8))
    assert list(cin) == [0] * 6 and list(cout) == [0] * 5 + [7]


def test_dist_rows_vs_brute_force():
    """D(i, j) = smallest c with LCS(strip, b[i:c]) >= j, with LCS by enumeration."""
    r = np.random.default_rng(12)
    for _ in range(60):
        sig = int(r.integers(1, 4))
        h, n = int(r.integers(0, 6)), int(r.integers(0, 9))
        a = r.integers(0, sig, h).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        D = oracle.dist_rows(a, 0, h, b)
        for i in range(n + 1):
            for j in range(h + 1):
                want = n + 1
                for c in range(i, n + 1):
                    if brute.lcs_length(list(a), list(b[i:c])) >= j:
                        want = c
                        break
                assert D[i, j] == want, (a, b, i, j)


# ---------------------------------------------------------------- closed forms


def test_unary_alphabet_closed_form():
    for m, n in [(0, 5), (5, 0), (7, 7), (30, 12), (12, 30), (1, 1)]:
        a = np.zeros(m, np.uint8)
        b = np.zeros(n, np.uint8)
        L, ai, bi = oracle.lcs_witness(a, b)
        assert L == min(m, n) == oracle.lcs_length(a, b)
        if m >= n:
            assert list(ai) == [m - n + t for t in range(L)] and list(bi) == list(range(L))
        else:
            assert list(ai) == list(range(L)) and list(bi) == list(range(L))
        # D for a unary strip of h rows: D(i, j) = i + j while it fits
        if m <= 8:
            D = oracle.dist_rows(a, 0, m, b)
            for i in range(n + 1):
                for j in range(m + 1):
                    assert D[i, j] == (i + j if i + j <= n else n + 1)


def test_self_disjoint_empty():
    r = np.random.default_rng(13)
    x = r.integers(0, 20, 300).astype(np.uint8)
    L, ai, bi = oracle.lcs_witness(x, x)
    assert L == 300 and list(ai) == list(range(300)) and list(bi) == list(range(300))
    assert oracle.lcs_length(r.integers(0, 4, 200).astype(np.uint8),
                             r.integers(4, 8, 150).astype(np.uint8)) == 0
    assert oracle.lcs_length(np.zeros(0, np.uint8), x) == 0
    assert oracle.lcs_witness(x, np.zeros(0, np.uint8))[0] == 0


# ---------------------------------------------------------------- invariants


def test_length_invariants():
    r = np.random.default_rng(14)
    for _ in range(40):
        sig = int(r.integers(2, 21))
        m, n = int(r.integers(1, 120)), int(r.integers(1, 120))
        a = r.integers(0, sig, m).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        L = oracle.lcs_length(a, b)
        assert 0 <= L <= min(m, n)
        assert oracle.lcs_length(b, a) == L                       # symmetry
        assert oracle.lcs_length(a[::-1], b[::-1]) == L           # reversal
        perm = r.permutation(256).astype(np.uint8)
        assert oracle.lcs_length(perm[a], perm[b]) == L           # relabelling
        s = np.uint8(r.integers(0, sig))
        La = oracle.lcs_length(np.append(a, s), b)
        assert La - L in (0, 1)                                   # appending
        Lw, ai, bi = oracle.lcs_witness(a, b)                     # witness is valid
        assert Lw == L and np.all(a[ai] == b[bi])
        assert np.all(np.diff(ai) > 0) and np.all(np.diff(bi) > 0)


def test_dist_invariants():
    """D(i,0)=i, D(i,j) >= i+j, strictly increasing in j, interlacing across i."""
    r = np.random.default_rng(15)
    for _ in range(12):
        sig = int(r.integers(1, 6))
        h, n = int(r.integers(1, 20)), int(r.integers(1, 60))
        a = r.integers(0, sig, h).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        D = oracle.dist_rows(a, 0, h, b).astype(np.int64)
        INF = n + 1
        assert np.all(D[:, 0] == np.arange(n + 1))
        fin = D <= n
        J = np.arange(h + 1)[None, :]
        I = np.arange(n + 1)[:, None]
        assert np.all(D[fin] >= (I + J)[fin])
        for i in range(n + 1):
            f = D[i][D[i] <= n]
            assert np.all(np.diff(f) > 0)
            assert np.all(D[i][len(f):] == INF)            # unreachable entries form a suffix
        assert np.all(D[1:, :] >= D[:-1, :])                # non-decreasing in i
        assert np.all(D[1:, :-1] <= D[:-1, 1:])             # D(i+1, j) <= D(i, j+1)
        # top row against the textbook table: max{j : D(0,j) <= k} = C[h][k]
        row = oracle.lcs_last_row(a, b)
        for k in range(n + 1):
            assert int(np.sum(D[0] <= k)) - 1 == row[k]


def test_base_row_equals_single_row_definition():
    """Section II-B-3's construction equals the breakout definition for one row."""
    r = np.random.default_rng(16)
    for _ in range(50):
        sig = int(r.integers(1, 6))
        n = int(r.integers(0, 40))
        b = r.integers(0, sig, n).astype(np.uint8)
        s = int(r.integers(0, sig))
        D = oracle.dist_rows(np.array([s], np.uint8), 0, 1, b)
        assert list(oracle.base_row(s, b)) == list(D[:, 1])


# ---------------------------------------------------------------- combine


def test_combine_equation_reproduces_definition():
    """Section II-B-1 equation: combining the halves' D gives the whole strip's D."""
    r = np.random.default_rng(17)
    for _ in range(40):
        sig = int(r.integers(1, 5))
        h, n = int(r.integers(2, 14)), int(r.integers(0, 30))
        a = r.integers(0, sig, h).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        k = int(r.integers(1, h))
        DU = oracle.dist_rows(a, 0, k, b)
        DL = oracle.dist_rows(a, k, h, b)
        DG = oracle.dist_rows(a, 0, h, b)
        assert np.array_equal(oracle.combine(DU, DL, n), DG)


def test_paper_search_matches_brute_force_combine():
    """Alg. 1 + Alg. 2 (with the find_cell / partner / unset-column readings) give the
    same minima and the same smallest argmins as the brute-force equation."""
    r = np.random.default_rng(18)
    for _ in range(40):
        sig = int(r.integers(1, 5))
        hU, hL, n = int(r.integers(1, 8)), int(r.integers(1, 8)), int(r.integers(0, 25))
        a = r.integers(0, sig, hU + hL).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        DU = oracle.dist_rows(a, 0, hU, b)
        DL = oracle.dist_rows(a, hU, hU + hL, b)
        DG, K = oracle.combine(DU, DL, n, with_argk=True)
        PG, PK = paper_search.combine_by_colmins(DU.tolist(), DL.tolist(), n)
        assert np.array_equal(np.array(PG), DG)
        assert np.array_equal(np.array(PK), K)


def test_monotone_argmin_and_noncrossing():
    """Properties the search relies on: the smallest argmin is non-decreasing in j
    (Section II-B-1, monotone matrix) and the crossing column D_U(i, k*) is
    non-decreasing in i (leftmost optimal paths do not cross)."""
    r = np.random.default_rng(19)
    for _ in range(30):
        sig = int(r.integers(1, 5))
        hU, hL, n = int(r.integers(1, 10)), int(r.integers(1, 10)), int(r.integers(1, 40))
        a = r.integers(0, sig, hU + hL).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        DU = oracle.dist_rows(a, 0, hU, b)
        DL = oracle.dist_rows(a, hU, hU + hL, b)
        DG, K = oracle.combine(DU, DL, n, with_argk=True)
        for i in range(n + 1):
            ks = K[i][K[i] >= 0]
            assert np.all(np.diff(ks) >= 0)
        for j in range(hU + hL + 1):
            xs = [DU[i, K[i, j]] for i in range(n + 1) if K[i, j] >= 0]
            assert np.all(np.diff(xs) >= 0)
