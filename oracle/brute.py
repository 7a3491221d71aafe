"""Brute-force LCS for tiny strings (length <= 12) -- test infrastructure only.

Nothing here uses a dynamic program: it enumerates index subsets directly, so it
pins the dynamic-program oracle from outside (problem statement, Section I).
"""
from __future__ import annotations

from itertools import combinations


def is_subsequence(s, t) -> bool:
    """True if the sequence s can be read, in order, inside t."""
    it = iter(t)
    return all(any(x == y for y in it) for x in s)


def lcs_length(a, b) -> int:
    """Largest k such that some k symbols of the shorter string, kept in order, occur in the other."""
    a, b = list(a), list(b)
    short, other = (a, b) if len(a) <= len(b) else (b, a)
    for k in range(len(short), 0, -1):
        for idx in combinations(range(len(short)), k):
            if is_subsequence([short[i] for i in idx], other):
                return k
    return 0


def canonical_witness(a, b):
    """(L, a_idx, b_idx) characterised without a table.

    Among all maximum alignments take the lexicographically smallest tuple of
    b positions; for that symbol string take the embedding in a whose
    positions are as large as possible (greedy from the right).
    """
    a, b = list(a), list(b)
    L = lcs_length(a, b)
    if L == 0:
        return 0, [], []
    for bidx in combinations(range(len(b)), L):          # lexicographic order
        syms = [b[j] for j in bidx]
        if is_subsequence(syms, a):
            aidx = []
            pos = len(a) - 1
            for s in reversed(syms):
                while a[pos] != s:
                    pos -= 1
                aidx.append(pos)
                pos -= 1
            return L, list(reversed(aidx)), list(bidx)
    raise AssertionError("unreachable")


def common_subsequences_of_length(a, b, k):
    """Every symbol string of length k that is a subsequence of both a and b."""
    out = set()
    for idx in combinations(range(len(a)), k):
        s = tuple(a[i] for i in idx)
        if s not in out and is_subsequence(s, b):
            out.add(s)
    return out


def max_paths(a, b):
    """Every heaviest monotone path of the grid graph (Section II-A), enumerated
    move by move: right, down, or the weight-1 diagonal where a[r] == b[c].
    Each path is returned as its (col_in, col_out) per grid row r = 0..m.
    For tiny strings only (the count of paths grows exponentially)."""
    a, b = list(a), list(b)
    m, n = len(a), len(b)
    best, found = -1, []

    def walk(r, c, w, rows):
        nonlocal best, found
        rows[r][0] = min(rows[r][0], c)
        rows[r][1] = max(rows[r][1], c)
        if r == m and c == n:
            if w > best:
                best, found = w, []
            if w == best:
                found.append(tuple((x, y) for x, y in rows))
            return
        if c < n:
            walk(r, c + 1, w, [list(x) for x in rows])
        if r < m:
            nxt = [list(x) for x in rows]
            walk(r + 1, c, w, nxt)
            if c < n and a[r] == b[c]:
                walk(r + 1, c + 1, w + 1, [list(x) for x in rows])

    walk(0, 0, 0, [[n + 1, -1] for _ in range(m + 1)])
    return best, found


def leftmost_path_rows(a, b):
    """(L, col_in, col_out) of the leftmost heaviest path: row by row the
    smallest entry and exit columns over ALL heaviest paths.  Asserts that this
    row-wise minimum is itself one of the heaviest paths (the leftmost one)."""
    L, paths = max_paths(a, b)
    m = len(list(a))
    cin = [min(p[r][0] for p in paths) for r in range(m + 1)]
    cout = [min(p[r][1] for p in paths) for r in range(m + 1)]
    assert tuple(zip(cin, cout)) in set(paths), "row-wise minimum is not a heaviest path"
    return max(L, 0), cin, cout
