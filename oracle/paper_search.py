"""Alg. 1 (column minima) and Alg. 2 (minimum index) of the paper, in its order.

TEST INFRASTRUCTURE ONLY.  Pure Python, small inputs.  Used to pin three
readings of the printed pseudo-code against the brute-force combine:

* ``find_cell`` is used but never defined in the paper.  Reading: the
  candidate value of split k for column ``col`` of vertex ``vertex``,
  D_L(D_U(vertex, k), col - k), unreachable when k > col, k > hU,
  col - k > hL or D_U(vertex, k) is unreachable.
* The partner index of Alg. 2 is printed garbled.  Reading:
  (j AND NOT exp) OR (exp - 1), i.e. the last element of the lower half block
  (a Sklansky prefix network); ``<=`` keeps the earlier index on ties.
* Alg. 1 leaves ``mins`` unset right of a column whose minimum is
  unreachable.  Reading: those columns are unreachable.
"""
from __future__ import annotations


def find_cell(DU, DL, vertex, k, col, hU, hL, INF):
    if k < 0 or k > col or k > hU or col - k > hL:
        return INF
    x = DU[vertex][k]
    if x >= INF:
        return INF
    return min(int(DL[x][col - k]), INF)


def find_min_index(DU, DL, vertex, col, top, bottom, hU, hL, INF):
    """Alg. 2: index (offset by ``top``) of the minimum of a column, ties to the smallest."""
    listsize = bottom - top + 1
    prefix = [find_cell(DU, DL, vertex, i + top, col, hU, hL, INF) for i in range(listsize)]
    min_index = list(range(listsize))
    exp = 1
    while exp < listsize:
        expm1 = exp - 1
        # one parallel round; the partner never has bit ``exp`` set, so no
        # element is both read and written within a round
        for j in range(listsize):
            if j & exp:
                partner = (j & ~exp) | expm1
                if prefix[partner] <= prefix[j]:
                    prefix[j] = prefix[partner]
                    min_index[j] = min_index[partner]
        exp <<= 1
    return min_index[listsize - 1] + top


def find_col_mins(DU, DL, vertex, left, right, top, bottom, mins, firstind, hU, hL, INF):
    """Alg. 1: column minima of a monotone matrix by divide and conquer."""
    cols = right - left + 1
    if cols < 1:
        return
    mid = (right + left + 1) // 2                      # ceiling of the midpoint
    mi = find_min_index(DU, DL, vertex, mid, top, bottom, hU, hL, INF)
    mins[firstind + mid - left] = mi
    if find_cell(DU, DL, vertex, mi, mid, hU, hL, INF) != INF:
        find_col_mins(DU, DL, vertex, left, mid - 1, top, mi, mins, firstind, hU, hL, INF)
        find_col_mins(DU, DL, vertex, mid + 1, right, mi, bottom, mins,
                      firstind + mid - left + 1, hU, hL, INF)
    else:
        find_col_mins(DU, DL, vertex, left, mid - 1, top, bottom, mins, firstind, hU, hL, INF)


def combine_by_colmins(DU, DL, n):
    """D_G and its argmins for every vertex via Alg. 1 + Alg. 2 (unset columns unreachable)."""
    INF = n + 1
    hU, hL = len(DU[0]) - 1, len(DL[0]) - 1
    H = hU + hL
    DG, K = [], []
    for v in range(n + 1):
        mins = [None] * (H + 1)
        find_col_mins(DU, DL, v, 0, H, 0, hU, mins, 0, hU, hL, INF)
        row, krow = [], []
        for col in range(H + 1):
            val = INF if mins[col] is None else find_cell(DU, DL, v, mins[col], col, hU, hL, INF)
            row.append(val)
            krow.append(mins[col] if val < INF else -1)
        DG.append(row)
        K.append(krow)
    return DG, K
