/*
 * CPU oracle for the LCS hot path of "Parallel Longest Common SubSequence
 * Analysis In Chapel" (Vahidi, Schieber, Du, Bader; arXiv 2309.09072).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file: only tests/, __graft_entry__.smoke() and the cpu_baseline
 * leg of bench.py use it.  It shares no code, header, table or helper with the
 * HIP path.  Everything here is plain, single-threaded and slow on purpose, so
 * that each function can be checked against the paper by eye.
 *
 * Conventions (0-indexed): a is the row string (length m), b the column string
 * (length n).  Grid vertices are (r, c), 0 <= r <= m, 0 <= c <= n.  A column
 * value above n stands for "no such vertex" (the paper's infinity); the value
 * written is n + 1.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * Textbook dynamic program (Section I): C[i][j] = C[i-1][j-1] + 1 when
 * a[i-1] == b[j-1], else max(C[i-1][j], C[i][j-1]); C[0][*] = C[*][0] = 0.
 * Two rolling rows.  Returns C[m][n].
 */
int64_t oracle_lcs_length(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n)
{
    if (m <= 0 || n <= 0) return 0;
    int32_t *prev = calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *cur = calloc((size_t)n + 1, sizeof(int32_t));
    if (!prev || !cur) { free(prev); free(cur); return -1; }
    for (int64_t i = 1; i <= m; i++) {
        cur[0] = 0;
        for (int64_t j = 1; j <= n; j++) {
            if (a[i - 1] == b[j - 1])
                cur[j] = prev[j - 1] + 1;
            else
                cur[j] = prev[j] > cur[j - 1] ? prev[j] : cur[j - 1];
        }
        int32_t *t = prev; prev = cur; cur = t;
    }
    int64_t L = prev[n];
    free(prev); free(cur);
    return L;
}

/*
 * Last row of the textbook dynamic program: row[c] = LCS(a, b[0:c]) for
 * c = 0..n.  Used by the semi-local checks of the breakout matrices.
 */
int oracle_lcs_last_row(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n, int32_t *row)
{
    int32_t *prev = calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *cur = calloc((size_t)n + 1, sizeof(int32_t));
    if (!prev || !cur) { free(prev); free(cur); return -1; }
    for (int64_t i = 1; i <= m; i++) {
        cur[0] = 0;
        for (int64_t j = 1; j <= n; j++) {
            if (a[i - 1] == b[j - 1])
                cur[j] = prev[j - 1] + 1;
            else
                cur[j] = prev[j] > cur[j - 1] ? prev[j] : cur[j - 1];
        }
        int32_t *t = prev; prev = cur; cur = t;
    }
    memcpy(row, prev, sizeof(int32_t) * ((size_t)n + 1));
    free(prev); free(cur);
    return 0;
}

/*
 * Canonical witness.  Builds the full textbook table and walks back from
 * (m, n), preferring LEFT (same score one column to the left), then DIAG (a
 * match that accounts for the score), then UP.  The emitted match pairs
 * (a index, b index) are returned in increasing order.  This walk yields the
 * optimal path whose entry column in every row is as small as possible.
 * Returns L, or -1 if the table cannot be allocated.
 */
int64_t oracle_lcs_witness(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                           int32_t *a_idx, int32_t *b_idx)
{
    if (m <= 0 || n <= 0) return 0;
    size_t W = (size_t)n + 1;
    int wide = (m > 65535 && n > 65535);
    void *tab = calloc(((size_t)m + 1) * W, wide ? sizeof(int32_t) : sizeof(uint16_t));
    if (!tab) return -1;
    uint16_t *T16 = (uint16_t *)tab;
    int32_t *T32 = (int32_t *)tab;
#define CELL(i, j) (wide ? (int64_t)T32[(size_t)(i) * W + (size_t)(j)] \
                         : (int64_t)T16[(size_t)(i) * W + (size_t)(j)])
#define SETC(i, j, v) do { if (wide) T32[(size_t)(i) * W + (size_t)(j)] = (int32_t)(v); \
                           else T16[(size_t)(i) * W + (size_t)(j)] = (uint16_t)(v); } while (0)
    for (int64_t i = 1; i <= m; i++) {
        for (int64_t j = 1; j <= n; j++) {
            int64_t v;
            if (a[i - 1] == b[j - 1]) v = CELL(i - 1, j - 1) + 1;
            else {
                int64_t up = CELL(i - 1, j), left = CELL(i, j - 1);
                v = up > left ? up : left;
            }
            SETC(i, j, v);
        }
    }
    int64_t L = CELL(m, n);
    int64_t i = m, j = n, t = L;
    while (i > 0 && j > 0) {
        int64_t c = CELL(i, j);
        if (CELL(i, j - 1) == c) {
            j--;                                   /* LEFT */
        } else if (a[i - 1] == b[j - 1]) {
            t--;                                   /* DIAG: a match */
            a_idx[t] = (int32_t)(i - 1);
            b_idx[t] = (int32_t)(j - 1);
            i--; j--;
        } else {
            i--;                                   /* UP */
        }
    }
#undef CELL
#undef SETC
    free(tab);
    return L;
}

/*
 * Breakout matrix by definition (Section II-B-1): for the strip made of rows
 * r0..r1 of the grid (symbols a[r0:r1]), D(i, j) is the smallest column c >= i
 * of the strip's bottom row reachable from top-row column i by a path of
 * weight j, i.e. the smallest c with LCS(a[r0:r1], b[i:c]) >= j; n + 1 if
 * there is none.  The 0-th breakout of vertex i is i itself (Section II-B-3).
 *
 * For every requested vertex verts[v] (0 <= verts[v] <= n) this runs a fresh
 * textbook dynamic program of a[r0:r1] against b[i:n] and reads the answer
 * off its last row.  out is row-major, nverts x (h + 1), h = r1 - r0.
 */
int oracle_dist_rows(const uint8_t *a, int64_t r0, int64_t r1, const uint8_t *b, int64_t n,
                     const int32_t *verts, int64_t nverts, int32_t *out)
{
    int64_t h = r1 - r0;
    if (h < 0) return -1;
    int32_t *row = malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!row) return -1;
    for (int64_t v = 0; v < nverts; v++) {
        int64_t i = verts[v];
        if (i < 0 || i > n) { free(row); return -1; }
        int64_t len = n - i;
        if (oracle_lcs_last_row(a + r0, h, b + i, len, row) != 0) { free(row); return -1; }
        for (int64_t j = 0; j <= h; j++) {
            int64_t d = n + 1;
            for (int64_t c = 0; c <= len; c++) {
                if (row[c] >= j) { d = i + c; break; }
            }
            out[v * (h + 1) + j] = (int32_t)d;
        }
    }
    free(row);
    return 0;
}

/*
 * Base case of Section II-B-3, following its steps in order for the two-row
 * grid of one symbol ah = a_h against b (1-indexed inside, as in the paper):
 *   1. list the positions j_1 < ... < j_r where b_j == a_h;
 *   2. write j_1 + 1 into cell 1 and the gap j_k - j_{k-1} into cell
 *      j_{k-1} + 1 (1 < k <= r); the other cells are still empty (zero);
 *   3. replace each cell k by the sum of cells 1..k;
 *   4. mark the cells after the last match as unreachable.  The printed worked
 *      example makes every cell from j_r + 1 on unreachable, and that is the
 *      reading taken here (a start at column j_r + 1 sees no match to its
 *      right).
 * out receives, 0-indexed, the first breakout of each top vertex c = 0..n:
 * out[c] = (paper cell c + 1) - 1, and n + 1 for "unreachable"; the vertex
 * c = n always has none.  Returns the number of matches r.
 */
int64_t oracle_base_row(uint8_t ah, const uint8_t *b, int64_t n, int32_t *out)
{
    int64_t *pos = malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t *cell = calloc((size_t)n + 2, sizeof(int64_t));   /* cells 1..n used */
    if (!pos || !cell) { free(pos); free(cell); return -1; }
    int64_t r = 0;
    for (int64_t j = 1; j <= n; j++)                          /* step 1 */
        if (b[j - 1] == ah) pos[++r - 1] = j;
    if (r > 0) {
        cell[1] = pos[0] + 1;                                  /* step 2 */
        for (int64_t k = 2; k <= r; k++) cell[pos[k - 2] + 1] = pos[k - 1] - pos[k - 2];
        for (int64_t k = 2; k <= n; k++) cell[k] += cell[k - 1];   /* step 3 */
    }
    for (int64_t c = 0; c <= n; c++) {
        int64_t k = c + 1;                                     /* paper's vertex index */
        if (r == 0 || k > pos[r - 1] || c == n)                 /* step 4 */
            out[c] = (int32_t)(n + 1);
        else
            out[c] = (int32_t)(cell[k] - 1);
    }
    free(pos); free(cell);
    return r;
}

/*
 * The combine equation of Section II-B-1, evaluated by brute force over every
 * admissible split: for a strip G whose upper part U has hU rows and lower
 * part L has hL rows,
 *     D_G(i, j) = min over k of D_L(D_U(i, k), j - k),
 * with k from max(0, j - hL) to min(j, hU).  The k = j term is the paper's
 * D_GU(i, j) and the k = 0 term its D_GL(i, j).  A D_U entry above n stands for
 * "no vertex" and makes the term unreachable.  DU is (n + 1) x (hU + 1), DL is
 * (n + 1) x (hL + 1), DG receives (n + 1) x (hU + hL + 1), all row-major.
 * If argk is not NULL it receives the smallest minimising k (-1 when the
 * entry is unreachable).
 */
int oracle_combine(const int32_t *DU, int64_t hU, const int32_t *DL, int64_t hL, int64_t n,
                   int32_t *DG, int32_t *argk)
{
    int64_t H = hU + hL;
    for (int64_t i = 0; i <= n; i++) {
        for (int64_t j = 0; j <= H; j++) {
            int64_t best = n + 1, bk = -1;
            int64_t lo = j - hL > 0 ? j - hL : 0;
            int64_t hi = j < hU ? j : hU;
            for (int64_t k = lo; k <= hi; k++) {
                int64_t x = DU[i * (hU + 1) + k];
                if (x > n) continue;
                int64_t v = DL[x * (hL + 1) + (j - k)];
                if (v <= n && v < best) { best = v; bk = k; }
            }
            DG[i * (H + 1) + j] = (int32_t)best;
            if (argk) argk[i * (H + 1) + j] = (int32_t)bk;
        }
    }
    return 0;
}

/*
 * Every vertex of the canonical path, row by row (Section II-E: the vertices
 * between two cross vertices of a row, with the reading that a horizontal run
 * ends where the path goes down or takes a match).  Builds the textbook table
 * and walks back from (m, n) with the same LEFT > DIAG > UP preference as
 * oracle_lcs_witness, all the way to (0, 0) (along row 0 or column 0 once one
 * string is used up).  For every grid row r = 0..m, col_in[r] receives the
 * smallest and col_out[r] the largest column the walk visits on that row.
 * Returns the LCS length, or -1 if the table cannot be allocated.
 */
int64_t oracle_path_rows(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                         int32_t *col_in, int32_t *col_out)
{
    size_t W = (size_t)n + 1;
    int32_t *T = calloc(((size_t)m + 1) * W, sizeof(int32_t));
    if (!T) return -1;
    for (int64_t i = 1; i <= m; i++) {
        for (int64_t j = 1; j <= n; j++) {
            int32_t v;
            if (a[i - 1] == b[j - 1]) v = T[(size_t)(i - 1) * W + (size_t)(j - 1)] + 1;
            else {
                int32_t up = T[(size_t)(i - 1) * W + (size_t)j];
                int32_t left = T[(size_t)i * W + (size_t)(j - 1)];
                v = up > left ? up : left;
            }
            T[(size_t)i * W + (size_t)j] = v;
        }
    }
    for (int64_t r = 0; r <= m; r++) { col_in[r] = (int32_t)(n + 1); col_out[r] = -1; }
    int64_t i = m, j = n;
    for (;;) {
        if (j < col_in[i]) col_in[i] = (int32_t)j;
        if (j > col_out[i]) col_out[i] = (int32_t)j;
        if (i == 0 && j == 0) break;
        int32_t c = T[(size_t)i * W + (size_t)j];
        if (j > 0 && T[(size_t)i * W + (size_t)(j - 1)] == c) {
            j--;                                   /* LEFT */
        } else if (i > 0 && j > 0 && a[i - 1] == b[j - 1]) {
            i--; j--;                              /* DIAG: a match */
        } else {
            i--;                                   /* UP */
        }
    }
    int64_t L = T[(size_t)m * W + (size_t)n];
    free(T);
    return L;
}
