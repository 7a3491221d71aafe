// Device building blocks of the LCS hot path for gfx950 (CDNA4, wave64).
//
// Each routine is the body of ONE 256-thread work-group and takes plain
// pointers, so the per-level kernels (lcs_kernels.hip) and the persistent
// batch kernel (lcs_batch.hip) run the same code.
//
// Value conventions: vertex columns 0..n, INF = n + 1 ("unreachable"), every
// breakout matrix has an all-INF sentinel row n + 1 (see lcs_geom.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lcs_geom.h"

namespace lcs {

constexpr int kBlock = 256;  // threads per work-group for every task
constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr int kJChunk = 32;  // weights per bracket block (a block may take kJChunk + 1)
constexpr int kBatch = 4;    // candidates whose loads are issued together
constexpr int kMaxTile = 32;

__host__ __device__ __forceinline__ int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }
__host__ __device__ __forceinline__ int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }
// min of two values read as unsigned: a stray negative value can never win,
// so a row index stays inside [0, bound] even if its input were corrupt
__device__ __forceinline__ int32_t umin(int32_t a, int32_t b) {
    return (int32_t)((uint32_t)a < (uint32_t)b ? (uint32_t)a : (uint32_t)b);
}

// ---------------------------------------------------------------------------
// Wave-level inclusive suffix minimum: lane l receives min(v[l..63]).
// Within each row of 16 lanes DPP row_shl:1,2,4,8 pulls values from higher
// lanes; the row totals (held by lanes 16, 32, 48) are then folded in with
// readlane.  Lanes whose DPP source lies outside the row are masked by lane id,
// so the result does not depend on the out-of-row DPP fill value.
__device__ __forceinline__ int32_t wave_suffix_min(int32_t v) {
    const int lane = __lane_id();
    const int rl = lane & 15;
    int32_t t;
    t = __builtin_amdgcn_mov_dpp(v, 0x101, 0xF, 0xF, false);  // row_shl:1
    if (rl < 15) v = imin(v, t);
    t = __builtin_amdgcn_mov_dpp(v, 0x102, 0xF, 0xF, false);  // row_shl:2
    if (rl < 14) v = imin(v, t);
    t = __builtin_amdgcn_mov_dpp(v, 0x104, 0xF, 0xF, false);  // row_shl:4
    if (rl < 12) v = imin(v, t);
    t = __builtin_amdgcn_mov_dpp(v, 0x108, 0xF, 0xF, false);  // row_shl:8
    if (rl < 8) v = imin(v, t);
    const int32_t r1 = __builtin_amdgcn_readlane(v, 16);
    const int32_t r2 = __builtin_amdgcn_readlane(v, 32);
    const int32_t r3 = __builtin_amdgcn_readlane(v, 48);
    if (lane < 48) v = imin(v, r3);
    if (lane < 32) v = imin(v, r2);
    if (lane < 16) v = imin(v, r1);
    return v;
}

// ---------------------------------------------------------------------------
// Next-match table of one symbol x (the base case of Section II-B-3 for every
// row whose symbol is x): nm[c] = 1 + (first t >= c with b[t] == x), or INF,
// for c = 0..n+1.  Row r of a base strip needs only the table of a[r], so
// sigma tables serve all m rows.  Each thread scans a run of columns, a
// block-wide suffix minimum (wave DPP scan + LDS across waves) carries the
// first match of the runs to its right, then each run is written right to
// left.  lds: kWaves int32.
__device__ void nextmatch_block(const uint8_t *__restrict__ b, int32_t n, int32_t x,
                                int32_t *__restrict__ nm, int32_t *lds) {
    const int32_t INF = n + 1;
    const int32_t total = n + 2;
    const int32_t R = (total + kBlock - 1) / kBlock;
    const int32_t c0 = (int32_t)threadIdx.x * R;
    const int32_t c1 = imin(c0 + R, total);
    int32_t first = INF;
    for (int32_t c = c0; c < c1 && c < n; ++c) {
        if (b[c] == x) {
            first = c + 1;
            break;
        }
    }
    const int32_t incl = wave_suffix_min(first);
    int32_t nxt = __shfl_down(incl, 1, kWave);
    const int lane = __lane_id();
    const int w = threadIdx.x / kWave;
    if (lane == 0) lds[w] = incl;
    __syncthreads();
    int32_t carry = (lane < kWave - 1) ? nxt : INF;
    for (int w2 = w + 1; w2 < kWaves; ++w2) carry = imin(carry, lds[w2]);
    int32_t cur = carry;
    for (int32_t c = c1 - 1; c >= c0; --c) {
        if (c < n && b[c] == x) cur = c + 1;
        nm[c] = cur;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// One base strip of h <= H0 rows, 256 consecutive top vertices v0..v0+255
// (vertex n + 1 is the sentinel row).  Each lane keeps the breakout row D(i, .)
// of its vertex in registers and appends the strip's rows one at a time: a
// row append is the combine equation with a one-row lower strip, whose D is
// the next-match table of that row's symbol, so
//     D'(i, j) = min(D(i, j), nm_{a[r]}[D(i, j - 1)])        (j = r+1 .. 1).
// The finished rows go through LDS so the store to HBM is contiguous: rows
// v..v+63 of a strip matrix are adjacent in memory.  The waves take turns on
// one 64-row buffer, and all 256 threads copy each turn out.
// lds: kWave*(H0+1) int32.
template <int H0>
__device__ void base_strip_block(const uint8_t *__restrict__ arow, int32_t h, int32_t n,
                                 int32_t sigma, const int32_t *__restrict__ nm,
                                 int32_t *__restrict__ out, int32_t v0, int32_t *err,
                                 int32_t *lds) {
    const int32_t INF = n + 1;
    const int lane = __lane_id();
    const int w = threadIdx.x / kWave;
    const int32_t i = v0 + (int32_t)threadIdx.x;
    int32_t D[H0 + 1];
    D[0] = (i <= n) ? i : INF;
#pragma unroll
    for (int j = 1; j <= H0; ++j) D[j] = INF;
    bool bad = false;
#pragma unroll
    for (int r = 0; r < H0; ++r) {
        if (r < h) {
            const int32_t x = arow[r];
            if (x < sigma) {
                const int32_t *__restrict__ nmx = nm + (size_t)x * (size_t)(n + 2);
#pragma unroll
                for (int j = r + 1; j >= 1; --j) D[j] = umin(D[j], nmx[D[j - 1]]);
            } else {
                bad = true;
            }
        }
    }
    if (bad && threadIdx.x == 0) atomicOr(err, kErrSymbol);
    const int32_t hp1 = h + 1;
    for (int w2 = 0; w2 < kWaves; ++w2) {
        if (w == w2) {
#pragma unroll
            for (int j = 0; j <= H0; ++j) lds[lane * (H0 + 1) + j] = D[j];
        }
        __syncthreads();
        const int32_t wv0 = v0 + w2 * kWave;
        const int32_t nrows = imin(kWave, n + 2 - wv0);
        if (nrows > 0) {
            int32_t *dst = out + (size_t)wv0 * (size_t)hp1;
            if (h == H0) {
                for (int32_t e = threadIdx.x; e < nrows * (H0 + 1); e += kBlock) dst[e] = lds[e];
            } else {
                for (int32_t e = threadIdx.x; e < nrows * hp1; e += kBlock) {
                    const int32_t rr = e / hp1;
                    dst[e] = lds[rr * (H0 + 1) + (e - rr * hp1)];
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Candidate scan of the combine equation for one output (vertex row urow of
// D_U, weight j): candidates k = k0, k0+step, ... in increasing order, value
// D_L(D_U(i, k), j - k).  Every k with max(0, j-hL) <= k <= min(j, hU) is a
// term of the equation, so a value of ANY such candidate is >= the true
// minimum, and no candidate below the smallest minimising k reaches it.
// Hence a batch may evaluate candidates outside the search window freely:
// taking the first strict minimum over the batch keeps the exact value and
// the smallest argmin.  The search-window tests only decide whether the scan
// may stop, and each of them is monotone in k:
//   k > hi;  x = D_U(i, k) > xb (crossings right of the bracket);
//   x - k >= best - j (then D_L(x, w) >= x + w > best for every later k);
//   best == vlo, a proven lower bound of the result.
// So they are tested once, on the last candidate of the batch.  The batch has
// no branches: indices are clamped into the window (the loads stay in bounds,
// a row x = n + 1 is the all-unreachable sentinel row) and results selected.
// Returns true when the scan is finished; otherwise it resumes at
// k0 + kBatch * step.  best starts at n + 2 ("nothing yet").
__device__ __forceinline__ bool scan_batch(const int32_t *__restrict__ urow,
                                           const int32_t *__restrict__ L, int32_t ldL, int32_t j,
                                           int32_t k0, int32_t step, int32_t hi, int32_t xb,
                                           int32_t vlo, int32_t n, int32_t &best, int32_t &bk,
                                           int32_t &bx) {
    int32_t xs[kBatch], vs[kBatch];
#pragma unroll
    for (int t = 0; t < kBatch; ++t) xs[t] = umin(urow[imin(k0 + t * step, hi)], n + 1);
#pragma unroll
    for (int t = 0; t < kBatch; ++t) {
        const int32_t kc = imin(k0 + t * step, hi);
        const int32_t v = L[(uint32_t)xs[t] * (uint32_t)ldL + (uint32_t)(j - kc)];
        vs[t] = (k0 + t * step <= hi) ? v : 0x7fffffff;
    }
#pragma unroll
    for (int t = 0; t < kBatch; ++t) {
        const bool upd = vs[t] < best;
        best = upd ? vs[t] : best;
        bk = upd ? k0 + t * step : bk;
        bx = upd ? xs[t] : bx;
    }
    const int32_t klast = k0 + (kBatch - 1) * step;
    const int32_t xl = xs[kBatch - 1];
    return (klast >= hi) | (xl > xb) | (best == vlo) | ((best <= n) & (xl - klast >= best - j));
}

// Whole scan over [lo, hi] with stride step (loop of batches).
__device__ __forceinline__ void scan_candidates(const int32_t *__restrict__ urow,
                                                const int32_t *__restrict__ L, int32_t ldL,
                                                int32_t j, int32_t lo, int32_t hi, int32_t step,
                                                int32_t xb, int32_t vlo, int32_t n, int32_t &best,
                                                int32_t &bk, int32_t &bx) {
    best = n + 2;
    bk = -1;
    bx = n + 1;
    if (lo <= hi)
        for (int32_t k0 = lo;; k0 += kBatch * step)
            if (scan_batch(urow, L, ldL, j, k0, step, hi, xb, vlo, n, best, bk, bx)) break;
    if (best > n) {
        best = n + 1;
        bk = -1;
        bx = n + 1;
    }
}

// ---------------------------------------------------------------------------
// Combine, anchor vertex (Alg. 1 with Alg. 2's tie rule).  For the vertex
// `vtx` of parent G = U (+) L, every column j of D_G(vtx, .) is
//     min over k of D_L(D_U(vtx, k), j - k),  max(0, j-hL) <= k <= min(j, hU)
// (the combine equation of Section II-B-1; k = j and k = 0 are the paper's
// D_GU and D_GL terms).  The smallest minimising k, k*(j), is non-decreasing
// in j (the monotone-matrix property of Section II-B-1), so Alg. 1's divide
// and conquer applies: a column is searched only between the argmins of the
// nearest columns already solved on its left and right, and a column whose
// minimum is unreachable makes every column to its right unreachable.
//
// GPU form: the recursion tree is walked level-synchronously over positions
// 0..P-2 (P a power of two > H): at stride s the columns s-1+2st are solved,
// bounded by columns c-s and c+s (position -1 and positions >= H are the open
// bounds 0 and hU).  Few wide columns get many threads each (strided scan +
// LDS 64-bit atomic min of (value, k), i.e. Alg. 2's minimum with the smaller
// index on ties); many narrow columns get one thread each.  A scan in
// increasing k stops early once D_U(vtx, k) - k >= best - j: since
// D_L(x, w) >= x + w, no later k can reach `best`.
// Krow (global, H entries) receives k*(j) or -1; D_G row vtx receives values.
// lds: kBlock uint64.
__device__ void anchor_block(const int32_t *__restrict__ U, int32_t hU,
                             const int32_t *__restrict__ L, int32_t hL, int32_t *__restrict__ G,
                             int32_t n, int32_t vtx, int32_t *__restrict__ Krow,
                             unsigned long long *lds) {
    const int32_t INF = n + 1;
    const int32_t H = hU + hL + 1;
    int32_t P = 1;
    while (P < H + 1) P <<= 1;
    const int32_t *__restrict__ urow = U + (size_t)vtx * (size_t)(hU + 1);
    int32_t *__restrict__ grow = G + (size_t)vtx * (size_t)H;
    const int32_t ldL = hL + 1;
    for (int32_t s = P >> 1; s >= 1; s >>= 1) {
        const int32_t ncols = (H - s) >= 0 ? imin((H - s) / (2 * s) + 1, P / (2 * s)) : 0;
        int32_t g = 1;  // threads per column (power of two), all columns in one pass
        while (2 * g <= kBlock && 2 * g * ncols <= kBlock) g <<= 1;
        const int32_t cpp = kBlock / g;  // columns per pass
        const int32_t gl = (int32_t)threadIdx.x & (g - 1);
        const int32_t slot = (int32_t)threadIdx.x / g;
        for (int32_t base = 0; base < ncols; base += cpp) {
            const int32_t t = base + slot;
            const bool act = t < ncols;
            const int32_t c = s - 1 + t * 2 * s;
            unsigned long long key = ~0ull;
            bool dead = false;
            if (act) {
                const int32_t cl = c - s, cr = c + s;
                int32_t kl = 0, kr = hU;
                if (cl >= 0) {
                    kl = Krow[cl];
                    if (kl < 0) dead = true;
                }
                if (cr < H) {
                    const int32_t t2 = Krow[cr];
                    if (t2 >= 0) kr = t2;
                }
                if (!dead) {
                    const int32_t lo = imax(kl, imax(c - hL, 0));
                    const int32_t hi = imin(kr, imin(c, hU));
                    int32_t best, bk, bx;
                    scan_candidates(urow, L, ldL, c, lo + gl, hi, g, n, -1, n, best, bk, bx);
                    if (best <= n) key = ((unsigned long long)(uint32_t)best << 32) | (uint32_t)bk;
                }
            }
            if (g > 1) {
                if (gl == 0) lds[slot] = ~0ull;
                __syncthreads();
                if (act && !dead && key != ~0ull) atomicMin(&lds[slot], key);
                __syncthreads();
                if (act && gl == 0) key = dead ? ~0ull : lds[slot];
                __syncthreads();
            }
            if (act && gl == 0) {
                if (key == ~0ull) {
                    Krow[c] = -1;
                    grow[c] = INF;
                } else {
                    Krow[c] = (int32_t)(uint32_t)(key & 0xffffffffull);
                    grow[c] = (int32_t)(key >> 32);
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Combine, bracketed vertices.  Between two solved vertices ia < ib the
// leftmost optimal paths do not cross, so for every weight j the crossing
// column x*(i, j) = D_U(i, k*(i, j)) of a vertex ia < i < ib lies in
// [x*(ia, j), x*(ib, j)].  Because D(i + d, k) <= D(i, k + d) (rows of a
// breakout matrix interlace), that confines k*(i, j) to
// [k*(ia, j) - (i - ia), k*(ib, j) + (ib - i)]; candidates whose D_U value lies
// outside the crossing interval are skipped without touching D_L.  Three exits
// cut the scan: D_G(i, j) >= D_G(ia, j), so reaching that value ends it; the
// D_L(x, w) >= x + w bound of the anchor search; and x leaving the interval.
// If D_G(ia, j) is unreachable so is D_G(i, j); if only D_G(ib, j) is, the
// upper bound falls back to min(j, hU).
//
// One block solves tile vertices i0..i0+len (both ends already solved) for
// weights j0..j0+jn-1, bisecting the tile (vertex len/2 first, then the
// quarter points, ...).  Per-vertex state (k*, x*, value) for the block's
// weights lives in LDS; values reach D_G in contiguous row segments.
// SIMD efficiency: within a bisection level every output first runs exactly
// one batch of candidates; the few that are not finished are queued in LDS and
// completed by all threads together, so a wave never waits for its slowest lane
// during the common case.
struct BracketSmem {
    int32_t k[(kMaxTile + 1) * (kJChunk + 1)];
    int32_t x[(kMaxTile + 1) * (kJChunk + 1)];
    int32_t v[(kMaxTile + 1) * (kJChunk + 1)];
    int32_t nk[(kMaxTile + 1) * (kJChunk + 1)];  // resume point of a queued output
    int32_t q[(kMaxTile + 1) * (kJChunk + 1)];   // queued outputs (slot * S + jj)
    int32_t qn;
};

struct BracketWindow {
    int32_t lo, hi, xb, vlo;
    bool dead;
};

__device__ __forceinline__ BracketWindow bracket_window(const BracketSmem &sm, int32_t v,
                                                        int32_t va, int32_t vb, int32_t jj,
                                                        int32_t j, int32_t hU, int32_t hL,
                                                        int32_t n) {
    constexpr int32_t S = kJChunk + 1;
    BracketWindow w;
    const int32_t ka = sm.k[va * S + jj];
    const int32_t kb = sm.k[vb * S + jj];
    w.dead = ka < 0;
    w.hi = imin(j, hU);
    w.xb = n;
    if (kb >= 0) {
        w.hi = imin(kb + (vb - v), w.hi);
        w.xb = sm.x[vb * S + jj];
    }
    w.lo = imax(ka - (v - va), imax(j - hL, 0));
    w.vlo = sm.v[va * S + jj];
    return w;
}

__device__ void bracket_block(const int32_t *__restrict__ U, int32_t hU,
                              const int32_t *__restrict__ L, int32_t hL, int32_t *__restrict__ G,
                              int32_t n, int32_t i0, int32_t len, int32_t j0, int32_t jn,
                              const int32_t *__restrict__ Ka, const int32_t *__restrict__ Kb,
                              BracketSmem &sm) {
    if (len < 2 || jn <= 0) return;
    constexpr int32_t S = kJChunk + 1;  // LDS row stride (weights); item slots per vertex
    const int32_t INF = n + 1;
    const int32_t H = hU + hL + 1;
    const int32_t ldU = hU + 1, ldL = hL + 1;
    const int32_t lane = __lane_id();
    // the two solved ends of the tile
    for (int32_t side = 0; side < 2; ++side) {
        const int32_t slot = side ? len : 0;
        const int32_t vert = i0 + slot;
        const int32_t *K = side ? Kb : Ka;
        for (int32_t jj = threadIdx.x; jj < jn; jj += kBlock) {
            const int32_t k = K[j0 + jj];
            sm.k[slot * S + jj] = k;
            sm.v[slot * S + jj] = G[(size_t)vert * H + j0 + jj];
            sm.x[slot * S + jj] = (k >= 0) ? U[(size_t)vert * ldU + k] : INF;
        }
    }
    if (threadIdx.x == 0) sm.qn = 0;
    __syncthreads();
    int32_t P2 = 1;
    while (P2 < len) P2 <<= 1;
    for (int32_t st = P2; st >= 2; st >>= 1) {
        const int32_t half = st >> 1;
        const int32_t nv = (len > half) ? (len - half + st - 1) / st : 0;
        // pass 1: one batch per output; item e -> (vertex t, weight jj)
        const int32_t nitems = nv * S;
        for (int32_t base = 0; base < nitems; base += kBlock) {
            const int32_t e = base + threadIdx.x;
            const int32_t t = e / S, jj = e - t * S;
            const int32_t v = half + t * st;
            const bool act = (e < nitems) && (jj < jn);
            bool queued = false;
            if (act) {
                const int32_t va = v - half, vb = imin(v + half, len);
                const int32_t j = j0 + jj;
                const BracketWindow w = bracket_window(sm, v, va, vb, jj, j, hU, hL, n);
                int32_t best = n + 2, bk = -1, bx = INF;
                bool done = w.dead || w.lo > w.hi;
                if (!done)
                    done = scan_batch(U + (size_t)(i0 + v) * ldU, L, ldL, j, w.lo, 1, w.hi, w.xb,
                                      w.vlo, n, best, bk, bx);
                const int32_t id = v * S + jj;
                sm.k[id] = bk;
                sm.x[id] = bx;
                sm.v[id] = best;
                sm.nk[id] = w.lo + kBatch;
                queued = !done;
            }
            // reserve queue slots with one LDS atomic per wave
            const unsigned long long mask = __ballot(queued);
            if (mask) {
                const int32_t leader = __ffsll((long long)mask) - 1;
                int32_t qbase = 0;
                if (lane == leader) qbase = atomicAdd(&sm.qn, __popcll(mask));
                qbase = __shfl(qbase, leader, kWave);
                if (queued) {
                    const unsigned long long below = mask & ((1ull << lane) - 1ull);
                    sm.q[qbase + __popcll(below)] = v * S + jj;
                }
            }
        }
        __syncthreads();
        // pass 2: the queued outputs, one per thread
        const int32_t qn = sm.qn;
        for (int32_t e = threadIdx.x; e < qn; e += kBlock) {
            const int32_t id = sm.q[e];
            const int32_t v = id / S, jj = id - v * S;
            const int32_t va = v - half, vb = imin(v + half, len);
            const int32_t j = j0 + jj;
            const BracketWindow w = bracket_window(sm, v, va, vb, jj, j, hU, hL, n);
            const int32_t *__restrict__ urow = U + (size_t)(i0 + v) * ldU;
            int32_t best = sm.v[id], bk = sm.k[id], bx = sm.x[id];
            for (int32_t k0 = sm.nk[id];; k0 += kBatch)
                if (scan_batch(urow, L, ldL, j, k0, 1, w.hi, w.xb, w.vlo, n, best, bk, bx)) break;
            sm.k[id] = bk;
            sm.x[id] = bx;
            sm.v[id] = best;
        }
        __syncthreads();
        // normalise unreachable results
        for (int32_t e = threadIdx.x; e < nitems; e += kBlock) {
            const int32_t t = e / S, jj = e - t * S;
            const int32_t id = (half + t * st) * S + jj;
            if (jj < jn && sm.v[id] > n) {
                sm.v[id] = INF;
                sm.k[id] = -1;
                sm.x[id] = INF;
            }
        }
        if (threadIdx.x == 0) sm.qn = 0;
        __syncthreads();
    }
    for (int32_t e = threadIdx.x; e < (len - 1) * S; e += kBlock) {
        const int32_t t = 1 + e / S, jj = e - (t - 1) * S;
        if (jj < jn) G[(size_t)(i0 + t) * H + j0 + jj] = sm.v[t * S + jj];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Length (Sections II-B-1, II-C): L = max{ j : D_top(0, j) <= n } and the end
// column y = D_top(0, L).  Finite entries of a row form a prefix, so L is the
// number of finite entries of row 0 minus one.  Writes hdr[1] = L,
// hdr[2] = y and the root trace node (0, L, y, 0).  lds: 1 int32.
__device__ void length_block(const int32_t *__restrict__ top, int32_t m, int32_t n,
                             int32_t *hdr, int4 *root, int32_t *lds) {
    if (threadIdx.x == 0) lds[0] = 0;
    __syncthreads();
    int32_t cnt = 0;
    for (int32_t j = threadIdx.x; j <= m; j += kBlock) cnt += (top[j] <= n) ? 1 : 0;
    atomicAdd(lds, cnt);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t L = imax(lds[0] - 1, 0);
        const int32_t y = top[L];
        hdr[1] = L;
        hdr[2] = y;
        *root = make_int4(0, L, y, 0);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Midpoint trace, one split (Section II-D).  Node (source s, weight w, end e)
// of G = U (+) L, with e = D_G(s, w).  The cross vertex on the boundary row is
// x = D_U(s, k*) for the SMALLEST k with D_L(D_U(s, k), w - k) == e (Alg. 2's
// tie rule), which is the leftmost crossing of any optimal path.  Children:
// (s, k*, x) in U and (x, w - k*, e) in L; the witness offset of the L child
// grows by k*, the number of matches above the boundary.  lds: 1 int32.
__device__ void trace_split_block(const int32_t *__restrict__ U, int32_t hU,
                                  const int32_t *__restrict__ L, int32_t hL, int32_t n, int4 node,
                                  int4 *outU, int4 *outL, int32_t *err, int32_t *lds) {
    const int32_t s = umin(node.x, n), w = node.y, e = node.z, off = node.w;
    const int32_t lo = imax(0, w - hL), hi = imin(w, hU);
    const int32_t *__restrict__ urow = U + (size_t)s * (hU + 1);
    const int32_t ldL = hL + 1;
    if (threadIdx.x == 0) lds[0] = 0x7fffffff;
    __syncthreads();
    int32_t found = 0x7fffffff;
    for (int32_t base = lo; base <= hi; base += kBlock) {
        const int32_t k = base + (int32_t)threadIdx.x;
        if (k <= hi) {
            const int32_t x = urow[k];
            if ((uint32_t)x <= (uint32_t)n && L[(size_t)x * ldL + (w - k)] == e) atomicMin(lds, k);
        }
        __syncthreads();
        found = lds[0];
        __syncthreads();
        if (found != 0x7fffffff) break;
    }
    if (threadIdx.x == 0) {
        if (found == 0x7fffffff) {
            atomicOr(err, kErrTrace);
            *outU = make_int4(s, 0, s, off);
            *outL = make_int4(s, 0, s, off);
        } else {
            const int32_t x = umin(urow[found], n);
            *outU = make_int4(s, found, x, off);
            *outL = make_int4(x, w - found, e, off + found);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Midpoint trace inside a base strip of h <= H0 rows.  The breakout rows of
// the single source s after each appended row, D_r(s, .) for r = 0..h, are
// recomputed into LDS; the walk then goes back from (h, w, e): at row r the
// split with the smaller upper weight is the one where row r-1 contributes a
// match, taken when nm_{a[r-1]}[D_{r-1}(s, w-1)] == e (match (row0 + r - 1,
// e - 1)); otherwise the path enters row r at the same column.  Matches are
// written at witness offsets off .. off + w - 1 in increasing order; wcap
// (= min(m, n)) bounds every write.
// lds: (H0+1)*(H0+1) int32.
template <int H0>
__device__ void trace_leaf_block(const uint8_t *__restrict__ arow, int32_t h, int32_t n,
                                 int32_t sigma, const int32_t *__restrict__ nm, int4 node,
                                 int32_t row0, int32_t *__restrict__ a_idx,
                                 int32_t *__restrict__ b_idx, int32_t wcap, int32_t *err,
                                 int32_t *lds) {
    const int32_t INF = n + 1;
    const int32_t s = umin(node.x, n);
    const int32_t S = H0 + 1;
    const int32_t tid = threadIdx.x;
    if (tid <= h) lds[tid] = (tid == 0) ? s : INF;
    __syncthreads();
    for (int32_t r = 0; r < h; ++r) {
        const int32_t x = arow[r];
        if (tid <= h) {
            int32_t d = lds[r * S + tid];
            if (tid >= 1 && x < sigma) d = umin(d, nm[(size_t)x * (n + 2) + lds[r * S + tid - 1]]);
            lds[(r + 1) * S + tid] = d;
        }
        __syncthreads();
    }
    if (tid == 0) {
        int32_t w = imin(imax(node.y, 0), h), e = node.z;
        const int32_t off = imax(node.w, 0);
        for (int32_t r = h; r >= 1; --r) {
            const int32_t x = arow[r - 1];
            if (w >= 1 && x < sigma) {
                const int32_t p = lds[(r - 1) * S + (w - 1)];
                if (p <= n && nm[(size_t)x * (n + 2) + p] == e) {
                    if (off + w <= wcap) {
                        a_idx[off + w - 1] = row0 + r - 1;
                        b_idx[off + w - 1] = e - 1;
                    }
                    e = p;
                    --w;
                }
            }
        }
        if (w != 0 || e != s) atomicOr(err, kErrTrace);
    }
    __syncthreads();
}

}  // namespace lcs
