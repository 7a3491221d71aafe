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
constexpr int kBatch = 8;    // candidates whose loads are issued together
constexpr int kAnchorEval = 8;  // anchor search: candidates per thread per depth
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
// left.  The work-group of symbol 0 also checks every symbol of b against the
// alphabet (a symbol >= sigma sets kErrSymbol in *err).  lds: kWaves int32.
__device__ void nextmatch_block(const uint8_t *__restrict__ b, int32_t n, int32_t x, int32_t sigma,
                                int32_t *__restrict__ nm, int32_t *lds, int32_t *err) {
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
    bool bad = false;
    for (int32_t c = c1 - 1; c >= c0; --c) {
        if (c < n) {
            const int32_t y = b[c];
            if (y == x) cur = c + 1;
            bad |= y >= sigma;
        }
        nm[c] = cur;
    }
    if (__syncthreads_or(bad && x == 0) && threadIdx.x == 0) atomicOr(err, kErrSymbol);
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
//
// Table window: the ~h^2/2 lookups per vertex are gathers, and served by the
// vector memory path they cost ~16 cycles per wave instruction; from LDS they
// cost a few.  The work-group copies columns v0 .. v0+T-1 of every symbol's
// table into LDS as uint16 values relative to v0 (entry T of each symbol is a
// marker above every value), keeps D relative to v0, and clamps lookup
// indices to T.  A clamped lookup stands for a table value above T (the next
// match after column c is > c), so by induction over the rows every computed
// entry <= T is exact and every exact entry <= T is computed; only entries > T
// can be wrong.  Hence the result is exact when the window reaches the
// sentinel column n + 1, or when no entry ends above T; in the remaining case
// the work-group recomputes the strip from the global tables.
// The window is for small alphabets: for random strings the matches of a
// strip's rows lie about H0 * sigma columns past the vertex, so a large
// alphabet needs a window sigma times wider per symbol, and there the global
// tables are read directly.  (A one-byte table of gaps to the next match,
// which fits alphabet 20, measured no faster than the global tables on the
// 16384 x 16384 alphabet-20 pair: 2.72 vs 2.65 ms.)
// smem: base_smem_bytes<H0, kMode>() bytes, shared by the table and, once
// the rows are done, the 64-row transposition buffer (kWave*(H0+1) int32).
constexpr int32_t kBaseTab16 = 8192;   // table entries at most
constexpr int32_t kBaseTabCap = 2047;  // at most this many columns per symbol
template <int H0>
struct BaseSmem {
    static constexpr int32_t kTrans = kWave * (H0 + 1) * 4;  // transposition buffer
    static constexpr int32_t kTab = 2 * kBaseTab16;
    static constexpr int32_t kBytes = kTab > kTrans ? kTab : kTrans;
};

// Table form of a base-strip launch: global tables or the uint16 window
// (host and device; the launcher picks the kernel instance with it).
constexpr int32_t kBaseGlobal = 0, kBaseTab16Mode = 1;
__host__ __device__ inline int32_t base_tab_cols(int32_t sigma) {
    return imin(kBaseTab16 / sigma - 1, kBaseTabCap);
}
template <int H0>
__host__ __device__ inline int32_t base_tab_mode(int32_t n, int32_t sigma) {
    if (n + 2 > 65535 || sigma < 1) return kBaseGlobal;
    return (kBlock + 2 * H0 * sigma <= base_tab_cols(sigma)) ? kBaseTab16Mode : kBaseGlobal;
}
// bytes of LDS a base-strip work-group of this table form takes
template <int H0, int kMode>
constexpr int32_t base_smem_bytes() {
    return kMode == kBaseTab16Mode ? BaseSmem<H0>::kBytes : BaseSmem<H0>::kTrans;
}

// Appends the strip's rows to D: look(x, d) is the next-match table of
// symbol x at column d (the candidate for the entry to its right).
template <int H0, class Look>
__device__ __forceinline__ bool base_append_rows(const uint8_t *__restrict__ arow, int32_t h,
                                                 int32_t sigma, int32_t (&D)[H0 + 1], Look look) {
    bool bad = false;
#pragma unroll
    for (int r = 0; r < H0; ++r) {
        if (r < h) {
            const int32_t x = arow[r];
            if (x < sigma) {
#pragma unroll
                for (int j = r + 1; j >= 1; --j) D[j] = umin(D[j], look(x, D[j - 1]));
            } else {
                bad = true;
            }
        }
    }
    return bad;
}

template <int H0, int kMode = kBaseGlobal>
__device__ void base_strip_block(const uint8_t *__restrict__ arow, int32_t h, int32_t n,
                                 int32_t sigma, const int32_t *__restrict__ nm,
                                 int32_t *__restrict__ out, int32_t v0, int32_t *err,
                                 int32_t *lds, uint8_t *smem = nullptr) {
    const int32_t INF = n + 1;
    const int lane = __lane_id();
    const int w = threadIdx.x / kWave;
    const int32_t i = v0 + (int32_t)threadIdx.x;
    const size_t ldn = (size_t)(n + 2);
    int32_t D[H0 + 1];
    bool bad = false;
    bool done = false;
    // (the launcher checked n + 2 <= 65535; testing it again at run time
    // measurably keeps the register allocation of this path small)
    if (kMode == kBaseTab16Mode && n + 2 <= 65535) {
        const int32_t T = imin(n + 2 - v0, base_tab_cols(sigma));
        const int32_t ts = T + 1;  // per-symbol stride
        uint16_t *tab = reinterpret_cast<uint16_t *>(smem);
        for (int32_t x = 0; x < sigma; ++x) {  // 8 loads in flight per thread
            const int32_t *src = nm + (size_t)x * ldn + v0;
            for (int32_t c0 = threadIdx.x; c0 < ts; c0 += 8 * kBlock) {
                int32_t nv[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) nv[t] = src[imin(c0 + t * kBlock, T - 1)];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int32_t c = c0 + t * kBlock;
                    if (c < ts) tab[x * ts + c] = (c < T) ? (uint16_t)(nv[t] - v0) : (uint16_t)0xFFFF;
                }
            }
        }
        __syncthreads();
        D[0] = (i <= n) ? (int32_t)threadIdx.x : INF - v0;
#pragma unroll
        for (int j = 1; j <= H0; ++j) D[j] = INF - v0;
        bad = base_append_rows<H0>(arow, h, sigma, D, [&](int32_t x, int32_t d) {
            return (int32_t)tab[x * ts + umin(d, T)];
        });
        bool unsure = false;
        if (v0 + T < n + 1) {
#pragma unroll
            for (int j = 0; j <= H0; ++j) unsure |= D[j] > T;
        }
        done = !__syncthreads_or(unsure);
        if (done) {
#pragma unroll
            for (int j = 0; j <= H0; ++j) D[j] += v0;
        }
    }
    if (!done) {
        D[0] = (i <= n) ? i : INF;
#pragma unroll
        for (int j = 1; j <= H0; ++j) D[j] = INF;
        bad = base_append_rows<H0>(arow, h, sigma, D, [&](int32_t x, int32_t d) {
            return nm[(size_t)x * ldn + (size_t)d];
        });
    }
    if (bad && threadIdx.x == 0) atomicOr(err, kErrSymbol);
    __syncthreads();  // the table (if any) is dead; its memory is the transposition buffer
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
// Base strips from a combed seaweed permutation.  The breakout rows of a
// strip are a function of LCS(a[r0:r1], b[i:c]) over all i <= c, and that
// whole family is encoded by one permutation of "seaweeds" (Tiskin's
// semi-local LCS): h seaweeds enter on the left (row r, label -(r+1)) and n
// on the top (column c, label c); in each cell the two arriving seaweeds
// turn at a match, and at a mismatch they cross unless they crossed before,
// which with these labels is exactly "the horizontal label is the larger".
// Row by row, with x the horizontal label entering column c and y the
// vertical one:
//     match:     down <- x, right <- y
//     mismatch:  down <- max(x, y), right <- min(x, y).
// Let bot[q] be the label leaving the bottom of column q.  The column where
// the j-th step of LCS(strip, b[i:c]) happens as c grows is the j-th
// smallest q + 1 with q >= i and bot[q] < i (a seaweed that started left of
// i and ends below column q), so
//     D(i, 0) = i,  D(i, j) = j-th such q + 1, n + 1 past the last,
// and there are h - #{right-side exits with label < i} of them.  From vertex
// i - 1 to i the set loses the element i (if bot[i-1] < i-1) and gains
// pos[i-1] + 1 (pos = where top seaweed i-1 ends, if below a column >= i).
// The result equals the row-append recurrence's exactly (both are D); the
// work is O(h n) combing plus O(h) per vertex instead of O(h^2) per vertex.
//
// Combing of one strip by one work-group of NT threads, C columns per thread
// per tile: the horizontal label of row r passes every column of the
// tile from left to right, so each row is a prefix scan over the threads of
// the per-column maps x -> (match ? y : min(x, y)), which compose within the
// family {x -> const v} u {x -> min(x, v)}; the tiles go left to right, the
// labels leaving a tile on the right entering the next.  Writes bot[0..n),
// pos[0..n) (n + 1 for a seaweed that leaves on the right) and right[0..h).
constexpr int32_t kCombMaxThreads = 1024;
constexpr int32_t kCombMaxRows = 1024;
constexpr int32_t kCombPackedMaxN = 32767;  // labels -h..n-1 and the padding 0x7fff fit int16
// columns per thread and threads of the combing work-group for n columns
__host__ __device__ inline int32_t comb_cols(int32_t n) {
    if (n > kCombPackedMaxN) return 16;
    int32_t c = 4;
    while (c < 32 && c * 512 < n) c *= 2;
    return c;
}
__host__ __device__ inline int32_t comb_threads(int32_t n, int32_t C) {
    const int32_t t = (n + C - 1) / C;
    const int32_t r = (t + kWave - 1) / kWave * kWave;
    return r < kWave ? kWave : (r > kCombMaxThreads ? kCombMaxThreads : r);
}

// (c, v) stands for x -> c ? v : min(x, v); b := b after a
__device__ __forceinline__ void comb_fn_after(int32_t ac, int32_t av, int32_t &bc, int32_t &bv) {
    bv = bc ? bv : imin(av, bv);
    bc |= ac;
}

// Inclusive scan of the maps over the lanes of a wave (lane l: lanes 0..l
// composed in order).  Within each row of 16 lanes DPP row_shr:1,2,4,8 pulls
// the maps of lower lanes (masked by lane id, as in wave_suffix_min; alone,
// row_fn_scan); the row totals of lanes 15, 31, 47 are folded in with
// readlane.
__device__ __forceinline__ void row_fn_scan(int32_t &c, int32_t &v) {
    const int rl = __lane_id() & 15;
    int32_t tc, tv;
    tc = __builtin_amdgcn_mov_dpp(c, 0x111, 0xF, 0xF, false);  // row_shr:1
    tv = __builtin_amdgcn_mov_dpp(v, 0x111, 0xF, 0xF, false);
    if (rl >= 1) comb_fn_after(tc, tv, c, v);
    tc = __builtin_amdgcn_mov_dpp(c, 0x112, 0xF, 0xF, false);  // row_shr:2
    tv = __builtin_amdgcn_mov_dpp(v, 0x112, 0xF, 0xF, false);
    if (rl >= 2) comb_fn_after(tc, tv, c, v);
    tc = __builtin_amdgcn_mov_dpp(c, 0x114, 0xF, 0xF, false);  // row_shr:4
    tv = __builtin_amdgcn_mov_dpp(v, 0x114, 0xF, 0xF, false);
    if (rl >= 4) comb_fn_after(tc, tv, c, v);
    tc = __builtin_amdgcn_mov_dpp(c, 0x118, 0xF, 0xF, false);  // row_shr:8
    tv = __builtin_amdgcn_mov_dpp(v, 0x118, 0xF, 0xF, false);
    if (rl >= 8) comb_fn_after(tc, tv, c, v);
}
__device__ __forceinline__ void wave_fn_scan(int32_t &c, int32_t &v) {
    const int lane = __lane_id();
    row_fn_scan(c, v);
    int32_t pc = __builtin_amdgcn_readlane(c, 15), pv = __builtin_amdgcn_readlane(v, 15);
    const int32_t r1c = __builtin_amdgcn_readlane(c, 31), r1v = __builtin_amdgcn_readlane(v, 31);
    const int32_t r2c = __builtin_amdgcn_readlane(c, 47), r2v = __builtin_amdgcn_readlane(v, 47);
    int32_t qc = r1c, qv = r1v;
    comb_fn_after(pc, pv, qc, qv);  // rows 0..1
    int32_t sc = r2c, sv = r2v;
    comb_fn_after(qc, qv, sc, sv);  // rows 0..2
    if (lane >= 48) {
        comb_fn_after(sc, sv, c, v);
    } else if (lane >= 32) {
        comb_fn_after(qc, qv, c, v);
    } else if (lane >= 16) {
        comb_fn_after(pc, pv, c, v);
    }
}

// Packed 16-bit lanes (two labels or two symbols per register).
typedef short comb_s2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_min_i16(uint32_t a, uint32_t b) {
    const comb_s2 x = __builtin_bit_cast(comb_s2, a), y = __builtin_bit_cast(comb_s2, b);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(x, y));
}
__device__ __forceinline__ uint32_t pk_max_i16(uint32_t a, uint32_t b) {
    const comb_s2 x = __builtin_bit_cast(comb_s2, a), y = __builtin_bit_cast(comb_s2, b);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, y));
}
// 0xffff in each half where the halves of a and b are equal, else 0:
// min(a ^ b, 1) - 1 per half.  Written as the packed instructions themselves
// (register operands only): as plain code the compiler splits it into
// per-half compares and re-packs, which costs more than the unpacked form.
__device__ __forceinline__ uint32_t pk_eq_mask(uint32_t a, uint32_t b) {
    const uint32_t one = 0x00010001u;
    uint32_t t, m;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(t) : "v"(a ^ b), "v"(one));
    asm("v_pk_sub_u16 %0, %1, %2" : "=v"(m) : "v"(t), "v"(one));
    return m;
}
// (m & a) | (~m & b) in one instruction
__device__ __forceinline__ uint32_t bit_select(uint32_t m, uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(m), "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ int32_t sext16(uint32_t v) { return (int32_t)(int16_t)(v & 0xffffu); }

// lds: 3 * h + 4 * (NT / kWave) int32.  kPacked (n <= 32767, so every label
// and the padding label 0x7fff fit int16): register e of a thread holds
// columns cb + e and cb + C/2 + e in its two halves, two independent chains
// whose maps compose as (high after low), so a row costs about half the
// instructions: v_pk_min/max_i16, a bit-select for the match, and a packed
// equality mask per symbol pair.
template <int NT, int C, bool kPacked>
__device__ void comb_strip_block(const uint8_t *__restrict__ arow, int32_t h,
                                 const uint8_t *__restrict__ b, int32_t n, int32_t sigma,
                                 int32_t *__restrict__ bot, int32_t *__restrict__ pos,
                                 int32_t *__restrict__ right, int32_t *lds, int32_t *err) {
    constexpr int32_t NW = NT / kWave;
    constexpr int32_t P = C / 2;
    static_assert(NW <= 16, "the wave totals are scanned by one row of 16 lanes");
    static_assert(C % 2 == 0, "packed columns come in pairs");
    const int32_t tid = threadIdx.x;
    const int32_t nthr = (int32_t)blockDim.x;  // <= NT, a multiple of kWave
    const int32_t w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int lane = __lane_id();
    int32_t *hin = lds, *hout = lds + h;                 // labels entering / leaving a tile, per row
    int32_t *xs = lds + 2 * h;                           // the strip's row symbols
    int32_t *wsc = lds + 3 * h, *wsv = wsc + 2 * NW;     // wave totals, two buffers
    bool bad = false;
    for (int32_t r = tid; r < h; r += nthr) {
        hin[r] = -(r + 1);
        xs[r] = arow[r];
        bad |= xs[r] >= sigma;
    }
    const int32_t T = nthr * C;
    for (int32_t c0 = 0; c0 < n; c0 += T) {
        int32_t v[kPacked ? 1 : C], bs[kPacked ? 1 : C];
        uint32_t v2[kPacked ? P : 1], b2[kPacked ? P : 1];
        const int32_t cb = c0 + tid * C;
        if constexpr (kPacked) {
#pragma unroll
            for (int e = 0; e < P; ++e) {
                const int32_t cl = cb + e, ch = cb + P + e;
                const uint32_t vl = (cl < n) ? (uint32_t)cl : 0x7fffu, vh = (ch < n) ? (uint32_t)ch : 0x7fffu;
                const uint32_t sl = (cl < n) ? (uint32_t)b[cl] : 0x100u, sh = (ch < n) ? (uint32_t)b[ch] : 0x100u;
                v2[e] = vl | (vh << 16);
                b2[e] = sl | (sh << 16);
            }
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e) {
                const int32_t c = cb + e;
                v[e] = (c < n) ? c : 0x7fffffff;   // a padding column maps x -> x
                bs[e] = (c < n) ? (int32_t)b[c] : 0x100;
            }
        }
        __syncthreads();  // hin of this tile written
        int32_t buf = 0;
        for (int32_t r = 0; r < h; ++r) {
            const int32_t x = xs[r];
            int32_t fc = 0, fv = 0x7fffffff;
            uint32_t m2[kPacked ? P : 1];
            int32_t clo = 0, vlo = 0;
            if constexpr (kPacked) {
                const uint32_t xx = (uint32_t)x * 0x00010001u;
                uint32_t fc2 = 0, fv2 = 0x7fff7fffu;
#pragma unroll
                for (int e = 0; e < P; ++e) {
                    m2[e] = pk_eq_mask(b2[e], xx);
                    fv2 = bit_select(m2[e], v2[e], pk_min_i16(fv2, v2[e]));
                    fc2 |= m2[e];
                }
                clo = (fc2 & 0xffffu) != 0;
                vlo = sext16(fv2);
                const int32_t chi = (fc2 >> 16) != 0, vhi = (int32_t)fv2 >> 16;
                fc = clo | chi;
                fv = chi ? vhi : imin(vlo, vhi);
            } else {
#pragma unroll
                for (int e = 0; e < C; ++e) {
                    const bool m = bs[e] == x;
                    fv = m ? v[e] : imin(fv, v[e]);
                    fc |= (int32_t)m;
                }
            }
            wave_fn_scan(fc, fv);
            if (lane == kWave - 1) {
                wsc[buf * NW + w] = fc;
                wsv[buf * NW + w] = fv;
            }
            __syncthreads();
            // the waves before w, composed: lanes 0..NW-1 scan the wave totals
            int32_t pc = 0, pv = 0x7fffffff;
            if (w > 0) {
                int32_t tc = 0, tv = 0x7fffffff;
                if (lane < NW) {
                    tc = wsc[buf * NW + lane];
                    tv = wsv[buf * NW + lane];
                }
                row_fn_scan(tc, tv);
                pc = __builtin_amdgcn_readlane(tc, w - 1);
                pv = __builtin_amdgcn_readlane(tv, w - 1);
            }
            const int32_t xin = hin[r];
            const int32_t xw = pc ? pv : imin(xin, pv);      // label entering wave w
            const int32_t xl = fc ? fv : imin(xw, fv);       // label leaving this thread
            // label entering this thread: the left neighbour's (wave_shr:1), lane 0: xw
            int32_t hh = __builtin_amdgcn_update_dpp(xw, xl, 0x138, 0xF, 0xF, false);
            if constexpr (kPacked) {
                const int32_t hhi = clo ? vlo : imin(hh, vlo);  // entering the high chain
                uint32_t h2 = ((uint32_t)hh & 0xffffu) | ((uint32_t)hhi << 16);
#pragma unroll
                for (int e = 0; e < P; ++e) {
                    const uint32_t y = v2[e];
                    const uint32_t lo = pk_min_i16(h2, y), hi = pk_max_i16(h2, y);
                    v2[e] = bit_select(m2[e], h2, hi);
                    h2 = bit_select(m2[e], y, lo);
                }
                hh = (int32_t)h2 >> 16;
            } else {
#pragma unroll
                for (int e = 0; e < C; ++e) {
                    const int32_t y = v[e];
                    const bool m = bs[e] == x;
                    v[e] = m ? hh : imax(hh, y);
                    hh = m ? y : imin(hh, y);
                }
            }
            if (tid == nthr - 1) hout[r] = hh;
            buf ^= 1;
        }
        if constexpr (kPacked) {
#pragma unroll
            for (int e = 0; e < P; ++e) {
                const int32_t cl = cb + e, ch = cb + P + e;
                const int32_t ll = sext16(v2[e]), lh = (int32_t)v2[e] >> 16;
                if (cl < n) {
                    bot[cl] = ll;
                    if (ll >= 0) pos[ll] = cl;
                }
                if (ch < n) {
                    bot[ch] = lh;
                    if (lh >= 0) pos[lh] = ch;
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e) {
                const int32_t c = cb + e;
                if (c < n) {
                    bot[c] = v[e];
                    if (v[e] >= 0) pos[v[e]] = c;
                }
            }
        }
        __syncthreads();  // hout complete, every read of hin done
        int32_t *t = hin;
        hin = hout;
        hout = t;
    }
    __syncthreads();
    for (int32_t r = tid; r < h; r += nthr) {
        const int32_t lab = hin[r];
        right[r] = lab;
        if (lab >= 0) pos[lab] = n + 1;
    }
    if (__syncthreads_or(bad) && tid == 0) atomicOr(err, kErrSymbol);
}

// Combing of one strip (n <= 32767, packed labels) as a pipeline of the
// work-group's waves instead of a block-wide scan per row: wave w owns
// columns [64 C w, 64 C (w + 1)), lane l the C columns 64 C w + C l ...
// For row r a wave first composes its own columns' maps (they depend only on
// its columns' labels and the row symbol) and scans them over its lanes; only
// then does it need the label entering its first column, which is the label
// leaving wave w - 1 in row r.  That label crosses the wave with one map
// application (no barrier, no block scan), is written to the LDS slot
// ring[w][r] (every slot starts at a sentinel no label takes) and read there
// by wave w + 1, so the row's waves run staggered by one LDS hop and the
// apply of every wave overlaps the next waves' hops.  A wait past
// kCombSpinLimit polls reports kErrTrace instead of hanging.  lds: 64 C-column
// waves K = blockDim.x / 64 <= 16; ring K x h int32, then h int32 of row
// symbols.
constexpr uint32_t kCombSpinLimit = 1u << 22;
constexpr int32_t kCombPipeWaves = 16;  // waves of a pipelined combing work-group, at most
constexpr size_t kCombPipeMaxLds = 64 * 1024;  // its dynamic LDS (ring and row symbols), at most
// Columns per lane of the pipelined combing: up to 32, so that 8 waves cover n
// (16 for n > 16384).  Each wave's row scan costs about as much as 16 packed
// columns; fewer, longer waves cut that per row (16384^2 base strips: 16 waves
// 0.83 ms, 8 waves 0.76, 4 waves of 64 columns 0.79).
__host__ __device__ inline int32_t comb_pipe_cols(int32_t n) {
    int32_t c = 4;
    while (c < 32 && (n + 64 * c - 1) / (64 * c) > kCombPipeWaves / 2) c *= 2;
    return c;
}
constexpr int32_t kCombSentinel = (int32_t)0x80000000;
template <int C>
__device__ void comb_strip_pipe(const uint8_t *__restrict__ arow, int32_t h,
                                const uint8_t *__restrict__ b, int32_t n, int32_t sigma,
                                int32_t *__restrict__ bot, int32_t *__restrict__ pos,
                                int32_t *__restrict__ right, int32_t *lds, int32_t *err) {
    constexpr int32_t P = C / 2;
    const int32_t tid = threadIdx.x;
    const int32_t nthr = (int32_t)blockDim.x;
    const int32_t K = nthr / kWave;
    const int32_t w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int lane = __lane_id();
    int32_t *ring = lds;          // ring[w * h + r]: label leaving wave w in row r
    int32_t *xs = lds + K * h;    // row symbols
    bool bad = false;
    for (int32_t i = tid; i < K * h; i += nthr) ring[i] = kCombSentinel;
    for (int32_t r = tid; r < h; r += nthr) {
        xs[r] = arow[r];
        bad |= xs[r] >= sigma;
    }
    uint32_t v2[P], b2[P];
    const int32_t cb = tid * C;
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int32_t cl = cb + e, ch = cb + P + e;
        const uint32_t vl = (cl < n) ? (uint32_t)cl : 0x7fffu, vh = (ch < n) ? (uint32_t)ch : 0x7fffu;
        const uint32_t sl = (cl < n) ? (uint32_t)b[cl] : 0x100u, sh = (ch < n) ? (uint32_t)b[ch] : 0x100u;
        v2[e] = vl | (vh << 16);
        b2[e] = sl | (sh << 16);
    }
    __syncthreads();
    bool stall = false;
    for (int32_t rb = 0; rb < h; rb += kWave) {
        const int32_t xr = xs[rb + imin(lane, h - 1 - rb)];
        const int32_t rn = imin(kWave, h - rb);
        for (int32_t rr = 0; rr < rn; ++rr) {
            const int32_t r = rb + rr;
            const uint32_t xx = (uint32_t)__builtin_amdgcn_readlane(xr, rr) * 0x00010001u;
            uint32_t m2[P];
            uint32_t fc2 = 0, fv2 = 0x7fff7fffu;
#pragma unroll
            for (int e = 0; e < P; ++e) {
                m2[e] = pk_eq_mask(b2[e], xx);
                fv2 = bit_select(m2[e], v2[e], pk_min_i16(fv2, v2[e]));
                fc2 |= m2[e];
            }
            const int32_t clo = (fc2 & 0xffffu) != 0, vlo = sext16(fv2);
            const int32_t chi = (fc2 >> 16) != 0, vhi = (int32_t)fv2 >> 16;
            int32_t fc = clo | chi, fv = chi ? vhi : imin(vlo, vhi);
            wave_fn_scan(fc, fv);  // lane l: lanes 0..l of this wave composed
            // the label entering this wave in row r
            int32_t xin = -(r + 1);
            if (w > 0) {
                const int32_t *slot = ring + (w - 1) * h + r;
                xin = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                uint32_t spins = 0;
                while (xin == kCombSentinel) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kCombSpinLimit) {
                        stall = true;
                        xin = 0;
                        break;
                    }
                    xin = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                }
            }
            const int32_t xl = fc ? fv : imin(xin, fv);  // label leaving this lane's columns
            const int32_t xout = __builtin_amdgcn_readlane(xl, kWave - 1);
            if (lane == 0)
                __hip_atomic_store(ring + w * h + r, xout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            // label entering this lane: the left neighbour's (wave_shr:1), lane 0: xin
            const int32_t hh = __builtin_amdgcn_update_dpp(xin, xl, 0x138, 0xF, 0xF, false);
            const int32_t hhi = clo ? vlo : imin(hh, vlo);  // entering the high chain
            uint32_t h2 = ((uint32_t)hh & 0xffffu) | ((uint32_t)hhi << 16);
#pragma unroll
            for (int e = 0; e < P; ++e) {
                const uint32_t y = v2[e];
                const uint32_t lo = pk_min_i16(h2, y), hi = pk_max_i16(h2, y);
                v2[e] = bit_select(m2[e], h2, hi);
                h2 = bit_select(m2[e], y, lo);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int32_t cl = cb + e, ch = cb + P + e;
        const int32_t ll = sext16(v2[e]), lh = (int32_t)v2[e] >> 16;
        if (cl < n) {
            bot[cl] = ll;
            if (ll >= 0) pos[ll] = cl;
        }
        if (ch < n) {
            bot[ch] = lh;
            if (lh >= 0) pos[lh] = ch;
        }
    }
    __syncthreads();  // every ring slot of the last wave written
    for (int32_t r = tid; r < h; r += nthr) {
        const int32_t lab = ring[(K - 1) * h + r];
        right[r] = lab;
        if (lab >= 0) pos[lab] = n + 1;
    }
    if (__syncthreads_or(bad) && tid == 0) atomicOr(err, kErrSymbol);
    if (__syncthreads_or(stall) && tid == 0) atomicOr(err, kErrTrace);
}

// One column segment of a strip combed by several work-groups: segment g
// (columns [c0, c0 + 64 C K) of n, K = blockDim.x / 64 waves, a pipeline as in
// comb_strip_pipe) takes the labels entering its first column from the
// records of segment g - 1 and gives the labels leaving its last column to
// segment g + 1.  A record is one 64-bit word, (row + 1) << 32 | label, so
// the row tag and the label become visible together (relaxed atomics at
// device scope; the records are cleared before the launch).  The first wave
// reads 64 rows' records at a time and polls again only past the last ready
// one; a wait past kCombSpinLimit polls reports kErrTrace.  The read of the
// records after a window is issued as soon as the window is taken, so its
// round trip overlaps the window's rows (a record never changes once tagged,
// so an early read is exact; rows not yet tagged then are read again): a
// segment then trails the one before it by a few rows instead of about a
// window, which is what the fill of the segment pipeline costs.  Work-group
// numbers grow with g, so every segment waits only on one dispatched before
// it.  The last segment writes right[] and the right-side entries of pos[].
// lds: K x h int32 (ring), then h int32 (row symbols).
template <int C>
__device__ void comb_strip_seg(const uint8_t *__restrict__ arow, int32_t h,
                               const uint8_t *__restrict__ b, int32_t n, int32_t sigma, int32_t c0,
                               bool first, bool last, const unsigned long long *rec_in,
                               unsigned long long *rec_out, int32_t *__restrict__ bot,
                               int32_t *__restrict__ pos, int32_t *__restrict__ right, int32_t *lds,
                               int32_t *err) {
    constexpr int32_t P = C / 2;
    const int32_t tid = threadIdx.x;
    const int32_t nthr = (int32_t)blockDim.x;
    const int32_t K = nthr / kWave;
    const int32_t w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int lane = __lane_id();
    int32_t *ring = lds;
    int32_t *xs = lds + K * h;
    bool bad = false;
    for (int32_t i = tid; i < K * h; i += nthr) ring[i] = kCombSentinel;
    for (int32_t r = tid; r < h; r += nthr) {
        xs[r] = arow[r];
        bad |= xs[r] >= sigma;
    }
    uint32_t v2[P], b2[P];
    const int32_t cb = c0 + tid * C;
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int32_t cl = cb + e, ch = cb + P + e;
        const uint32_t vl = (cl < n) ? (uint32_t)cl : 0x7fffu, vh = (ch < n) ? (uint32_t)ch : 0x7fffu;
        const uint32_t sl = (cl < n) ? (uint32_t)b[cl] : 0x100u, sh = (ch < n) ? (uint32_t)b[ch] : 0x100u;
        v2[e] = vl | (vh << 16);
        b2[e] = sl | (sh << 16);
    }
    __syncthreads();
    bool stall = false;
    int32_t rbase = 0, rready = 0;  // first wave of a later segment: records rbase .. rbase+rready-1 in rwin
    int32_t rwin = 0;
    int32_t pfb = -1;  // first row of the records read ahead into pf (-1: none)
    unsigned long long pf = 0ull;
    for (int32_t rb = 0; rb < h; rb += kWave) {
        const int32_t xr = xs[rb + imin(lane, h - 1 - rb)];
        const int32_t rn = imin(kWave, h - rb);
        for (int32_t rr = 0; rr < rn; ++rr) {
            const int32_t r = rb + rr;
            const uint32_t xx = (uint32_t)__builtin_amdgcn_readlane(xr, rr) * 0x00010001u;
            uint32_t m2[P];
            uint32_t fc2 = 0, fv2 = 0x7fff7fffu;
#pragma unroll
            for (int e = 0; e < P; ++e) {
                m2[e] = pk_eq_mask(b2[e], xx);
                fv2 = bit_select(m2[e], v2[e], pk_min_i16(fv2, v2[e]));
                fc2 |= m2[e];
            }
            const int32_t clo = (fc2 & 0xffffu) != 0, vlo = sext16(fv2);
            const int32_t chi = (fc2 >> 16) != 0, vhi = (int32_t)fv2 >> 16;
            int32_t fc = clo | chi, fv = chi ? vhi : imin(vlo, vhi);
            wave_fn_scan(fc, fv);
            int32_t xin = -(r + 1);
            if (w > 0) {
                const int32_t *slot = ring + (w - 1) * h + r;
                xin = __builtin_amdgcn_readfirstlane(
                    __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                uint32_t spins = 0;
                while (xin == kCombSentinel) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kCombSpinLimit) {
                        stall = true;
                        xin = 0;
                        break;
                    }
                    xin = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                }
            } else if (!first) {
                if (r >= rbase + rready) {  // (re)load the records from row r on
                    int32_t cnt0 = 0;
                    if (pfb == r) {  // the records read ahead
                        const bool ok = (r + lane < h) && (int32_t)(pf >> 32) == r + lane + 1;
                        const unsigned long long mk = __ballot(ok);
                        cnt0 = (~mk == 0ull) ? kWave : (int32_t)__builtin_ctzll(~mk);
                        if (cnt0 > 0) {
                            rbase = r;
                            rready = cnt0;
                            rwin = (int32_t)(uint32_t)pf;
                        }
                    }
                    uint32_t spins = 0;
                    while (cnt0 == 0) {
                        unsigned long long v = 0ull;
                        if (r + lane < h)
                            v = __hip_atomic_load(rec_in + r + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const bool ok = (r + lane < h) && (int32_t)(v >> 32) == r + lane + 1;
                        const unsigned long long mk = __ballot(ok);
                        const int32_t cnt = (~mk == 0ull) ? kWave : (int32_t)__builtin_ctzll(~mk);  // ready from r on
                        if (cnt > 0) {
                            rbase = r;
                            rready = cnt;
                            rwin = (int32_t)(uint32_t)v;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                        if (++spins > kCombSpinLimit) {
                            stall = true;
                            rbase = r;
                            rready = h;
                            rwin = 0;
                            break;
                        }
                    }
                    // read the next window's records now; they are looked at
                    // when this window is used up
                    pfb = rbase + rready;
                    pf = 0ull;
                    if (pfb < h && pfb + lane < h)
                        pf = __hip_atomic_load(rec_in + pfb + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                xin = __builtin_amdgcn_readlane(rwin, r - rbase);
            }
            const int32_t xl = fc ? fv : imin(xin, fv);
            const int32_t xout = __builtin_amdgcn_readlane(xl, kWave - 1);
            if (lane == 0) {
                if (w < K - 1 || last)
                    __hip_atomic_store(ring + w * h + r, xout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                else
                    __hip_atomic_store(rec_out + r, ((unsigned long long)(uint32_t)(r + 1) << 32) | (uint32_t)xout,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            const int32_t hh = __builtin_amdgcn_update_dpp(xin, xl, 0x138, 0xF, 0xF, false);
            const int32_t hhi = clo ? vlo : imin(hh, vlo);
            uint32_t h2 = ((uint32_t)hh & 0xffffu) | ((uint32_t)hhi << 16);
#pragma unroll
            for (int e = 0; e < P; ++e) {
                const uint32_t y = v2[e];
                const uint32_t lo = pk_min_i16(h2, y), hi = pk_max_i16(h2, y);
                v2[e] = bit_select(m2[e], h2, hi);
                h2 = bit_select(m2[e], y, lo);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < P; ++e) {
        const int32_t cl = cb + e, ch = cb + P + e;
        const int32_t ll = sext16(v2[e]), lh = (int32_t)v2[e] >> 16;
        if (cl < n) {
            bot[cl] = ll;
            if (ll >= 0) pos[ll] = cl;
        }
        if (ch < n) {
            bot[ch] = lh;
            if (lh >= 0) pos[lh] = ch;
        }
    }
    __syncthreads();
    if (last) {
        for (int32_t r = tid; r < h; r += nthr) {
            const int32_t lab = ring[(K - 1) * h + r];
            right[r] = lab;
            if (lab >= 0) pos[lab] = n + 1;
        }
    }
    if (__syncthreads_or(bad && first) && tid == 0) atomicOr(err, kErrSymbol);
    if (__syncthreads_or(stall) && tid == 0) atomicOr(err, kErrTrace);
}



// Breakout rows of vertices i0 .. i1-1 of one base strip (h rows) from its
// combing, by one wave; vertex n + 1 is the all-unreachable sentinel row.
// The wave keeps the sorted set {q + 1 : q >= i, bot[q] < i} (at most h
// values, E per lane, element 64 e + lane in register e) and moves from
// vertex to vertex by dropping the element i and inserting pos[i-1] + 1.
// The first vertex's set comes from a scan of bot[i0..].  lst: 64 E int32 of
// LDS for this wave alone.  out: the strip matrix, row length h + 1.
template <int E>
__device__ void dgen_wave(const int32_t *__restrict__ bot, const int32_t *__restrict__ pos,
                          const int32_t *__restrict__ right, int32_t h, int32_t n, int32_t i0,
                          int32_t i1, int32_t *__restrict__ out, int32_t *lst) {
    const int32_t INF = n + 1;
    const int32_t hp1 = h + 1;
    const int lane = __lane_id();
    const int32_t iend = imin(i1, n + 1);  // rows with a vertex
    int32_t L[E];
#pragma unroll
    for (int e = 0; e < E; ++e) L[e] = INF;
    if (i0 < iend) {
        int32_t below = 0;  // right-side exits with label < i0
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int32_t r = e * kWave + lane;
            below += __popcll(__ballot(r < h && right[r] < i0));
        }
        const int32_t K = h - below;
        int32_t found = 0;
        const unsigned long long lt = (1ull << lane) - 1ull;
        for (int32_t q0 = i0; found < K && q0 < n; q0 += 4 * kWave) {
            int32_t bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t q = q0 + u * kWave + lane;
                bv[u] = (q < n) ? bot[q] : 0x7fffffff;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool hit = bv[u] < i0;
                const unsigned long long mk = __ballot(hit);
                const int32_t slot = found + __popcll(mk & lt);
                if (hit && slot < E * kWave) lst[slot] = q0 + u * kWave + lane + 1;
                found += __popcll(mk);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        const int32_t cnt = imin(imin(found, K), E * kWave);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int32_t j = e * kWave + lane;
            if (j < cnt) L[e] = lst[j];
        }
    }
    int32_t pv = INF;  // pos[i - 1 ..] for the next 64 vertices, one per lane
    for (int32_t i = i0; i < iend; ++i) {
        if (i > i0) {
            const int32_t k = (i - 1 - i0) & (kWave - 1);
            if (k == 0) {
                const int32_t q = i - 1 + lane;
                pv = (q < n) ? pos[q] : INF;
            }
            const int32_t t = __builtin_amdgcn_readlane(pv, k);
            if (__builtin_amdgcn_readlane(L[0], 0) == i) {  // drop element i
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int32_t nx = (e + 1 < E) ? __builtin_amdgcn_readlane(L[e + 1 < E ? e + 1 : e], 0) : INF;
                    L[e] = __builtin_amdgcn_update_dpp(nx, L[e], 0x130, 0xF, 0xF, false);  // wave_shl:1
                }
            }
            if (t >= i && t < n) {  // insert t + 1
                const int32_t val = t + 1;
                int32_t pr[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int32_t pe = (e > 0) ? __builtin_amdgcn_readlane(L[e > 0 ? e - 1 : 0], kWave - 1) : -1;
                    pr[e] = __builtin_amdgcn_update_dpp(pe, L[e], 0x138, 0xF, 0xF, false);  // wave_shr:1
                }
#pragma unroll
                for (int e = 0; e < E; ++e) L[e] = (L[e] < val) ? L[e] : ((pr[e] < val) ? val : pr[e]);
            }
        }
        int32_t *row = out + (size_t)i * (size_t)hp1;
        if (lane == 0) row[0] = i;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int32_t j = e * kWave + lane;
            if (j < h) row[1 + j] = L[e];
        }
    }
    if (i1 == n + 2) {
        int32_t *row = out + (size_t)(n + 1) * (size_t)hp1;
        for (int32_t j = lane; j <= h; j += kWave) row[j] = INF;
    }
}

// ---------------------------------------------------------------------------
// Candidate scan of the combine equation for one output (vertex row at offset urow of
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
// k0 + kBatch * step.  best starts at n + 2 ("nothing yet").  The three
// phases (D_U loads, D_L loads, reduction) are separate so that a caller can
// keep the loads of several outputs in flight together.
// Element idx of a matrix of fewer than 2^30 cells: the byte offset fits in 32
// bits, so the load takes a scalar base and one 32-bit vector offset.
__device__ __forceinline__ int32_t ld_cell(const int32_t *__restrict__ base, uint32_t idx) {
    return *reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(base) + (idx << 2));
}
// D_U loads of a batch; urow = offset of the vertex row in U
template <int B = kBatch>
__device__ __forceinline__ void batch_load_u(const int32_t *__restrict__ U, uint32_t urow,
                                             int32_t k0, int32_t step, int32_t hi, int32_t n,
                                             int32_t (&xs)[B]) {
#pragma unroll
    for (int t = 0; t < B; ++t)
        xs[t] = umin(ld_cell(U, urow + (uint32_t)imin(k0 + t * step, hi)), n + 1);
}
// D_L loads of a batch.  Row x <= n + 1 and row length ldL are below 2^24
// (a plan limit), so the row offset is one 24-bit multiply.  A candidate past
// hi is clamped to hi: with unit step, hi itself comes earlier in the same
// batch with the same value, so the duplicate can never be a strict minimum
// and needs no mask; with a larger step it is masked out.
template <bool kUnitStep, int B = kBatch>
__device__ __forceinline__ void batch_load_l(const int32_t *__restrict__ L, int32_t ldL, int32_t j,
                                             int32_t k0, int32_t step, int32_t hi,
                                             const int32_t (&xs)[B], int32_t (&vs)[B]) {
#pragma unroll
    for (int t = 0; t < B; ++t) {
        const int32_t kc = imin(k0 + t * step, hi);
        const int32_t v =
            ld_cell(L, __umul24((uint32_t)xs[t], (uint32_t)ldL) + (uint32_t)(j - kc));
        vs[t] = (kUnitStep || k0 + t * step <= hi) ? v : 0x7fffffff;
    }
}
template <int B = kBatch>
__device__ __forceinline__ bool batch_reduce(int32_t j, int32_t k0, int32_t step, int32_t hi,
                                             int32_t xb, int32_t vlo, int32_t n,
                                             const int32_t (&xs)[B], const int32_t (&vs)[B],
                                             int32_t &best, int32_t &bk) {
#pragma unroll
    for (int t = 0; t < B; ++t) {
        const bool upd = vs[t] < best;
        best = upd ? vs[t] : best;
        bk = upd ? k0 + t * step : bk;
    }
    const int32_t klast = k0 + (B - 1) * step;
    const int32_t xl = xs[B - 1];
    return (klast >= hi) | (xl > xb) | (best == vlo) | ((best <= n) & (xl - klast >= best - j));
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
// 0..P-2 (P a power of two > H), with a fan-out f per depth instead of
// Alg. 1's halving: when the columns c with (c + 1) % S == 0 are solved, the
// next depth solves every column with (c + 1) % (S / f) == 0 in between, each
// bounded by the two solved columns around it (position -1 and positions >= H
// are the open bounds 0 and hU).  Monotonicity bounds a column by ANY solved
// column on either side, so the result is the same for every f; f = 2 is
// Alg. 1's order.  f is the largest power of two that keeps a depth's
// candidates near kAnchorEval per thread, so a top-level row of 4097 columns
// takes 5-7 depths instead of 13.
// Within a depth the candidates of all new columns form one flat list (an
// exclusive prefix sum over the columns' window sizes) cut into equal
// consecutive runs, one per thread: the cost of a depth is its total number
// of candidates over the thread count, whatever the shape of the windows.
// A column-per-thread scan would instead wait for its longest window, and on
// rows with many unreachable columns (right of the vertex's LCS) the
// windows beside the reachable boundary are hundreds of candidates long.
// Each thread folds its run's (value, k) keys per column and merges them into
// the column's LDS 64-bit minimum, i.e. Alg. 2's minimum with the smaller
// index on ties.  Windows stop at KU, the largest k with D_U(vtx, k) <= n:
// beyond it D_U is the unreachable sentinel and so is every candidate.
// Krow (global, H entries) receives k*(j) or -1; D_G row vtx receives values.
// NT threads; a depth's new columns are processed NT * CPT at a time.  kLds:
// the D_U row and the k* row live in LDS (us: hU + 1 entries, ks: H entries;
// Krow is written once at the end), so that a candidate costs one global load
// (the D_L gather); otherwise both are read from global memory.
template <int NT, int CPT>
struct AnchorSmem {
    static constexpr int32_t kCols = NT * CPT;  // columns per segment
    unsigned long long key[kCols];              // per-column (value, k) minimum
    int32_t cps[kCols + 1];                     // exclusive prefix of window sizes
    int32_t clo[kCols];                         // first k of each window
    int32_t wsum[NT / kWave];
    int32_t ku;
};

// Inclusive prefix sum over a wave: lane l receives v[0] + ... + v[l].
__device__ __forceinline__ int32_t wave_prefix_sum(int32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}
// An anchor search runs on a whole block (NT = block size) or on one wave
// (NT = kWave, several searches per block).  In the wave form the wave's
// lanes are the threads and the barriers are wave-level: LDS operations of a
// wave complete in order, so waiting for them and keeping the compiler from
// moving memory operations across the point is enough.
template <int NT>
__device__ __forceinline__ int32_t anchor_tid() {
    return NT == kWave ? (int32_t)__lane_id() : (int32_t)threadIdx.x;
}
template <int NT>
__device__ __forceinline__ void anchor_sync() {
    if constexpr (NT == kWave) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Exclusive prefix sum over the NT threads of a block (or the lanes of a
// wave when NT = kWave); total receives the sum of all.  wsum: NT / kWave
// int32 of LDS, reusable after the next barrier (unused for one wave).
template <int NT>
__device__ __forceinline__ int32_t block_exclusive_sum(int32_t v, int32_t *wsum, int32_t &total) {
    const int32_t incl = wave_prefix_sum(v);
    if constexpr (NT == kWave) {
        total = __shfl(incl, kWave - 1, kWave);
        return incl - v;
    }
    const int w = (int)threadIdx.x / kWave;
    if (__lane_id() == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int32_t before = 0;
    total = 0;
#pragma unroll
    for (int w2 = 0; w2 < NT / kWave; ++w2) {
        const int32_t t = wsum[w2];
        before += (w2 < w) ? t : 0;
        total += t;
    }
    return before + incl - v;
}

template <bool kLds, typename KT>
__device__ __forceinline__ int32_t anchor_u(const int32_t *__restrict__ U, uint32_t urow,
                                            const KT *us, int32_t k, int32_t n) {
    if (kLds) return (int32_t)us[k];
    return umin(ld_cell(U, urow + (uint32_t)k), n + 1);
}

// kLds: the vertex's D_U row and k* row live in LDS (us, ks), as int32 or,
// with KT = uint16_t (n + 1 <= 65535 and hU <= 65533), as 16-bit values with
// k* stored as k* + 1, so that -1 is 0: half the LDS per work-group.
template <bool kLds, int NT, int CPT, typename KT = int32_t>
__device__ __forceinline__ void anchor_block_t(const int32_t *__restrict__ U, int32_t hU,
                               const int32_t *__restrict__ L, int32_t hL, int32_t *__restrict__ G,
                               int32_t n, int32_t vtx, int32_t *__restrict__ Krow,
                               AnchorSmem<NT, CPT> &sm, KT *us, KT *ks) {
    static_assert(sizeof(KT) == 4 || kLds, "16-bit rows are LDS rows");
    constexpr int32_t CM = AnchorSmem<NT, CPT>::kCols;
    const int32_t tid = anchor_tid<NT>();
    const int32_t INF = n + 1;
    const int32_t H = hU + hL + 1;
    int32_t P = 1;
    while (P < H + 1) P <<= 1;
    const uint32_t urow = (uint32_t)vtx * (uint32_t)(hU + 1);
    int32_t *__restrict__ grow = G + (size_t)vtx * (size_t)H;
    auto kget = [&](int32_t c) -> int32_t {
        if constexpr (!kLds)
            return Krow[c];
        else if constexpr (sizeof(KT) == 2)
            return (int32_t)ks[c] - 1;
        else
            return ks[c];
    };
    auto kput = [&](int32_t c, int32_t k) {
        if constexpr (!kLds)
            Krow[c] = k;
        else
            ks[c] = (KT)(sizeof(KT) == 2 ? k + 1 : k);
    };
    const int32_t ldL = hL + 1;
    if (tid == 0) sm.ku = -1;
    anchor_sync<NT>();
    // D_U row (non-decreasing in k) and KU
    for (int32_t k = tid; k <= hU; k += NT) {
        const int32_t x = umin(ld_cell(U, urow + (uint32_t)k), INF);
        const int32_t xn = (k < hU) ? umin(ld_cell(U, urow + (uint32_t)k + 1u), INF) : INF;
        if (kLds) us[k] = (KT)x;
        if (x <= n && xn > n) sm.ku = k;
    }
    anchor_sync<NT>();
    const int32_t KU = sm.ku;
    for (int32_t S = P; S > 1;) {
        // fan-out: the f - 1 new columns of each interval scan about
        // (f - 1) * (hU + 1 + intervals) candidates in all
        const int32_t rng = hU + 1 + (H + S - 1) / S;
        int32_t f = 2;
        while (f < S && (2 * f - 1) * rng <= NT * kAnchorEval) f <<= 1;
        const int32_t S2 = S / f;
        const int32_t ncols = H / S2;  // positions (t + 1) * S2 - 1 < H
        for (int32_t seg = 0; seg < ncols; seg += CM) {
            // windows of the segment's new columns (already solved positions
            // and dead columns get none)
            int32_t r[CPT];
            int32_t tsum = 0;
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int32_t idx = tid * CPT + u;
                const int32_t t = seg + idx;
                int32_t lo = 0;
                r[u] = 0;
                if (t < ncols && ((t + 1) & (f - 1)) != 0) {
                    const int32_t c = (t + 1) * S2 - 1;
                    const int32_t cl = ((t + 1) & ~(f - 1)) * S2 - 1, cr = cl + S;
                    int32_t kl = 0, kr = hU;
                    bool dead = false;
                    if (cl >= 0) {
                        kl = kget(cl);
                        dead = kl < 0;
                    }
                    if (cr < H) {
                        const int32_t t2 = kget(cr);
                        if (t2 >= 0) kr = t2;
                    }
                    lo = imax(kl, imax(c - hL, 0));
                    const int32_t hi = imin(imin(kr, KU), imin(c, hU));
                    if (!dead && lo <= hi) {
                        r[u] = hi - lo + 1;
                    } else {
                        kput(c, -1);
                        grow[c] = INF;
                    }
                }
                sm.key[idx] = ~0ull;
                sm.clo[idx] = lo;
                tsum += r[u];
            }
            int32_t W;
            int32_t ex = block_exclusive_sum<NT>(tsum, sm.wsum, W);
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                sm.cps[tid * CPT + u] = ex;
                ex += r[u];
            }
            if (tid == 0) sm.cps[CM] = W;
            anchor_sync<NT>();
            // candidates e0 .. e1-1 of the flat list
            const int32_t C = (W + NT - 1) / NT;
            const int32_t e0 = tid * C;
            const int32_t e1 = imin(e0 + C, W);
            if (e0 < e1) {
                // the column holding e0: the last index with cps <= e0 (a
                // non-empty window, since cps[CM] = W > e0)
                int32_t col = 0;
                for (int32_t hi2 = CM - 1; col < hi2;) {
                    const int32_t mid = (col + hi2 + 1) >> 1;
                    if (sm.cps[mid] <= e0)
                        col = mid;
                    else
                        hi2 = mid - 1;
                }
                int32_t cbeg = sm.cps[col], cend = sm.cps[col + 1], clo = sm.clo[col];
                int32_t rcol = col;
                unsigned long long run = ~0ull;
                for (int32_t e = e0; e < e1; e += kBatch) {
                    int32_t cix[kBatch], kk[kBatch], xs[kBatch], vs[kBatch];
#pragma unroll
                    for (int t = 0; t < kBatch; ++t) {
                        const int32_t ee = imin(e + t, e1 - 1);
                        while (ee >= cend) {
                            ++col;
                            cbeg = cend;
                            cend = sm.cps[col + 1];
                            clo = sm.clo[col];
                        }
                        cix[t] = col;
                        kk[t] = clo + (ee - cbeg);
                    }
#pragma unroll
                    for (int t = 0; t < kBatch; ++t) xs[t] = anchor_u<kLds, KT>(U, urow, us, kk[t], n);
#pragma unroll
                    for (int t = 0; t < kBatch; ++t) {
                        const int32_t c = (seg + cix[t] + 1) * S2 - 1;
                        vs[t] = ld_cell(L, __umul24((uint32_t)xs[t], (uint32_t)ldL) + (uint32_t)(c - kk[t]));
                    }
#pragma unroll
                    for (int t = 0; t < kBatch; ++t) {
                        if (e + t < e1) {
                            const unsigned long long key =
                                ((unsigned long long)(uint32_t)vs[t] << 32) | (uint32_t)kk[t];
                            if (cix[t] != rcol) {
                                atomicMin(&sm.key[rcol], run);
                                rcol = cix[t];
                                run = key;
                            } else {
                                run = key < run ? key : run;
                            }
                        }
                    }
                }
                atomicMin(&sm.key[rcol], run);
            }
            anchor_sync<NT>();
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                if (r[u] > 0) {
                    const int32_t idx = tid * CPT + u;
                    const int32_t c = (seg + idx + 1) * S2 - 1;
                    const unsigned long long key = sm.key[idx];
                    const uint32_t v = (uint32_t)(key >> 32);
                    if (v <= (uint32_t)n) {
                        kput(c, (int32_t)(uint32_t)(key & 0xffffffffull));
                        grow[c] = (int32_t)v;
                    } else {
                        kput(c, -1);
                        grow[c] = INF;
                    }
                }
            }
            anchor_sync<NT>();
        }
        S = S2;
    }
    if (kLds) {
        for (int32_t c = tid; c < H; c += NT) Krow[c] = kget(c);
        anchor_sync<NT>();
    }
}

// Global-memory form (the batch kernels: fixed LDS budget).
using AnchorSmemBlock = AnchorSmem<kBlock, 4>;
__device__ __forceinline__ void anchor_block(const int32_t *__restrict__ U, int32_t hU,
                                             const int32_t *__restrict__ L, int32_t hL,
                                             int32_t *__restrict__ G, int32_t n, int32_t vtx,
                                             int32_t *__restrict__ Krow, AnchorSmemBlock &sm) {
    anchor_block_t<false, kBlock, 4, int32_t>(U, hU, L, hL, G, n, vtx, Krow, sm, nullptr, nullptr);
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
// weights lives in LDS; values reach D_G as soon as they are final, in
// contiguous row segments.
// D_U in LDS: by the window above (applied level by level, and with k*
// non-decreasing in j) every candidate of vertex i0 + v lies in
// [k*(i0, j0) - v, k*(i1, jl) + (len - v)], jl the last weight that is
// reachable from i0.  When that parallelogram is at most kUW wide and
// k*(i1, jl) exists, the block first copies it from D_U into LDS and the
// bisection reads D_U only from there: one HBM round trip per level (the D_L
// gathers) instead of two.  Otherwise D_U is read from global memory.
// A block none of whose weights is reachable from i0 writes unreachable
// everywhere (reachability is monotone in the vertex).
// Latency: within a bisection level each thread owns up to 2
// outputs and issues the loads of all of them before it waits, and every
// output first runs exactly one batch of candidates; the few that are not
// finished are queued in LDS and completed by all threads together, so a wave
// never waits for its slowest lane during the common case.
// The last weight of a strip, j = hU + hL, has the single candidate k = hU; a
// block that holds it (jn = kJ + 1) evaluates it directly, so the
// bisection works on at most kJ weights.
constexpr int kCoarseItems = kBlock / 2;  // a level with at most this many outputs is coarse
constexpr int kCoarseBatch = 8;  // consecutive candidates per thread slice of a coarse level
constexpr int kPass2Batch = 8;   // candidates per batch of pass 2, one thread per output
constexpr int32_t kCoopPass2MinH = 256;  // child strip height from which pass 2 is cooperative
constexpr int32_t kWideWindowMinH = 2048;  // child strip height from which the D_U window is wide
// Shape of a bracket work-group: LDS state type, weights per block, width of
// the D_U parallelogram.  32-bit state: any size.  16-bit state (values and
// indices stored in 16 bits, k* stored as k* + 1 so that -1 is 0): needs
// n + 1 <= 65535 and strip heights <= 65534, and holds twice the weights in
// about the same LDS, which halves the per-work-group overhead per output.
template <typename T, int J, int UW, int CB = 8>
struct BracketCfg {
    using St = T;
    static constexpr int kJ = J;
    static constexpr int kUW = UW;
    static constexpr int kCoopB = CB;  // candidates per thread slice of the cooperative pass 2
};
using BracketCfg32 = BracketCfg<int32_t, 32, 64>;
using BracketCfg16 = BracketCfg<uint16_t, 64, 100>;
using BracketCfg16Mid = BracketCfg<uint16_t, 64, 128, 6>;  // 256+ rows: still 8 work-groups per CU
using BracketCfg16Wide = BracketCfg<uint16_t, 64, 160>;  // tall strips: wider D_U window

template <class C>
struct __align__(16) BracketSmemT {
    using St = typename C::St;
    St k[(kMaxTile + 1) * C::kJ];
    St v[(kMaxTile + 1) * C::kJ];
    St u[(kMaxTile + 1) * C::kUW];  // D_U parallelogram (row v starts at k*(i0, j0) - v)
    St q[(kMaxTile / 2) * C::kJ];   // queued outputs of one level (slot * kJ + jj)
    unsigned long long key[kCoarseItems];  // slice minima (value, k) of a coarse level
    int32_t qn[2];                         // queue lengths, alternating between levels
    int32_t xlast[kMaxTile];               // D_U(i0 + v, hU) for the strip's last weight
};
using BracketSmem = BracketSmemT<BracketCfg32>;

template <class C>
__device__ __forceinline__ int32_t ldk(const BracketSmemT<C> &sm, int32_t i) {
    if constexpr (sizeof(typename C::St) == 2)
        return (int32_t)sm.k[i] - 1;
    else
        return sm.k[i];
}
template <class C>
__device__ __forceinline__ void stk(BracketSmemT<C> &sm, int32_t i, int32_t k) {
    if constexpr (sizeof(typename C::St) == 2)
        sm.k[i] = (uint16_t)(k + 1);
    else
        sm.k[i] = k;
}

struct BracketWindow {
    int32_t lo, hi, xb, vlo, vhi;
    bool dead;
};

// D_U(i0 + v, k) of a tile vertex: from the LDS parallelogram (kLds; the
// index is clamped into the row, so any k reads inside it) or from global
// memory.
template <class C, bool kLds>
__device__ __forceinline__ int32_t bracket_u(const BracketSmemT<C> &sm, const int32_t *__restrict__ U,
                                             int32_t ldU, int32_t hU, int32_t i0, int32_t ubase,
                                             int32_t v, int32_t k, int32_t n) {
    if (kLds) return (int32_t)sm.u[v * C::kUW + imin(imax(k - ubase + v, 0), C::kUW - 1)];
    return umin(ld_cell(U, (uint32_t)(i0 + v) * (uint32_t)ldU + (uint32_t)imin(imax(k, 0), hU)),
                n + 1);
}

// Search window of output (v, j) from the solved vertices va < v < vb; the
// crossing bound x*(vb, j) = D_U(i0 + vb, k*(vb, j)) is looked up from k*.
template <class C, bool kLds>
__device__ __forceinline__ BracketWindow bracket_window(const BracketSmemT<C> &sm,
                                                        const int32_t *__restrict__ U, int32_t ldU,
                                                        int32_t i0, int32_t ubase, int32_t v,
                                                        int32_t va, int32_t vb, int32_t jj,
                                                        int32_t js, int32_t j, int32_t hU,
                                                        int32_t hL, int32_t n) {
    constexpr int32_t S = C::kJ;
    BracketWindow w;
    const int32_t ka = ldk(sm, va * S + jj);
    const int32_t kb = ldk(sm, vb * S + jj);
    w.dead = ka < 0;
    w.hi = imin(j, hU);
    w.xb = n;
    if (kb >= 0) {
        w.hi = imin(kb + (vb - v), w.hi);
        w.xb = bracket_u<C, kLds>(sm, U, ldU, hU, i0, ubase, vb, kb, n);
    }
    w.lo = imax(ka - (v - va), imax(j - hL, 0));
    // value bounds from the rows of the two brackets (rows of a breakout
    // matrix interlace: D(i + d, j - d) <= D(i, j) <= D(i - d, j + d)), with
    // the weights that lie inside this block's range
    w.vlo = (int32_t)sm.v[va * S + jj];
    w.vhi = (int32_t)sm.v[vb * S + jj];
    if (jj >= vb - v) w.vlo = imax(w.vlo, (int32_t)sm.v[vb * S + jj - (vb - v)]);
    if (jj + (v - va) < js) w.vhi = imin(w.vhi, (int32_t)sm.v[va * S + jj + (v - va)]);
    return w;
}

// Final result of one output: the LDS state that finer levels read; the block
// writes all of its outputs to D_G at the end, row segment by row segment.
template <class C>
__device__ __forceinline__ void bracket_store(BracketSmemT<C> &sm, int32_t id, int32_t n,
                                              int32_t best, int32_t bk) {
    if (best > n) {
        best = n + 1;
        bk = -1;
    }
    stk(sm, id, bk);
    sm.v[id] = (typename C::St)best;
}

// D_U loads of one batch of tile vertex v (LDS parallelogram or global).
template <class C, int B, bool kLds>
__device__ __forceinline__ void bracket_load_u(const BracketSmemT<C> &sm, const int32_t *__restrict__ U,
                                               int32_t ldU, int32_t hU, int32_t i0, int32_t ubase,
                                               int32_t v, int32_t k0, int32_t hi, int32_t n,
                                               int32_t (&xs)[B]) {
#pragma unroll
    for (int t = 0; t < B; ++t)
        xs[t] = bracket_u<C, kLds>(sm, U, ldU, hU, i0, ubase, v, imin(k0 + t, hi), n);
}

// Pass 1 of one bisection level with R outputs per thread: every output runs
// one batch of candidates.  The loads carry no branches (an idle output reads
// vertex i0, weight 0, which is in bounds) so that the loads of all R outputs
// are in flight together.  Unfinished outputs are queued for pass 2.
template <class C, int R, int B, bool kLds>
__device__ __forceinline__ void bracket_pass1(BracketSmemT<C> &sm, const int32_t *__restrict__ U,
                                              int32_t hU, const int32_t *__restrict__ L,
                                              int32_t hL, int32_t *__restrict__ G, int32_t n,
                                              int32_t i0, int32_t len, int32_t j0, int32_t js,
                                              int32_t half, int32_t st, int32_t nitems,
                                              int32_t par, int32_t ubase, int32_t ebase) {
    constexpr int32_t S = C::kJ;
    // a wave without outputs at this level skips it (no barrier inside)
    if (ebase + (int32_t)(threadIdx.x & ~(kWave - 1)) >= nitems) return;
    const int32_t INF = n + 1;
    const int32_t H = hU + hL + 1;
    const int32_t ldU = hU + 1, ldL = hL + 1;
    const int32_t lane = __lane_id();
    int32_t id[R], vr[R], jv[R], lo[R], hi[R], xb[R], vlo[R];
    bool act[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int32_t e = ebase + (int32_t)threadIdx.x + r * kBlock;
        const int32_t t = e / S, jj = e - t * S;
        const int32_t v = half + t * st;
        id[r] = v * S + jj;
        vr[r] = 0;
        jv[r] = 0;
        lo[r] = kLds ? ubase : 0;
        hi[r] = lo[r];
        xb[r] = n;
        vlo[r] = -1;
        act[r] = false;
        if ((e < nitems) && (jj < js)) {
            const int32_t j = j0 + jj;
            const BracketWindow w = bracket_window<C, kLds>(sm, U, ldU, i0, ubase, v, v - half,
                                                         imin(v + half, len), jj, js, j, hU, hL, n);
            if (w.dead || w.lo > w.hi) {
                bracket_store(sm, id[r], n, INF, -1);
            } else {
                act[r] = true;
                vr[r] = v;
                jv[r] = j;
                lo[r] = w.lo;
                hi[r] = w.hi;
                xb[r] = w.xb;
                vlo[r] = w.vlo;
            }
        }
    }
    int32_t xs[R][B], vs[R][B];
#pragma unroll
    for (int r = 0; r < R; ++r)
        bracket_load_u<C, B, kLds>(sm, U, ldU, hU, i0, ubase, vr[r], lo[r], hi[r], n, xs[r]);
#pragma unroll
    for (int r = 0; r < R; ++r)
        batch_load_l<true, B>(L, ldL, jv[r], lo[r], 1, hi[r], xs[r], vs[r]);
    // The loaded values are needed on every path from here: keeps the compiler
    // from sinking the loads of an idle output into a branch, which would
    // serialise the outputs' loads again.  (An empty statement, no instruction.)
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < B; ++t) asm volatile("" : "+v"(vs[r][t]), "+v"(xs[r][t]));
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int32_t best = n + 2, bk = -1;
        const bool done =
            batch_reduce<B>(jv[r], lo[r], 1, hi[r], xb[r], vlo[r], n, xs[r], vs[r], best, bk);
        bool queued = false;
        if (act[r]) {
            if (done) {
                bracket_store(sm, id[r], n, best, bk);
            } else {  // provisional state; pass 2 resumes at lo + B
                stk(sm, id[r], bk);
                sm.v[id[r]] = (typename C::St)imin(best, n + 1);
                queued = true;
            }
        }
        // reserve queue slots with one LDS atomic per wave
        const unsigned long long mask = __ballot(queued);
        if (mask) {
            const int32_t leader = __ffsll((long long)mask) - 1;
            int32_t qbase = 0;
            if (lane == leader) qbase = atomicAdd(&sm.qn[par], __popcll(mask));
            qbase = __shfl(qbase, leader, kWave);
            if (queued) {
                const unsigned long long below = mask & ((1ull << lane) - 1ull);
                sm.q[qbase + __popcll(below)] = (typename C::St)id[r];
            }
        }
    }
}

// Finest bisection level (every other vertex; only values are needed).  Each
// wave first tries the value bounds of its outputs, which meet for most of
// them (the rows of the two neighbours interlace around each), and collects
// the others in a wave-local list; it then searches the listed outputs one
// per lane, B candidates each with all loads in flight, so no candidate is
// loaded for an output whose value is already fixed and one round trip serves
// all of the wave's searched outputs.  Unfinished outputs go to the level
// queue for pass 2 (which resumes at lo + B).  The list lives in sm.key (128
// entries per wave), which no other part of the block uses meanwhile; it is
// set back to the all-ones state the coarse levels and pass 2 expect.
template <class C, int B, bool kLds>
__device__ __forceinline__ void bracket_finest(BracketSmemT<C> &sm, const int32_t *__restrict__ U,
                                               int32_t hU, const int32_t *__restrict__ L,
                                               int32_t hL, int32_t n, int32_t i0, int32_t len,
                                               int32_t j0, int32_t js, int32_t nitems, int32_t par,
                                               int32_t ubase) {
    constexpr int32_t S = C::kJ;
    constexpr int32_t kCap = 2 * kWave;  // list entries per wave
    static_assert(sizeof(sm.key) >= (size_t)kWaves * kCap * sizeof(uint16_t), "list space");
    const int32_t INF = n + 1;
    const int32_t ldU = hU + 1, ldL = hL + 1;
    const int32_t lane = __lane_id();
    const int32_t wv = (int32_t)threadIdx.x / kWave;
    uint16_t *list = reinterpret_cast<uint16_t *>(sm.key) + wv * kCap;
    const int32_t rounds = (nitems + kBlock - 1) / kBlock;
    int32_t cnt = 0;  // wave-uniform
    for (int32_t r = 0; r < rounds; ++r) {
        const int32_t e = r * kBlock + (int32_t)threadIdx.x;
        const int32_t t = e / S, jj = e - t * S;
        const int32_t v = 1 + 2 * t;
        bool pend = false;
        if (e < nitems && jj < js) {
            const BracketWindow w = bracket_window<C, kLds>(sm, U, ldU, i0, ubase, v, v - 1,
                                                         imin(v + 1, len), jj, js, j0 + jj, hU, hL, n);
            if (w.dead || w.lo > w.hi)
                bracket_store(sm, v * S + jj, n, INF, -1);
            else if (w.vlo == w.vhi)  // the interlacing bounds meet: the value is fixed
                bracket_store(sm, v * S + jj, n, w.vlo, 0);
            else
                pend = true;
        }
        const unsigned long long m = __ballot(pend);
        if (pend) list[cnt + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)(v * S + jj);
        cnt += __popcll(m);
        if (cnt <= kWave && r < rounds - 1) continue;
        anchor_sync<kWave>();  // the list is written before any lane reads it
        for (int32_t p0 = 0; p0 < cnt; p0 += kWave) {
            const bool act = p0 + lane < cnt;
            const int32_t id = act ? (int32_t)list[p0 + lane] : 0;
            const int32_t vq = id / S, jq = id - vq * S;
            int32_t vr = 0, jv = 0, lo = kLds ? ubase : 0, hi = lo, xb = n, vlo = -1;
            if (act) {
                const BracketWindow w = bracket_window<C, kLds>(sm, U, ldU, i0, ubase, vq, vq - 1,
                                                             imin(vq + 1, len), jq, js, j0 + jq, hU,
                                                             hL, n);
                vr = vq;
                jv = j0 + jq;
                lo = w.lo;
                hi = w.hi;
                xb = w.xb;
                vlo = w.vlo;
            }
            int32_t xs[B], vs[B];
            bracket_load_u<C, B, kLds>(sm, U, ldU, hU, i0, ubase, vr, lo, hi, n, xs);
            batch_load_l<true, B>(L, ldL, jv, lo, 1, hi, xs, vs);
            int32_t best = n + 2, bk = -1;
            const bool done = batch_reduce<B>(jv, lo, 1, hi, xb, vlo, n, xs, vs, best, bk);
            bool queued = false;
            if (act) {
                if (done) {
                    bracket_store(sm, id, n, best, bk);
                } else {  // provisional state; pass 2 resumes at lo + B
                    stk(sm, id, bk);
                    sm.v[id] = (typename C::St)imin(best, n + 1);
                    queued = true;
                }
            }
            const unsigned long long mq = __ballot(queued);
            if (mq) {
                const int32_t leader = __ffsll((long long)mq) - 1;
                int32_t qbase = 0;
                if (lane == leader) qbase = atomicAdd(&sm.qn[par], __popcll(mq));
                qbase = __shfl(qbase, leader, kWave);
                if (queued) sm.q[qbase + __popcll(mq & ((1ull << lane) - 1ull))] = (typename C::St)id;
            }
        }
        anchor_sync<kWave>();  // every lane has read the list before it is refilled
        cnt = 0;
    }
    // the list space back to the all-ones (value, k) minima
    if (lane < kCap * (int32_t)sizeof(uint16_t) / 8)
        sm.key[wv * (kCap * (int32_t)sizeof(uint16_t) / 8) + lane] = ~0ull;
}

// Coarse bisection level (at most kCoarseItems outputs, wide windows): g
// threads per output scan consecutive slices of kCoarseBatch candidates of its
// window in the same round, so the output sees g * kCoarseBatch candidates for one
// round trip.  Slice minima meet through a 64-bit LDS atomic min of
// (value, k), which keeps the smallest minimising k.  The stop tests then run
// on the whole range; an unfinished output resumes in pass 2 after it.
template <class C, bool kLds>
__device__ __forceinline__ void bracket_coarse(BracketSmemT<C> &sm, const int32_t *__restrict__ U,
                                               int32_t hU, const int32_t *__restrict__ L,
                                               int32_t hL, int32_t *__restrict__ G, int32_t n,
                                               int32_t i0, int32_t len, int32_t j0, int32_t js,
                                               int32_t half, int32_t st, int32_t nitems,
                                               int32_t par, int32_t ubase, int32_t g) {
    constexpr int32_t S = C::kJ;
    const int32_t INF = n + 1;
    const int32_t H = hU + hL + 1;
    const int32_t ldU = hU + 1, ldL = hL + 1;
    const int32_t lane = __lane_id();
    {  // slices
        const int32_t e = (int32_t)threadIdx.x / g, sub = (int32_t)threadIdx.x - e * g;
        const int32_t t = e / S, jj = e - t * S;
        if (e < nitems && jj < js) {
            const int32_t v = half + t * st, j = j0 + jj;
            const BracketWindow w = bracket_window<C, kLds>(sm, U, ldU, i0, ubase, v, v - half,
                                                         imin(v + half, len), jj, js, j, hU, hL, n);
            const int32_t k0 = w.lo + sub * kCoarseBatch;
            if (!w.dead && k0 <= w.hi) {
                int32_t xs[kCoarseBatch], vs[kCoarseBatch];
                bracket_load_u<C, kCoarseBatch, kLds>(sm, U, ldU, hU, i0, ubase, v, k0, w.hi, n, xs);
                batch_load_l<false, kCoarseBatch>(L, ldL, j, k0, 1, w.hi, xs, vs);
                int32_t best = n + 2, bk = -1;
                batch_reduce<kCoarseBatch>(j, k0, 1, w.hi, w.xb, w.vlo, n, xs, vs, best, bk);
                if (best <= n)
                    atomicMin(&sm.key[e], ((unsigned long long)(uint32_t)best << 32) | (uint32_t)bk);
            }
        }
    }
    __syncthreads();
    // one thread per output: stop tests on the whole range, store or queue
    bool queued = false;
    int32_t qid = 0;
    const int32_t e = (int32_t)threadIdx.x;
    const int32_t t = e / S, jj = e - t * S;
    if (e < nitems && jj < js) {
        const int32_t v = half + t * st, j = j0 + jj;
        const int32_t id = v * S + jj;
        const BracketWindow w = bracket_window<C, kLds>(sm, U, ldU, i0, ubase, v, v - half,
                                                     imin(v + half, len), jj, js, j, hU, hL, n);
        const unsigned long long key = sm.key[e];
        sm.key[e] = ~0ull;  // ready for the next coarse level
        if (w.dead || w.lo > w.hi) {
            bracket_store(sm, id, n, INF, -1);
        } else {
            int32_t best = n + 2, bk = -1;
            if (key != ~0ull) {
                best = (int32_t)(key >> 32);
                bk = (int32_t)(uint32_t)(key & 0xffffffffull);
            }
            const int32_t kend = w.lo + g * kCoarseBatch - 1;
            const int32_t xl = bracket_u<C, kLds>(sm, U, ldU, hU, i0, ubase, v, imin(kend, w.hi), n);
            const bool done = (kend >= w.hi) | (xl > w.xb) | (best == w.vlo) |
                              ((best <= n) & (xl - kend >= best - j));
            if (done) {
                bracket_store(sm, id, n, best, bk);
            } else {  // provisional state; pass 2 resumes at lo + g * kCoarseBatch
                stk(sm, id, bk);
                sm.v[id] = (typename C::St)imin(best, n + 1);
                queued = true;
                qid = id;
            }
        }
    }
    const unsigned long long mask = __ballot(queued);
    if (mask) {
        const int32_t leader = __ffsll((long long)mask) - 1;
        int32_t qbase = 0;
        if (lane == leader) qbase = atomicAdd(&sm.qn[par], __popcll(mask));
        qbase = __shfl(qbase, leader, kWave);
        if (queued) {
            const unsigned long long below = mask & ((1ull << lane) - 1ull);
            sm.q[qbase + __popcll(below)] = (typename C::St)qid;
        }
    }
}

template <class C, bool kLds, bool kCoop>
__device__ __forceinline__ void bracket_levels(BracketSmemT<C> &sm, const int32_t *__restrict__ U,
                                               int32_t hU, const int32_t *__restrict__ L,
                                               int32_t hL, int32_t *__restrict__ G, int32_t n,
                                               int32_t i0, int32_t len, int32_t j0, int32_t js,
                                               int32_t ubase) {
    constexpr int32_t S = C::kJ;
    const int32_t H = hU + hL + 1;
    const int32_t ldU = hU + 1, ldL = hL + 1;
    int32_t P2 = 1;
    while (P2 < len) P2 <<= 1;
    int32_t par = 0;
    for (int32_t st = P2; st >= 2; st >>= 1, par ^= 1) {
        const int32_t half = st >> 1;
        const int32_t nv = (len > half) ? (len - half + st - 1) / st : 0;
        const int32_t nitems = nv * S;
        if (threadIdx.x == 0) sm.qn[par ^ 1] = 0;  // next level's queue (read after a barrier)
        // first pass: coarse levels spread each window over g threads; the
        // fine levels (most outputs, narrow windows) take small batches
        int32_t b1;
        if (st == 2) {
            b1 = 3;
            bracket_finest<C, 3, kLds>(sm, U, hU, L, hL, n, i0, len, j0, js, nitems, par, ubase);
        } else if (nitems <= kCoarseItems) {
            int32_t g = 2;
            while (2 * g * nitems <= kBlock) g <<= 1;
            b1 = g * kCoarseBatch;
            bracket_coarse<C, kLds>(sm, U, hU, L, hL, G, n, i0, len, j0, js, half, st, nitems,
                                    par, ubase, g);
        } else if (nitems > kBlock) {
            // two outputs per thread in flight together; a level of more than
            // 2 * kBlock outputs takes two such rounds.  Batches of 3 (the
            // narrowest windows here are 3 or 5 wide): measured 4% faster
            // than 4 and than 2 on both benchmark pairs
            b1 = 3;
            for (int32_t eb = 0; eb < nitems; eb += 2 * kBlock)
                bracket_pass1<C, 2, 3, kLds>(sm, U, hU, L, hL, G, n, i0, len, j0, js, half, st,
                                             nitems, par, ubase, eb);
        } else {
            // one output per thread; its window is at least st + 1 wide.
            // Batches of 6: with 4, 43% to 70% of this level's outputs went on
            // to pass 2 in the 2048- to 8192-row combines of the 16384² pair
            b1 = 6;
            bracket_pass1<C, 1, 6, kLds>(sm, U, hU, L, hL, G, n, i0, len, j0, js, half, st, nitems,
                                         par, ubase, 0);
        }
        __syncthreads();
        // pass 2: the queued outputs.  kCoop (tall strips) and few of them: g
        // threads each scan interleaved slices of C::kCoopB candidates, so an
        // output sees g * C::kCoopB candidates per round trip (slice minima meet
        // in the LDS (value, k) minimum; the provisional pass-1 result, whose
        // candidates all lie below, keeps ties).  Otherwise one thread each,
        // batch after batch.  Measured on both benchmark pairs: queued outputs
        // of strips below kCoopPass2MinH rows mostly finish in one more batch,
        // and the second barrier of the cooperative form then costs more than
        // it saves; above it they take several (measured again with combed
        // base strips: the 256-row children of 4096² gain too, 0.154 -> 0.145
        // ms).
        const int32_t qn = sm.qn[par];
        if (kCoop && qn > 0 && qn <= kCoarseItems) {
            int32_t g = 1;
            while (2 * g * qn <= kBlock) g <<= 1;
            const int32_t e = (int32_t)threadIdx.x / g, sub = (int32_t)threadIdx.x - e * g;
            if (e < qn) {
                const int32_t idq = (int32_t)sm.q[e];
                const int32_t v = idq / S, jj = idq - v * S;
                const int32_t j = j0 + jj;
                const BracketWindow wq = bracket_window<C, kLds>(sm, U, ldU, i0, ubase, v, v - half,
                                                              imin(v + half, len), jj, js, j, hU, hL, n);
                const int32_t best0 = (int32_t)sm.v[idq];
                int32_t best = best0, bk = -1;
                constexpr int CB = C::kCoopB;
                for (int32_t k0 = wq.lo + b1 + sub * CB; k0 <= wq.hi; k0 += g * CB) {
                    int32_t xs[CB], vs[CB];
                    bracket_load_u<C, CB, kLds>(sm, U, ldU, hU, i0, ubase, v, k0, wq.hi, n, xs);
                    batch_load_l<true, CB>(L, ldL, j, k0, 1, wq.hi, xs, vs);
                    if (batch_reduce<CB>(j, k0, 1, wq.hi, wq.xb, wq.vlo, n, xs, vs, best, bk)) break;
                }
                if (best < best0)
                    atomicMin(&sm.key[e], ((unsigned long long)(uint32_t)best << 32) | (uint32_t)bk);
            }
            __syncthreads();
            if ((int32_t)threadIdx.x < qn) {
                const int32_t idq = (int32_t)sm.q[threadIdx.x];
                const int32_t v = idq / S, jj = idq - v * S;
                const unsigned long long key = sm.key[threadIdx.x];
                sm.key[threadIdx.x] = ~0ull;
                int32_t best = (int32_t)sm.v[idq], bk = ldk(sm, idq);
                if (key != ~0ull) {
                    best = (int32_t)(key >> 32);
                    bk = (int32_t)(uint32_t)(key & 0xffffffffull);
                }
                bracket_store(sm, idq, n, best, bk);
            }
            __syncthreads();
        } else if (qn > 0) {
            for (int32_t e = threadIdx.x; e < qn; e += kBlock) {
                const int32_t idq = (int32_t)sm.q[e];
                const int32_t v = idq / S, jj = idq - v * S;
                const int32_t j = j0 + jj;
                const BracketWindow wq = bracket_window<C, kLds>(sm, U, ldU, i0, ubase, v, v - half,
                                                              imin(v + half, len), jj, js, j, hU, hL, n);
                int32_t best = (int32_t)sm.v[idq], bk = ldk(sm, idq);
                for (int32_t k0 = wq.lo + b1;; k0 += kPass2Batch) {
                    int32_t xs[kPass2Batch], vs[kPass2Batch];
                    bracket_load_u<C, kPass2Batch, kLds>(sm, U, ldU, hU, i0, ubase, v, k0, wq.hi, n, xs);
                    batch_load_l<true, kPass2Batch>(L, ldL, j, k0, 1, wq.hi, xs, vs);
                    if (batch_reduce<kPass2Batch>(j, k0, 1, wq.hi, wq.xb, wq.vlo, n, xs, vs, best, bk))
                        break;
                }
                bracket_store(sm, idq, n, best, bk);
            }
            __syncthreads();
        }
    }
}

// LDS copy of D_U for a tile: sm.u[v * kUW + c] = D_U(i0 + v, org - v + c)
// for v = 0..len and c = 0..kUW-1, with k clamped into 0..hU and values
// clamped to INF.  Four consecutive entries per thread and pass: one address,
// four loads, one LDS store.  All passes' loads are issued before the first
// LDS store, so the whole copy costs one memory round trip.
template <class C>
__device__ __forceinline__ void bracket_copy_u(BracketSmemT<C> &sm, const int32_t *__restrict__ U,
                                               int32_t ldU, int32_t hU, int32_t i0, int32_t len,
                                               int32_t org, int32_t INF) {
    constexpr int32_t UW = C::kUW;
    static_assert(UW % 4 == 0, "the D_U window is copied four entries at a time");
    constexpr int32_t Q = UW / 4;
    constexpr int32_t kPasses = ((kMaxTile + 1) * Q + kBlock - 1) / kBlock;
    const int32_t total = (len + 1) * Q;
    uint32_t x[kPasses][4];
#pragma unroll
    for (int it = 0; it < kPasses; ++it) {
        const int32_t e = (int32_t)threadIdx.x + it * kBlock;
        const int32_t v = imin(e, total - 1) / Q, c = (imin(e, total - 1) - v * Q) * 4;
        const int32_t k0 = org - v + c;
        const int32_t *__restrict__ row = U + (size_t)(i0 + v) * ldU;
        if (k0 >= 0 && k0 + 3 <= hU) {
#pragma unroll
            for (int t = 0; t < 4; ++t) x[it][t] = (uint32_t)row[k0 + t];
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) x[it][t] = (uint32_t)row[imin(imax(k0 + t, 0), hU)];
        }
    }
#pragma unroll
    for (int it = 0; it < kPasses; ++it) {
        const int32_t e = (int32_t)threadIdx.x + it * kBlock;
        if (e < total) {
            const int32_t v = e / Q, c = (e - v * Q) * 4;
            uint32_t y[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) y[t] = x[it][t] < (uint32_t)INF ? x[it][t] : (uint32_t)INF;
            if constexpr (sizeof(typename C::St) == 2) {
                *reinterpret_cast<uint2 *>(&sm.u[v * UW + c]) =
                    make_uint2(y[0] | (y[1] << 16), y[2] | (y[3] << 16));
            } else {
                *reinterpret_cast<uint4 *>(&sm.u[v * UW + c]) = make_uint4(y[0], y[1], y[2], y[3]);
            }
        }
    }
}

template <class C, bool kCoop = false>
__device__ __forceinline__ void bracket_block(const int32_t *__restrict__ U, int32_t hU,
                                              const int32_t *__restrict__ L, int32_t hL,
                                              int32_t *__restrict__ G, int32_t n, int32_t i0,
                                              int32_t len, int32_t j0, int32_t jn,
                                              const int32_t *__restrict__ Ka,
                                              const int32_t *__restrict__ Kb, BracketSmemT<C> &sm) {
    if (len < 2 || jn <= 0) return;
    constexpr int32_t S = C::kJ;  // LDS row stride; item slots per vertex
    constexpr int32_t NE = (S + kWave - 1) / kWave;  // tile-end weights per lane
    const int32_t INF = n + 1;
    const int32_t H = hU + hL + 1;
    const int32_t ldU = hU + 1, ldL = hL + 1;
    const int32_t js = imin(jn, S);  // weights solved by bisection
    const int32_t lane = __lane_id();
    // Weight j0 + S = hU + hL (a block with jn = S + 1) has the single
    // candidate k = hU.  Its D_U load travels with the tile-end loads (parked
    // in LDS, which keeps it out of the registers) and its D_L load with the
    // parallelogram copy, so it adds no round trip.
    if ((jn > S) && threadIdx.x >= 1 && (int32_t)threadIdx.x < len)
        sm.xlast[threadIdx.x] = (int32_t)umin(U[(size_t)(i0 + threadIdx.x) * ldU + hU], INF);
    // Short upper strips (hU + len + 1 <= kUW): the LDS window holds whole
    // D_U rows (origin k = 0), so its copy needs no tile end and travels with
    // the tile-end loads.
    constexpr int32_t UW = C::kUW;
    const bool full = hU + len + 1 <= UW;
    if (full) bracket_copy_u<C>(sm, U, ldU, hU, i0, len, 0, INF);
    // Tile ends, in every wave: lane l holds k*(i0, j0 + l + 64 c) and
    // k*(i1, j0 + l + 64 c); wave 0 also stores them (and the ends' values)
    // in LDS.  Reachability from i0 is a prefix of the weights.
    int32_t kA[NE], kB[NE];
    bool live = false;
    int32_t kbl = -1;  // k*(i1, jl), jl the last weight reachable from i0
#pragma unroll
    for (int c = 0; c < NE; ++c) {
        const int32_t jj = lane + c * kWave;
        const bool lend = jj < js;
        kA[c] = lend ? Ka[j0 + jj] : -1;
        kB[c] = lend ? Kb[j0 + jj] : -1;
    }
#pragma unroll
    for (int c = 0; c < NE; ++c) {
        const unsigned long long lv = __ballot(kA[c] >= 0);
        if (lv) {  // wave-uniform
            live = true;
            kbl = __shfl(kB[c], 63 - __clzll((long long)lv), kWave);
        }
    }
    const int32_t ka0 = __shfl(kA[0], 0, kWave);  // k*(i0, j0)
    if (threadIdx.x < kWave) {
#pragma unroll
        for (int c = 0; c < NE; ++c) {
            const int32_t jj = lane + c * kWave;
            if (jj < js) {
                stk(sm, jj, kA[c]);
                stk(sm, len * S + jj, kB[c]);
                sm.v[jj] = (typename C::St)umin(G[(size_t)i0 * H + j0 + jj], INF);
                sm.v[len * S + jj] = (typename C::St)umin(G[(size_t)(i0 + len) * H + j0 + jj], INF);
            }
        }
    }
    if (threadIdx.x < 2) sm.qn[threadIdx.x] = 0;
    if (threadIdx.x < kCoarseItems) sm.key[threadIdx.x] = ~0ull;
    if (!live) {  // nothing reachable from i0: the whole block is unreachable
        for (int32_t e = threadIdx.x; e < (len - 1) * S; e += kBlock) {
            const int32_t t = 1 + e / S, jj = e - (t - 1) * S;
            if (jj < js) G[(size_t)(i0 + t) * H + j0 + jj] = INF;
        }
        if ((jn > S) && threadIdx.x >= 1 && (int32_t)threadIdx.x < len)
            G[(size_t)(i0 + threadIdx.x) * H + j0 + S] = L[(size_t)sm.xlast[threadIdx.x] * ldL + (j0 + S - hU)];
        __syncthreads();
        return;
    }
    const bool lds_u = full || ((kbl >= 0) && (kbl - ka0 + len + 1 <= UW));
    const int32_t ubase = full ? 0 : ka0;
    // the D_U parallelogram (all rows: an idle output reads row 0)
    if (lds_u && !full) bracket_copy_u<C>(sm, U, ldU, hU, i0, len, ka0, INF);
    if ((jn > S) && threadIdx.x >= 1 && (int32_t)threadIdx.x < len)
        G[(size_t)(i0 + threadIdx.x) * H + j0 + S] = L[(size_t)sm.xlast[threadIdx.x] * ldL + (j0 + S - hU)];
    __syncthreads();
    if (lds_u)
        bracket_levels<C, true, kCoop>(sm, U, hU, L, hL, G, n, i0, len, j0, js, ubase);
    else
        bracket_levels<C, false, kCoop>(sm, U, hU, L, hL, G, n, i0, len, j0, js, ubase);
    // the block's outputs, tile vertices 1..len-1 x weights j0..j0+js-1, leave
    // LDS as contiguous row segments
    for (int32_t e = threadIdx.x; e < (len - 1) * S; e += kBlock) {
        const int32_t t = 1 + e / S, jj = e - (t - 1) * S;
        if (jj < js) G[(size_t)(i0 + t) * H + j0 + jj] = (int32_t)sm.v[t * S + jj];
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
// Semi-local query: LCS(a, b[i:k]) = the largest j with D_top(i, j) <= k
// (D_top(i, .) is strictly increasing on its finite prefix and
// D_top(i, 0) = i).  top: (n+2) x (m+1); m = 0 (no matrix) answers 0.
__device__ __forceinline__ int32_t semilocal_query(const int32_t *__restrict__ top, int32_t m,
                                                   int32_t n, int32_t i, int32_t k) {
    if (i < 0 || k < i || k > n) return -1;
    if (m == 0) return 0;
    const int32_t *__restrict__ row = top + (size_t)i * (size_t)(m + 1);
    int32_t lo = 0, hi = m;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (row[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Path listing of grid row r from the canonical witness (a_idx sorted, L
// pairs): t = matches above row r (binary search); the path enters at the
// column after the previous match and leaves at the column of row r's own
// match, or where it entered (a vertical step), or at n on the last row.
__device__ __forceinline__ void path_row(const int32_t *__restrict__ a_idx,
                                         const int32_t *__restrict__ b_idx, int32_t L, int32_t m,
                                         int32_t n, int32_t r, int32_t *cin, int32_t *cout) {
    int32_t lo = 0, hi = L;  // first t with a_idx[t] >= r
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (a_idx[mid] < r)
            lo = mid + 1;
        else
            hi = mid;
    }
    const int32_t c0 = lo > 0 ? imin(imax(b_idx[lo - 1] + 1, 0), n) : 0;
    int32_t c1 = c0;
    if (lo < L && a_idx[lo] == r) c1 = imin(imax(b_idx[lo], c0), n);
    if (r == m) c1 = n;
    *cin = c0;
    *cout = c1;
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
// nm_x[p] for a live lane, n + 1 otherwise: from the LDS window [s, s + W)
// (W >= 1), from the global table past it.  The LDS read is unconditional and
// the global one sits behind a wave-uniform branch: as the two arms of one
// select, the compiler merges them into a single flat load, which waits on
// both memory counters in every row of the dependent chain.
// The window holds int32 or, when n + 1 <= 65535, 16-bit entries (TT).
template <typename TT>
__device__ __forceinline__ int32_t leaf_lookup(bool live, int32_t x, int32_t p, int32_t s, int32_t n,
                                               const TT *tab, int32_t W,
                                               const int32_t *__restrict__ nm) {
    const int32_t q = imin(imax(p - s, 0), W - 1);
    int32_t cd = (int32_t)tab[(live ? x : 0) * W + q];  // inside the window for every lane
    if (!live) cd = n + 1;
    const bool far = live && p - s >= W;
    if (__ballot(far) != 0ull) {
        if (far) cd = nm[(size_t)x * (n + 2) + p];
        // use the value here, so that the wait for this load stays inside the
        // rare branch: at the merge the counter of vector memory operations also
        // covers the row stores of the tall leaf, and every row would wait for them
        asm volatile("" : "+v"(cd));
    }
    return cd;
}

// Midpoint trace inside a base strip of h <= H0 rows.  The breakout rows of
// the single source s after each appended row, D_r(s, .) for r = 0..h, are
// recomputed into LDS; the walk then goes back from (h, w, e): at row r the
// split with the smaller upper weight is the one where row r-1 contributes a
// match, taken when nm_{a[r-1]}[D_{r-1}(s, w-1)] == e (match (row0 + r - 1,
// e - 1)); otherwise the path enters row r at the same column.  Matches are
// written at witness offsets off .. off + w - 1 in increasing order; wcap
// (= min(m, n)) bounds every write.
// lds: (H0+1)*(H0+1) int32.
template <int H0, bool kFast = false>
__device__ void trace_leaf_block(const uint8_t *__restrict__ arow, int32_t h, int32_t n,
                                 int32_t sigma, const int32_t *__restrict__ nm, int4 node,
                                 int32_t row0, int32_t *__restrict__ a_idx,
                                 int32_t *__restrict__ b_idx, int32_t wcap, int32_t *err,
                                 int32_t *lds, int32_t *tab = nullptr, int32_t tabcap = 0) {
    const int32_t INF = n + 1;
    const int32_t s = umin(node.x, n);
    const int32_t S = H0 + 1;
    const int32_t tid = threadIdx.x;
    if constexpr (kFast) {
        // One wave (blockDim = kWave); lane l owns column l + 1 of the row
        // vector D_r(s, .), in a register; column 0 is s.  Columns
        // s .. s+W-1 of every symbol's next-match table are in LDS (lookups
        // at or past s + W read the global table).  Appending row r: the
        // column to the left comes from the neighbouring lane, the candidate
        // from the table, and the lanes where the candidate gives the new
        // value form the row's match mask (a ballot), kept by lane r.  The
        // walk back (Section II-C, the smaller upper weight first) then only
        // needs those masks: at row r with weight w it takes the match when
        // bit w - 1 of the mask is set, and the matched rows are written out
        // by their lanes afterwards, with D_r(s, w) read from LDS.
        static_assert(H0 <= kWave, "one lane per column");
        // Only weights up to w0 and columns up to e = D_h(s, w0) matter (as in
        // trace_leaf_pipe below): lookups from columns past e are skipped, so
        // the table window [s, e] serves every lookup when it fits.
        const int32_t w0c = imin(imax(node.y, 0), h);
        const int32_t eend = imin(imax(node.z, s), n + 1);
        const int32_t pmax = imin(eend, n);
        const int32_t W = imin(imin(n + 2 - s, tabcap / imax(sigma, 1)), eend - s + 1);
        for (int32_t x = 0; x < sigma; ++x) {
            const int32_t *src = nm + (size_t)x * (n + 2) + s;
            int32_t *dst = tab + x * W;
            for (int32_t c0 = 0; c0 < W; c0 += 8 * kWave) {
                int32_t v[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) v[t] = src[imin(c0 + t * kWave + tid, W - 1)];
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (c0 + t * kWave + tid < W) dst[c0 + t * kWave + tid] = v[t];
            }
        }
        const int32_t xrow = (tid < h) ? (int32_t)arow[tid] : 0;  // row symbols, one per lane
        const int32_t j = tid + 1;
        int32_t d = INF;                      // D_r(s, j)
        uint32_t mlo = 0, mhi = 0;            // lane r: match mask of row r + 1
        __syncthreads();                      // table in LDS
        for (int32_t r = 0; r < h; ++r) {
            const int32_t x = __builtin_amdgcn_readlane(xrow, r);
            // D_r(s, j - 1): lane l - 1's value by a whole-wave DPP shift
            // (wave_shr:1); lane 0 keeps `s`, column 0
            const int32_t p = __builtin_amdgcn_update_dpp(s, d, 0x138, 0xF, 0xF, false);
            const bool live = (j <= w0c) && (x < sigma) && (p <= pmax);
            const int32_t cd = leaf_lookup(live, x, p, s, n, tab, W, nm);
            const int32_t dn = umin(d, cd);
            const bool hit = live && (cd == dn);
            const unsigned long long mk = __ballot(hit);
            if (tid == r) {
                mlo = (uint32_t)mk;
                mhi = (uint32_t)(mk >> 32);
            }
            d = (j <= w0c) ? dn : INF;
            if (j <= h) lds[(r + 1) * S + j] = d;
        }
        // walk: uniform over the wave; lane w - 1 notes the row that matched
        // weight w
        const int32_t w0 = imin(imax(node.y, 0), h);
        const int32_t off = imax(node.w, 0);
        int32_t w = w0, mrow = 0;
        for (int32_t r = h; r >= 1 && w >= 1; --r) {
            const uint32_t lo = __builtin_amdgcn_readlane(mlo, r - 1);
            const uint32_t hi = __builtin_amdgcn_readlane(mhi, r - 1);
            const unsigned long long mk = ((unsigned long long)hi << 32) | lo;
            if ((mk >> (w - 1)) & 1ull) {
                if (tid == w - 1) mrow = r;
                --w;
            }
        }
        __syncthreads();  // LDS rows written above are read by other lanes
        const int32_t dend = (w0 >= 1) ? lds[h * S + w0] : s;
        if (tid == 0 && (w != 0 || dend != node.z)) atomicOr(err, kErrTrace);
        if (w == 0 && j <= w0 && mrow >= 1 && off + j <= wcap) {
            a_idx[off + j - 1] = row0 + mrow - 1;
            b_idx[off + j - 1] = lds[mrow * S + j] - 1;
        }
        __syncthreads();
        return;
    }
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

// ---------------------------------------------------------------------------
// Midpoint trace inside a base strip of up to 64 E rows (E = Ew K = 2, 4 or 8
// registers of columns), by K waves: the row appends of the one-wave form
// above with column j = 64 e + lane + 1 in register e (wave k holds registers
// Ew k .. Ew k + Ew - 1), restricted to the weights 1..w0 of the node.
// Column j of D_{r+1}(s, .) depends only on columns j - 1 and j of D_r(s, .),
// and the walk reads no weight above w0, so every lookup index is at most
// e = D_h(s, w0) and a table window [s, e] serves all of them when it fits in
// LDS (lookups past the window read the global table).  The row appends
// store each row's match masks and values in the strip's global scratch
// (leaf_scratch_bytes); the walk back picks the row where each weight matched
// and the weight's column is read from that row's stored values (their
// column - 1 is the match in b).
// The waves run as a pipeline: appending row r in wave k needs D_r(s, .) of
// the column just left of its own, which wave k - 1 holds.  Wave k - 1 stores
// that value for every row in an LDS ring and publishes its progress every
// kLeafLag rows; wave k runs at least kLeafLag rows behind it (a bounded
// wait: past kSpinLimit polls the trace reports kErrTrace).
// LDS: tab (tabcap entries of TT: int32, or 16 bits when n + 1 <= 65535, which
// doubles the window's columns in the same 64 KB: at 16384 columns and 20
// symbols 1638 columns instead of 819, more than a 1024-row strip's path
// spans), mrow and xs (64 E int32 each), ring ((K - 1) 64 E int32), sync
// (K + 2 int32).
constexpr int32_t kLeafTabTall = 16384;  // int32 next-match entries a tall leaf keeps in LDS, at most
__host__ __device__ inline int32_t leaf_tab_cap(int32_t sigma, int32_t n, int32_t entry_bytes = 4) {
    const int64_t all = (int64_t)(sigma < 1 ? 1 : sigma) * (n + 2);
    const int64_t cap = (int64_t)kLeafTabTall * 4 / entry_bytes;
    return (int32_t)(all < cap ? all : cap);
}
constexpr int32_t kLeafLag = 8;
constexpr uint32_t kLeafSpinLimit = 1u << 22;

// One row append for this wave's Ew registers; carry = D_r(s, jbase), the
// column left of the wave's first (s for the first wave).  The row's symbol x
// is uniform, and so is its window row trow (row 0 for a symbol outside the
// alphabet, xok false: then no lane is live).  Every register's LDS lookup is
// issued before one wave-uniform test for lookups past the window (kFar:
// compiled in only when the window can be shorter than the leaf's column
// range; their global reads wait inside that rare branch), so a row costs one
// LDS round trip whatever Ew.  A weight above wmax is never live, so its entry
// stays n + 1 without a select.
template <int Ew, typename TT, bool kFar>
__device__ __forceinline__ void leaf_row(int32_t (&d)[Ew], int32_t carry, int32_t jbase, int32_t x,
                                         bool xok, const TT *trow, int32_t s, int32_t n, int32_t wmax,
                                         int32_t pmax, int32_t W, const int32_t *__restrict__ nm,
                                         unsigned long long (&mk)[Ew]) {
    const int lane = __lane_id();
    const int32_t INF = n + 1;
    int32_t p[Ew];  // D_r(s, j - 1): the next lower column, across lanes and registers
#pragma unroll
    for (int e = 0; e < Ew; ++e) {
        const int32_t c = (e == 0) ? carry : __builtin_amdgcn_readlane(d[e > 0 ? e - 1 : 0], kWave - 1);
        p[e] = __builtin_amdgcn_update_dpp(c, d[e], 0x138, 0xF, 0xF, false);  // wave_shr:1
    }
    int32_t cd[Ew];
    bool live[Ew];
#pragma unroll
    for (int e = 0; e < Ew; ++e) {
        const int32_t j = jbase + e * kWave + lane + 1;
        live[e] = j <= wmax && xok && p[e] <= pmax;
        cd[e] = (int32_t)trow[imin(imax(p[e] - s, 0), W - 1)];  // inside the window for every lane
    }
    if constexpr (kFar) {
        bool far[Ew];
        bool anyfar = false;
#pragma unroll
        for (int e = 0; e < Ew; ++e) {
            far[e] = live[e] && p[e] - s >= W;
            anyfar |= far[e];
        }
        if (__ballot(anyfar) != 0ull) {
            const int32_t *__restrict__ grow = nm + (size_t)x * (n + 2);
#pragma unroll
            for (int e = 0; e < Ew; ++e) {
                if (far[e]) cd[e] = grow[p[e]];
                asm volatile("" : "+v"(cd[e]));  // the wait for these loads stays in this branch
            }
        }
    }
#pragma unroll
    for (int e = 0; e < Ew; ++e) {
        const int32_t c = live[e] ? cd[e] : INF;
        const int32_t dn = umin(d[e], c);
        mk[e] = __ballot(live[e] && c == dn);
        d[e] = dn;
    }
}

template <int Ew, int K, typename TT>
__device__ void trace_leaf_pipe(const uint8_t *__restrict__ arow, int32_t h, int32_t n,
                                int32_t sigma, const int32_t *__restrict__ nm, int4 node,
                                int32_t row0, int32_t *__restrict__ a_idx,
                                int32_t *__restrict__ b_idx, int32_t wcap, int32_t *err,
                                TT *tab, int32_t tabcap, uint8_t *scratch, int32_t *mrow,
                                int32_t *xs, int32_t *ring, int32_t *sync) {
    constexpr int32_t E = Ew * K;
    constexpr int32_t RH = E * kWave;  // ring entries per wave boundary (>= h)
    constexpr int32_t NT = K * kWave;
    // global scratch of this strip: masks[r E + e], then rows[r RH + j - 1] = D_{r+1}(s, j)
    unsigned long long *masks = reinterpret_cast<unsigned long long *>(scratch);
    int32_t *rows = reinterpret_cast<int32_t *>(scratch + (size_t)RH * E * 8);
    const int32_t INF = n + 1;
    const int32_t s = umin(node.x, n);
    const int lane = __lane_id();
    const int32_t tid = threadIdx.x;
    const int32_t wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int32_t jbase = wv * Ew * kWave;  // this wave: columns jbase + 1 .. jbase + 64 Ew
    const int32_t w0 = imin(imax(node.y, 0), h);
    const int32_t off = imax(node.w, 0);
    const int32_t eend = imin(imax(node.z, s), n + 1);
    // Values above e = D_h(s, w0) are never on the path, and a value <= e never
    // comes from one above e (next-match columns only grow), so lookups from
    // columns past e are skipped: those entries become n + 1 and every entry
    // <= e, and every match bit of a weight <= w0 at a column <= e, is unchanged.
    const int32_t pmax = imin(eend, n);
    const int32_t W = imin(imin(eend - s + 1, n + 2 - s), tabcap / imax(sigma, 1));
    for (int32_t x = 0; x < sigma; ++x) {
        const int32_t *src = nm + (size_t)x * (n + 2) + s;
        TT *dst = tab + x * W;
        for (int32_t c0 = 0; c0 < W; c0 += 8 * NT) {
            int32_t v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = src[imin(c0 + t * NT + tid, W - 1)];
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (c0 + t * NT + tid < W) dst[c0 + t * NT + tid] = (TT)v[t];
        }
    }
    for (int32_t r = tid; r < E * kWave; r += NT) {
        xs[r] = (r < h) ? (int32_t)arow[r] : 0;
        mrow[r] = 0;
    }
    if (tid < K) sync[tid] = 0;
    __syncthreads();
    int32_t d[Ew];
#pragma unroll
    for (int e = 0; e < Ew; ++e) d[e] = INF;
    int32_t stall = 0;  // wave-uniform
    int32_t avail = 0;  // rows of the wave to the left published so far (wave-uniform)
    // Rows go in runs of 64 (lane l holds the run's row symbol l and gathers
    // row l's match masks, written out per run) and each run in groups of
    // kLeafLag rows, the same partition in every wave: a wave waits for and
    // reads the left wave's ring values once per group, and publishes its own
    // group before appending the group's last row.  Inside a group a row is
    // straight-line code: the values handed on, the masks and the ring values
    // are gathered with selects.
    // lookups past the window only when it can be shorter than the columns
    // the leaf reads (pmax - s + 1 of them)
    const bool need_far = W < pmax - s + 1;
    for (int32_t rb = 0; rb < h; rb += kWave) {
        const int32_t xr = xs[rb + lane];
        const int32_t rn = imin(kWave, h - rb);
        const unsigned long long xokm = __ballot(xr < sigma);  // bit l: row rb + l's symbol is valid
        const int32_t xo = (xr < sigma ? xr : 0) * W;          // its window row
        uint32_t mlo[Ew], mhi[Ew];
#pragma unroll
        for (int e = 0; e < Ew; ++e) mlo[e] = mhi[e] = 0u;
        int32_t rv = INF;  // lane l: D_{rb+l}(s, last column of this wave)
        for (int32_t g0 = 0; g0 < rn; g0 += kLeafLag) {
            const int32_t r0 = rb + g0;
            const int32_t gn = imin(kLeafLag, rn - g0);
            int32_t win = INF;  // lane q < gn: D_{r0+q}(s, jbase) from the wave to the left
            if (wv > 0) {
                const int32_t want = r0 + gn;
                if (avail < want) {
                    int32_t got = __builtin_amdgcn_readfirstlane(
                        __hip_atomic_load(sync + wv - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                    uint32_t spins = 0;
                    while (got < want) {
                        __builtin_amdgcn_s_sleep(1);
                        if (++spins > kLeafSpinLimit) {
                            stall = 1;
                            got = h;
                            break;
                        }
                        got = __builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(sync + wv - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    avail = __builtin_amdgcn_readfirstlane(got);
                }
                if (lane < gn) win = ring[(wv - 1) * RH + r0 + lane];
            }
            for (int32_t q = 0; q < gn; ++q) {
                const int32_t r = r0 + q;
                const int32_t rr = g0 + q;
                if (wv < K - 1) {  // D_r(s, last column) for the wave to the right
                    const int32_t last = __builtin_amdgcn_readlane(d[Ew - 1], kWave - 1);
                    rv = (lane == rr) ? last : rv;
                    if (q == gn - 1) {
                        if (lane >= g0 && lane <= rr) ring[wv * RH + rb + lane] = rv;
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                        if (lane == 0)
                            __hip_atomic_store(sync + wv, r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
                const int32_t carry = (wv > 0) ? __builtin_amdgcn_readlane(win, q) : s;
                unsigned long long mk[Ew];
                const int32_t x = __builtin_amdgcn_readlane(xr, rr);
                const bool xok = (xokm >> rr) & 1ull;
                const TT *trow = tab + __builtin_amdgcn_readlane(xo, rr);
                if (need_far)
                    leaf_row<Ew, TT, true>(d, carry, jbase, x, xok, trow, s, n, w0, pmax, W, nm, mk);
                else
                    leaf_row<Ew, TT, false>(d, carry, jbase, x, xok, trow, s, n, w0, pmax, W, nm, mk);
#pragma unroll
                for (int e = 0; e < Ew; ++e) {
                    rows[(size_t)r * RH + jbase + e * kWave + lane] = d[e];
                    mlo[e] = (lane == rr) ? (uint32_t)mk[e] : mlo[e];
                    mhi[e] = (lane == rr) ? (uint32_t)(mk[e] >> 32) : mhi[e];
                }
            }
        }
        if (lane < rn) {
#pragma unroll
            for (int e = 0; e < Ew; ++e)
                masks[(rb + lane) * E + wv * Ew + e] = ((unsigned long long)mhi[e] << 32) | mlo[e];
        }
    }
    if (stall != 0 && lane == 0) atomicOr(err, kErrTrace);
    if (w0 >= 1 && ((w0 - 1) >> 6) / Ew == wv) {  // the wave holding column w0: D_h(s, w0)
        const int32_t er = ((w0 - 1) >> 6) - wv * Ew;
        int32_t v = INF;
#pragma unroll
        for (int e = 0; e < Ew; ++e)
            if (e == er) v = __builtin_amdgcn_readlane(d[e], (w0 - 1) & (kWave - 1));
        if (lane == 0) sync[K] = v;
    }
    __syncthreads();  // every wave's masks and rows stored
    if (wv == 0) {
        int32_t w = w0;
        for (int32_t rb = ((h - 1) / kWave) * kWave; rb >= 0 && w >= 1; rb -= kWave) {
            uint32_t mlo[E], mhi[E];  // lane l: the masks of row rb + l
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const unsigned long long m = (rb + lane < h) ? masks[(size_t)(rb + lane) * E + e] : 0ull;
                mlo[e] = (uint32_t)m;
                mhi[e] = (uint32_t)(m >> 32);
            }
            // the mask word of weight w only changes when w crosses a multiple of
            // 32: select it (a dynamic register index) only then
            int32_t half = -1;
            uint32_t cur = 0;
            for (int32_t r = imin(h, rb + kWave); r > rb && w >= 1; --r) {
                const int32_t hw = (w - 1) >> 5;
                if (hw != half) {
                    half = hw;
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        if (e == (hw >> 1)) cur = (hw & 1) ? mhi[e] : mlo[e];
                }
                const uint32_t word = (uint32_t)__builtin_amdgcn_readlane((int32_t)cur, r - 1 - rb);
                if ((word >> ((w - 1) & 31)) & 1u) {
                    if (lane == 0) mrow[w - 1] = r;
                    --w;
                }
            }
        }
        const int32_t dend = (w0 >= 1) ? sync[K] : s;
        if (lane == 0) {
            if (w != 0 || dend != node.z) atomicOr(err, kErrTrace);
            sync[K + 1] = w;
        }
    }
    __syncthreads();
    if (sync[K + 1] != 0 || w0 == 0) return;
    // weight j matched in row mrow[j - 1]; its column is D of that row - 1
#pragma unroll
    for (int e = 0; e < Ew; ++e) {
        const int32_t j = jbase + e * kWave + lane + 1;
        const int32_t mr = (j <= w0) ? mrow[j - 1] : 0;
        if (j <= w0 && mr >= 1 && off + j <= wcap) {
            a_idx[off + j - 1] = row0 + mr - 1;
            b_idx[off + j - 1] = rows[(size_t)(mr - 1) * RH + j - 1] - 1;
        }
    }
}

}  // namespace lcs
