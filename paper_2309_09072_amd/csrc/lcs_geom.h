// Geometry of the strip recursion, shared by the host planner and the kernels.
//
// The grid of a (m rows) x b (n columns) is cut into base strips of h0 rows
// (the last one may be shorter).  Level 0 holds the base strips; strip s of
// level l+1 is the combine of strips 2s and 2s+1 of level l, or -- when level l
// has an odd number of strips -- its last strip carried up unchanged (the
// same matrix, no copy).  The top level has one strip: the whole grid.
//
// Every strip of h rows owns one breakout matrix D (Section II-B-1) stored
// row-major as (n + 2) x (h + 1) int32: row i = top vertex i (0..n), column
// j = path weight, and a last all-unreachable sentinel row n + 1 so that a
// lookup D(x, .) with x = n + 1 ("unreachable") needs no branch.  Only the last
// strip of a level can be shorter than the others, so strip q of a level sits
// at base + q * (n + 2) * (hfull + 1) unless it is the last one.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace lcs {

// error bits of the workspace header word 0
constexpr int32_t kErrSymbol = 1;  // a symbol >= alphabet was read
constexpr int32_t kErrTrace = 2;   // the trace found no split reproducing a breakout

struct LevelGeom {
    int32_t nstrips;     // strips at this level
    int32_t hfull;       // rows of every strip except possibly the last
    int32_t hlast;       // rows of the last strip
    int32_t npairs;      // combines producing this level (0 at level 0)
    int32_t last_alias;  // 1: last strip is the lower level's last strip
    int64_t base;        // byte offset of strip 0 inside the workspace
    int64_t last_off;    // byte offset of the last strip's matrix
    int64_t bytes;       // bytes owned by this level (aliased strip excluded)
};

// Arguments of one combine level, passed by value to the kernels.
struct CombineArgs {
    const int32_t *cbase;  // child level: strip 0
    const int32_t *clast;  // child level: last strip
    int32_t hc;            // child full strip rows
    int32_t hclast;        // child last strip rows
    int32_t nc;            // child strip count
    int32_t *pbase;        // parent level: strip 0
    int32_t *plast;        // parent level: last strip
    int32_t np;            // parent strip count
    int32_t n;             // columns of the grid
    int32_t tile;          // vertices per search tile (anchors every `tile` vertices)
    int32_t nanch;         // anchors per pair = ceil(n / tile) + 1
    int32_t hs;            // anchor scratch row stride = 2 * hc + 1
    int32_t *anch;         // anchor argmins [pair][anchor][hs]
    int32_t jchunk;        // weights per bracket block
    int32_t nchunks;       // bracket blocks along the weights of the widest pair
};

// Every split level of a witness trace, for one launch (levels 1..top).
constexpr int kTraceMaxLev = 32;  // more than any layout has (fewer than 2^30 cells per matrix)
struct TraceSplitArgs {
    CombineArgs lev[kTraceMaxLev];  // lev[l]: the combine of level l
    int4 *node[kTraceMaxLev];       // node[l]: trace nodes of level l (one per strip)
    int32_t top;                    // top level
    int32_t *err;
};
static_assert(sizeof(TraceSplitArgs) <= 4096, "kernel arguments are limited to 4 KB");

struct StripRef {
    const int32_t *d;
    int32_t h;
};

#if defined(__HIPCC__) || defined(__HIP_DEVICE_COMPILE__)
#define LCS_HD __host__ __device__ __forceinline__
#else
#define LCS_HD inline
#endif

LCS_HD size_t strip_elems(int32_t n, int32_t h) { return (size_t)(n + 2) * (size_t)(h + 1); }

// Column segments (work-groups) per strip for the combing of a single pair's
// base strips: several when the strips are tall and few (then one work-group
// per strip would leave most of the chip idle), each 1024 columns (four waves
// of 4 packed columns per lane); 1 otherwise.  From 256 rows (4096²: 16
// strips of 256 rows combed in 0.145 ms with 4 segments each, 0.160 ms with
// one pipelined work-group per strip).
LCS_HD int32_t comb_segments(int32_t n, int32_t nstrips, int32_t h0) {
    if (h0 < 256 || n < 4096 || n > 32767 || nstrips * 8 > 256) return 1;
    const int32_t g = (n + 1023) / 1024;
    return g < 32 ? g : 32;
}

// Scratch of the trace inside one base strip of h0 > 64 rows (E = h0 / 64
// registers of columns): the match masks of every row (h0 E u64), then the
// row values D_r(s, 1..64 E) of every row r = 1..h0 (int32); 0 for h0 <= 64.
LCS_HD int64_t leaf_scratch_bytes(int32_t h0) {
    if (h0 <= 64) return 0;
    const int64_t E = (h0 + 63) / 64;
    return ((int64_t)h0 * E * 8 + (int64_t)h0 * 64 * E * 4 + 255) & ~(int64_t)255;
}

LCS_HD StripRef child_strip(const CombineArgs &c, int32_t q) {
    StripRef r;
    if (q < c.nc - 1) {
        r.d = c.cbase + (size_t)q * strip_elems(c.n, c.hc);
        r.h = c.hc;
    } else {
        r.d = c.clast;
        r.h = c.hclast;
    }
    return r;
}

LCS_HD int32_t *parent_strip(const CombineArgs &c, int32_t p) {
    return (p < c.np - 1) ? c.pbase + (size_t)p * strip_elems(c.n, 2 * c.hc) : c.plast;
}

// Work-groups go to the chip's 8 XCDs (each with its own L2) round-robin by
// linear id.  xcd_block maps the linear id b of N blocks to a logical block so
// that each XCD runs groups of g consecutive logical blocks; blocks of an
// incomplete last round keep their id.  With g = N / 8 every XCD gets one
// contiguous range.
LCS_HD int32_t xcd_block(int32_t b, int32_t N, int32_t g) {
    constexpr int32_t X = 8;
    if (g <= 1) return b;
    const int32_t full = (N / (X * g)) * (X * g);
    if (b >= full) return b;
    const int32_t x = b % X, q = b / X;
    return ((q / g) * X + x) * g + (q % g);
}

LCS_HD int32_t anchor_vertex(int32_t a, int32_t tile, int32_t n) {
    int64_t v = (int64_t)a * tile;
    return v < n ? (int32_t)v : n;
}

}  // namespace lcs
