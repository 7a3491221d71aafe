// Host-side planning of the strip recursion: workspace layout and per-level
// kernel arguments.  Shared by the single-pair API, the batch runner and the
// serving loop.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "lcs_geom.h"

namespace lcs {

constexpr int32_t kDefaultBaseRows = 64;
constexpr int32_t kDefaultTile = 32;
constexpr int32_t kHeaderWords = 64;  // hdr[0] error bits, hdr[1] L, hdr[2] end column

struct Layout {
    int32_t m = 0, n = 0, sigma = 0, h0 = 0, tile = 0;
    std::vector<LevelGeom> lev;      // level 0 = base strips, back() = whole grid
    std::vector<int64_t> node_off;   // per level: trace nodes (int4 per strip)
    std::vector<int64_t> anch_off;   // per level: anchor argmin rows of its combines
    int64_t off_hdr = 0, off_nm = 0, total = 0;
    int64_t off_rev = -1;  // reversed strings of an oriented build (rows, then columns)
    int64_t off_comb = 0;  // per base strip: the combed seaweeds (bot[n], pos[n], right[h0])
    int32_t comb_stride = 0;  // int32 per base strip in that region
    int64_t off_rec = 0;      // segment hand-off records of the combing (u64), and their
    int32_t rec_words = 0;    // size in int32 words (cleared before every combing)
    int64_t off_leaf = 0;     // per base strip of more than 64 rows: the trace leaf's
    int64_t leaf_stride = 0;  // match masks and rows (leaf_scratch_bytes), 0 otherwise
    int32_t nanch = 0;
};

inline int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Workspace layout for one pair of sizes (m, n).  Returns false when a strip
// matrix would have 2^30 or more cells or n + 2 >= 2^24.
inline bool make_layout(int32_t m, int32_t n, int32_t sigma, int32_t h0, int32_t tile, Layout &L) {
    L = Layout();
    L.m = m;
    L.n = n;
    L.sigma = sigma;
    L.h0 = h0;
    L.tile = tile;
    // every matrix has fewer than 2^30 cells, so a byte offset inside one fits in 32 bits
    if ((int64_t)(n + 2) * (int64_t)(m + 1) >= ((int64_t)1 << 30)) return false;
    // a row index (at most n + 1) and a row length are 24-bit factors of a cell index
    if (n + 2 >= (1 << 24)) return false;
    int64_t off = 0;
    L.off_hdr = off;
    off += 4 * kHeaderWords;
    L.off_nm = off;
    off = align256(off + 4 * (int64_t)sigma * (n + 2));
    if (m > 0 && n > 0) {
        LevelGeom g{};
        g.nstrips = (m + h0 - 1) / h0;
        g.hfull = h0;
        g.hlast = m - (g.nstrips - 1) * h0;
        g.base = off;
        g.last_off = off + 4 * (int64_t)(g.nstrips - 1) * (int64_t)strip_elems(n, h0);
        g.bytes = 4 * ((int64_t)(g.nstrips - 1) * (int64_t)strip_elems(n, h0) +
                       (int64_t)strip_elems(n, g.hlast));
        off = align256(off + g.bytes);
        L.lev.push_back(g);
        L.comb_stride = (2 * n + h0 + 63) & ~63;
        L.off_comb = off;
        off = align256(off + 4 * (int64_t)g.nstrips * L.comb_stride);
        {
            const int32_t G = comb_segments(n, g.nstrips, h0);
            L.rec_words = 2 * g.nstrips * (G - 1) * h0;
            L.off_rec = off;
            off = align256(off + 4 * (int64_t)L.rec_words);
        }
        L.leaf_stride = leaf_scratch_bytes(h0);
        L.off_leaf = off;
        off = align256(off + (int64_t)g.nstrips * L.leaf_stride);
        while (L.lev.back().nstrips > 1) {
            const LevelGeom pv = L.lev.back();
            LevelGeom q{};
            const int32_t nc = pv.nstrips;
            q.nstrips = (nc + 1) / 2;
            q.npairs = nc / 2;
            q.hfull = 2 * pv.hfull;
            q.base = off;
            const int64_t full = (int64_t)strip_elems(n, q.hfull);
            if (nc % 2) {
                q.hlast = pv.hlast;
                q.last_alias = 1;
                q.last_off = pv.last_off;
                q.bytes = 4 * (int64_t)(q.nstrips - 1) * full;
            } else {
                q.hlast = pv.hfull + pv.hlast;
                q.last_alias = 0;
                q.last_off = off + 4 * (int64_t)(q.nstrips - 1) * full;
                q.bytes = 4 * ((int64_t)(q.nstrips - 1) * full + (int64_t)strip_elems(n, q.hlast));
            }
            off = align256(off + q.bytes);
            L.lev.push_back(q);
        }
        // One region per level: in a persistent launch, combines of two levels
        // can be in flight at the same time.
        L.nanch = (n + tile - 1) / tile + 1;
        L.anch_off.push_back(0);
        for (size_t l = 1; l < L.lev.size(); ++l) {
            L.anch_off.push_back(off);
            off = align256(off + 4 * (int64_t)L.lev[l].npairs * L.nanch * (2 * L.lev[l - 1].hfull + 1));
        }
        for (size_t l = 0; l < L.lev.size(); ++l) {
            L.node_off.push_back(off);
            off = align256(off + 16 * (int64_t)L.lev[l].nstrips);
        }
    }
    L.total = off;
    return true;
}

inline CombineArgs combine_args(const Layout &L, uint8_t *ws, size_t l) {
    const LevelGeom &c = L.lev[l - 1], &p = L.lev[l];
    CombineArgs a{};
    a.cbase = reinterpret_cast<const int32_t *>(ws + c.base);
    a.clast = reinterpret_cast<const int32_t *>(ws + c.last_off);
    a.hc = c.hfull;
    a.hclast = c.hlast;
    a.nc = c.nstrips;
    a.pbase = reinterpret_cast<int32_t *>(ws + p.base);
    a.plast = reinterpret_cast<int32_t *>(ws + p.last_off);
    a.np = p.nstrips;
    a.n = L.n;
    a.tile = L.tile;
    a.nanch = L.nanch;
    a.hs = 2 * c.hfull + 1;
    a.anch = reinterpret_cast<int32_t *>(ws + L.anch_off[l]);
    a.jchunk = 32;
    const int32_t H = 2 * c.hfull + 1;
    a.nchunks = (H - 1 + a.jchunk - 1) / a.jchunk;
    if (a.nchunks < 1) a.nchunks = 1;
    return a;
}

}  // namespace lcs
