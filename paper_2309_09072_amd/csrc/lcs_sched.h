// Task schedule of the persistent batch kernel, shared by the device (decode
// of a task number) and the host (construction of the per-pair records and of
// the task order, and a sequential simulation that checks the schedule
// without a GPU).
//
// Each pair's work is a list of stages in the dependency order of the method:
// next-match tables (one task per symbol), base strips (one task per strip and
// 256-vertex block), for every combine level its anchors (one per anchor
// vertex) then its bracketed tiles (one per tile and weight chunk), the
// length, the trace splits from the top level down, the base-strip traces.
// The global task order runs over waves of pairs (the pairs that hold the
// workspace slots at one time): inside a wave, step by step of the method, the
// stage of every pair of the wave that has this step, pair by pair.  A task
// waits only on counters raised by tasks of earlier stages in this order, never
// on a task of its own stage, so the kernel hands out chunks of consecutive
// tasks of one stage and synchronises once per chunk.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "lcs_geom.h"

namespace lcs {

constexpr int kMaxLev = 16;
constexpr int kMaxStages = 4 + 3 * kMaxLev;

enum Stage : int32_t {
    ST_EMPTY = 0,        // m == 0 or n == 0: length 0
    ST_ANCHOR = 3,       // one anchor vertex of one combine
    ST_LENGTH = 5,       // length + root trace node
    ST_SPLIT = 6,        // one trace split
    ST_LEAF = 7,         // trace inside one base strip
    ST_NM_SYM = 16,      // next-match table of one symbol (u = symbol)
    ST_BASE_BLK = 17,    // u = strip * vertex_blocks + block
    ST_BRACKET_CH = 18,  // u = (q * tiles + tile) * chunks + chunk
    // staged mode only (the persistent schedule never lists them):
    ST_COMB = 19,        // seaweed combing of one base strip (u = strip)
    ST_DGEN = 20,        // breakout rows of one run of vertices of one strip
    ST_LEAF_TALL = 21,   // trace inside one base strip of 128 to 512 rows
};

struct PairRec {
    int64_t ws_off;  // byte offset of this pair's slot in the workspace
    int64_t a_off, b_off, wit_off;
    int64_t off_hdr, off_nm, total;
    int64_t node_off[kMaxLev];
    int64_t anch_off[kMaxLev];
    LevelGeom lev[kMaxLev];
    int32_t ctr_lev[kMaxLev];  // first counter of level l (relative to ctr_base)
    int32_t stage_start[kMaxStages + 1];
    int32_t stage_kind[kMaxStages];
    int32_t stage_level[kMaxStages];
    int32_t nstages;
    int32_t ctr_base;
    int32_t m, n, nlev, nanch;
    int32_t ntasks, nctr;
    int32_t sigma;   // next-match tasks (one per symbol)
    int32_t nvb;     // 256-vertex blocks of a base strip
    int32_t jchunk;  // weights per bracket task
    int32_t h0;      // rows per base strip
    int32_t comb_stride;  // int32 per base strip in the combing region
    int64_t off_comb;     // the combing region (bot, pos, right per strip)
    int64_t off_leaf;     // the trace leaves' scratch (leaf_stride bytes per strip)
    int64_t leaf_stride;
};

// One stage of one pair in the global order, cut into chunks of at most
// `chunk` consecutive tasks: its chunks are numbered start, start + 1, ...
// The table is sorted by start.
struct Seg {
    int64_t start;  // global number of the stage's first chunk
    int32_t pair, stage;
};

LCS_HD int32_t stage_tasks(const PairRec &P, int32_t st) {
    return P.stage_start[st + 1] - P.stage_start[st];
}

// counters of a pair: [0] next-match done, [1] base-strip traces done, then
// per level l: strip_done[S_l], anc_done[S_l], node_done[S_l]
constexpr int32_t kCtrNm = 0, kCtrLeaves = 1, kCtrHead = 2;

struct Task {
    int32_t pair, kind, level, u;
    int32_t nwait, nsig;
    int32_t wait_idx[2], wait_tgt[2];  // absolute counter indices and targets
    int32_t sig_idx[2];
};

LCS_HD int32_t vertex_blocks_of(int32_t n, int32_t block) { return (n + 2 + block - 1) / block; }

// weight chunks of every bracket tile of level l (a full-height parent)
LCS_HD int32_t level_chunks_of(const PairRec &P, int32_t l) {
    const int32_t w = 2 * P.lev[l - 1].hfull;  // weights of a full-height parent, minus one
    const int32_t c = (w + P.jchunk - 1) / P.jchunk;
    return c > 1 ? c : 1;
}

// "the work of pair Q is over": its base-strip traces have all run, or its
// single empty-pair task has
LCS_HD int32_t pair_finish_target(const PairRec &Q) { return Q.nlev ? Q.lev[0].nstrips : 1; }

// counter index and target of "strip s of level l is complete", following
// carried-up strips down to the level that produced them
LCS_HD void strip_done_ctr(const PairRec &P, int32_t l, int32_t s, int32_t *idx, int32_t *tgt) {
    while (l > 0 && s == P.lev[l].nstrips - 1 && P.lev[l].last_alias) {
        s = 2 * s;
        --l;
    }
    *idx = P.ctr_base + P.ctr_lev[l] + s;
    // its base blocks, or its bracket tasks (tiles x weight chunks)
    *tgt = (l == 0) ? P.nvb : (P.nanch - 1) * level_chunks_of(P, l);
}

// the segment holding chunk t (the last one with start <= t)
LCS_HD int32_t find_seg(const Seg *segs, int64_t nseg, int64_t t) {
    int64_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (segs[mid].start <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return (int32_t)lo;
}

// Everything task u of stage st of pair p waits on and signals.
LCS_HD Task decode_task(const PairRec *pairs, int32_t slots, int32_t p, int32_t st, int32_t u) {
    Task T;
    const PairRec &P = pairs[p];
    T.pair = p;
    T.kind = P.stage_kind[st];
    T.level = P.stage_level[st];
    T.u = u;
    T.nwait = 0;
    T.nsig = 0;
    const int32_t cb = P.ctr_base;
    const int32_t l = T.level;
    switch (T.kind) {
        case ST_EMPTY:
        case ST_NM_SYM:
            // every task of the first stage writes into the slot: all of them
            // wait until its previous occupant is done
            if (p >= slots) {
                const PairRec &Q = pairs[p - slots];
                T.wait_idx[T.nwait] = Q.ctr_base + kCtrLeaves;
                T.wait_tgt[T.nwait++] = pair_finish_target(Q);
            }
            T.sig_idx[T.nsig++] = cb + (T.kind == ST_EMPTY ? kCtrLeaves : kCtrNm);
            break;
        case ST_BASE_BLK:
            T.wait_idx[T.nwait] = cb + kCtrNm;
            T.wait_tgt[T.nwait++] = P.sigma;
            T.sig_idx[T.nsig++] = cb + P.ctr_lev[0] + u / P.nvb;
            break;
        case ST_ANCHOR: {
            const int32_t q = u / P.nanch;
            strip_done_ctr(P, l - 1, 2 * q, &T.wait_idx[0], &T.wait_tgt[0]);
            strip_done_ctr(P, l - 1, 2 * q + 1, &T.wait_idx[1], &T.wait_tgt[1]);
            T.nwait = 2;
            T.sig_idx[T.nsig++] = cb + P.ctr_lev[l] + P.lev[l].nstrips + q;
            break;
        }
        case ST_BRACKET_CH: {
            const int32_t q = u / ((P.nanch - 1) * level_chunks_of(P, l));
            T.wait_idx[T.nwait] = cb + P.ctr_lev[l] + P.lev[l].nstrips + q;
            T.wait_tgt[T.nwait++] = P.nanch;
            T.sig_idx[T.nsig++] = cb + P.ctr_lev[l] + q;
            break;
        }
        case ST_LENGTH:
            strip_done_ctr(P, P.nlev - 1, 0, &T.wait_idx[0], &T.wait_tgt[0]);
            T.nwait = 1;
            T.sig_idx[T.nsig++] = cb + P.ctr_lev[P.nlev - 1] + 2 * P.lev[P.nlev - 1].nstrips;
            break;
        case ST_SPLIT: {
            T.wait_idx[T.nwait] = cb + P.ctr_lev[l] + 2 * P.lev[l].nstrips + u;
            T.wait_tgt[T.nwait++] = 1;
            const int32_t nextc = cb + P.ctr_lev[l - 1] + 2 * P.lev[l - 1].nstrips;
            T.sig_idx[T.nsig++] = nextc + 2 * u;
            if (2 * u + 1 < P.lev[l - 1].nstrips) T.sig_idx[T.nsig++] = nextc + 2 * u + 1;
            break;
        }
        case ST_LEAF:
            T.wait_idx[T.nwait] = cb + P.ctr_lev[0] + 2 * P.lev[0].nstrips + u;
            T.wait_tgt[T.nwait++] = 1;
            T.sig_idx[T.nsig++] = cb + kCtrLeaves;
            break;
    }
    return T;
}

// Position of a (kind, level) step in the method's order, the same for
// every pair; a pair's own stages are in increasing rank.
LCS_HD int32_t step_rank(int32_t kind, int32_t level) {
    switch (kind) {
        case ST_EMPTY: return 0;
        case ST_NM_SYM: return 1;
        case ST_BASE_BLK: return 2;
        case ST_ANCHOR: return 3 + 2 * (level - 1);
        case ST_BRACKET_CH: return 4 + 2 * (level - 1);
        case ST_LENGTH: return 3 + 2 * kMaxLev;
        case ST_SPLIT: return 4 + 2 * kMaxLev + (kMaxLev - 1 - level);
        default: return 4 + 3 * kMaxLev;  // ST_LEAF
    }
}

}  // namespace lcs
