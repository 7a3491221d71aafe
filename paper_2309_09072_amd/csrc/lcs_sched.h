// Task schedule of the persistent batch kernel, shared by the device (decode
// of a task number) and the host (construction of the per-pair records and a
// sequential simulation that checks the schedule without a GPU).
//
// Tasks are numbered pair by pair; inside a pair the stages follow the
// dependency order of the method: next-match tables, base strips, for every
// combine level its anchors then its bracketed tiles, the length, the trace
// splits from the top level down, the base-strip traces.  A task waits only on
// counters raised by tasks with smaller numbers.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "lcs_geom.h"

namespace lcs {

constexpr int kMaxLev = 16;
constexpr int kMaxStages = 4 + 3 * kMaxLev;

enum Stage : int32_t {
    ST_EMPTY = 0,    // m == 0 or n == 0: length 0
    ST_NM = 1,       // next-match tables (all symbols)
    ST_BASE = 2,     // one base strip
    ST_ANCHOR = 3,   // one anchor vertex of one combine
    ST_BRACKET = 4,  // one tile (all weight chunks) of one combine
    ST_LENGTH = 5,   // length + root trace node
    ST_SPLIT = 6,    // one trace split
    ST_LEAF = 7,     // trace inside one base strip
};

struct PairRec {
    int64_t ws_off;  // byte offset of this pair's slot in the workspace
    int64_t a_off, b_off, wit_off;
    int64_t task_base;  // first global task number of the pair
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
};

// counters of a pair: [0] next-match done, [1] base-strip traces done, then
// per level l: strip_done[S_l], anc_done[S_l], node_done[S_l]
constexpr int32_t kCtrNm = 0, kCtrLeaves = 1, kCtrHead = 2;

struct Task {
    int32_t pair, kind, level, u;
    int32_t nwait, nsig;
    int32_t wait_idx[2], wait_tgt[2];  // absolute counter indices and targets
    int32_t sig_idx[2];
};

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
    *tgt = (l == 0) ? 1 : P.nanch - 1;  // one base task, or one bracket task per tile
}

LCS_HD int32_t find_pair(const PairRec *pairs, int32_t npairs, int64_t t) {
    int32_t lo = 0, hi = npairs - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pairs[mid].task_base <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Everything task t waits on and signals.
LCS_HD Task decode_task(const PairRec *pairs, int32_t npairs, int32_t slots, int64_t t) {
    Task T;
    const int32_t p = find_pair(pairs, npairs, t);
    const PairRec &P = pairs[p];
    const int32_t local = (int32_t)(t - P.task_base);
    int32_t st = 0;
    while (st + 1 < P.nstages && P.stage_start[st + 1] <= local) ++st;
    T.pair = p;
    T.kind = P.stage_kind[st];
    T.level = P.stage_level[st];
    T.u = local - P.stage_start[st];
    T.nwait = 0;
    T.nsig = 0;
    const int32_t cb = P.ctr_base;
    const int32_t l = T.level, u = T.u;
    switch (T.kind) {
        case ST_EMPTY:
        case ST_NM:
            if (p >= slots) {
                const PairRec &Q = pairs[p - slots];
                T.wait_idx[T.nwait] = Q.ctr_base + kCtrLeaves;
                T.wait_tgt[T.nwait++] = pair_finish_target(Q);
            }
            T.sig_idx[T.nsig++] = cb + (T.kind == ST_EMPTY ? kCtrLeaves : kCtrNm);
            break;
        case ST_BASE:
            T.wait_idx[T.nwait] = cb + kCtrNm;
            T.wait_tgt[T.nwait++] = 1;
            T.sig_idx[T.nsig++] = cb + P.ctr_lev[0] + u;
            break;
        case ST_ANCHOR: {
            const int32_t q = u / P.nanch;
            strip_done_ctr(P, l - 1, 2 * q, &T.wait_idx[0], &T.wait_tgt[0]);
            strip_done_ctr(P, l - 1, 2 * q + 1, &T.wait_idx[1], &T.wait_tgt[1]);
            T.nwait = 2;
            T.sig_idx[T.nsig++] = cb + P.ctr_lev[l] + P.lev[l].nstrips + q;
            break;
        }
        case ST_BRACKET: {
            const int32_t q = u / (P.nanch - 1);
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

}  // namespace lcs
