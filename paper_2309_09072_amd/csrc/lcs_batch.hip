// Batches of string pairs (lcs_batch_plan / lcs_batch_submit).
//
// LCS_BATCH_PER_PAIR runs the per-level kernels of the single-pair path pair
// after pair on one stream (the one-pair-per-launch baseline).
//
// LCS_BATCH_STAGED (the fast mode) runs one launch per step of the method for
// all pairs at once: next-match tables, base strips, for every combine level
// its anchors then its bracketed (tile x weight-chunk) blocks, lengths, trace
// splits level by level, base-strip traces.  Every launch is a queue of
// independent work-groups over all pairs' items, so pairs of uneven length fill
// the device together; the kernel boundaries order the steps (no in-kernel
// waits, no cross-die cache maintenance per item).  Pairs are packed into the
// arena in waves, and the whole sequence can be replayed as one hipGraph.
//
// LCS_BATCH_PERSISTENT runs the whole batch -- every pair's next-match tables,
// base strips, combine levels, length and witness trace -- in ONE launch of a
// persistent kernel: as many work-groups as fit on the device at once pop task
// indices from a device counter in increasing order.  The tasks are the items
// of the staged mode (one symbol, one strip block, one anchor vertex, one tile
// x weight chunk, ...).  They are numbered wave by wave of the pairs that hold
// the slots at one time, and inside a wave step by step of the method across
// all of its pairs, so the work-groups in flight work on one step of many
// pairs rather than on the dependency chain of one.  Every task waits
// (bounded spin) only on counters raised by tasks with smaller numbers, which
// were popped earlier by running work-groups; so the queue always drains.
// Pair p uses workspace slot p mod slots, and its first tasks also wait until
// pair p - slots has finished its trace, which bounds the memory of a batch of
// any size.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "lcs.h"
#include "lcs_device.h"
#include "lcs_launch.h"
#include "lcs_plan.h"
#include "lcs_sched.h"

namespace lcs {

bool valid_shape(int32_t base_rows, int32_t tile);
int32_t resolve(int32_t v, int32_t dflt);
struct Recorder;
int32_t enqueue_build(const Layout &L, uint8_t *ws, const uint8_t *a, const uint8_t *b,
                      hipStream_t s, Recorder *rec);
int32_t enqueue_trace(const Layout &L, uint8_t *ws, const uint8_t *a, int32_t *a_idx,
                      int32_t *b_idx, hipStream_t s, Recorder *rec);

struct BatchArgs {
    const PairRec *pairs;
    int32_t npairs;
    int32_t slots;
    int64_t nchunks;       // persistent mode: chunks of the task order
    int32_t chunk;         // tasks per chunk at most
    uint8_t *ws;
    const uint8_t *symbols;
    int32_t *lengths;
    int32_t *a_idx;
    int32_t *b_idx;
    int32_t *ctr;          // all pair counters
    unsigned long long *next;  // chunk (or pair) dispenser
    int32_t *gerr;         // bit 0: a dependency wait timed out
    int32_t sigma;
    int32_t tile;
    const Seg *segs;     // persistent mode: the global task order
    int64_t nseg;
    int32_t base_mode;   // table form of the base-strip tasks (kBase*Mode)
    int32_t base_rows;   // rows per base strip
};

constexpr uint32_t kSpinLimit = 1u << 22;  // ~ seconds: a dependency bug ends as an error, not a hang

// Counter polling and raising are relaxed atomics at device scope; the
// persistent kernel orders the data around them with one acquire fence after
// all waits of a chunk and one release fence before its raises (each such
// fence is cache maintenance of the whole L2 of the die).
__device__ __forceinline__ int32_t ld_ctr(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// thread 0 only; false when the bounded wait ran out
__device__ bool wait_ge(const int32_t *p, int32_t target, int32_t *gerr) {
    uint32_t spins = 0;
    while (ld_ctr(p) < target) {
        __builtin_amdgcn_s_sleep(4);
        if (++spins > kSpinLimit) {
            atomicOr(gerr, 1);
            return false;
        }
    }
    return true;
}

// A value every lane of the wave holds alike (read from LDS, or derived from
// the wave index): taken from the first lane, so that the compiler keeps it
// and everything derived from it (pair record fields, matrix addresses,
// sizes) in scalar registers.
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void raise_ctr(int32_t *p, int32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ CombineArgs pair_combine_args(const PairRec &P, uint8_t *ws, int32_t l,
                                                         int32_t tile) {
    const LevelGeom &c = P.lev[l - 1], &p = P.lev[l];
    CombineArgs a;
    a.cbase = reinterpret_cast<const int32_t *>(ws + c.base);
    a.clast = reinterpret_cast<const int32_t *>(ws + c.last_off);
    a.hc = c.hfull;
    a.hclast = c.hlast;
    a.nc = c.nstrips;
    a.pbase = reinterpret_cast<int32_t *>(ws + p.base);
    a.plast = reinterpret_cast<int32_t *>(ws + p.last_off);
    a.np = p.nstrips;
    a.n = P.n;
    a.tile = tile;
    a.nanch = P.nanch;
    a.hs = 2 * c.hfull + 1;
    a.anch = reinterpret_cast<int32_t *>(ws + P.anch_off[l]);
    a.jchunk = P.jchunk;
    a.nchunks = imax(1, (a.hs - 1 + a.jchunk - 1) / a.jchunk);
    return a;
}

union PersistentSmem {
    int32_t nm[kWaves];
    int32_t base[kWave * 65];  // also the table form's window, then its transposition
    AnchorSmemBlock anchor;
    BracketSmem bracket;
    BracketSmemT<BracketCfg16> bracket16;
    int32_t len[1];
    int32_t split[1];
    int32_t leaf[65 * 65];
};
static_assert(sizeof(int32_t) * kWave * 65 >= base_smem_bytes<64, kBaseTab16Mode>(),
              "the base member holds a table-form base strip of 64 rows");

__device__ __forceinline__ int32_t vertex_blocks(int32_t n) { return vertex_blocks_of(n, kBlock); }

// Base-strip task u of pair P (one strip x one 256-vertex block) in table
// form kMode; smem: base_smem_bytes<H0, kMode>() bytes.
template <int H0, int kMode>
__device__ __forceinline__ void base_task(const BatchArgs &A, uint8_t *ws, const PairRec &P,
                                          int32_t u, int32_t *lds, uint8_t *smem) {
    int32_t *hdr = reinterpret_cast<int32_t *>(ws + P.off_hdr);
    const int32_t *nm = reinterpret_cast<const int32_t *>(ws + P.off_nm);
    const uint8_t *a = A.symbols + P.a_off;
    const LevelGeom &g = P.lev[0];
    const int32_t nvb = vertex_blocks(P.n);
    const int32_t s0 = u / nvb;
    const bool last = (s0 == g.nstrips - 1);
    const int32_t h = last ? g.hlast : H0;
    int32_t *out = reinterpret_cast<int32_t *>(ws + (last ? g.last_off : g.base)) +
                   (last ? 0 : (size_t)s0 * strip_elems(P.n, H0));
    const int32_t vb = u - s0 * nvb;
    base_strip_block<H0, kMode>(a + (size_t)s0 * H0, h, P.n, A.sigma, nm, out, vb * kBlock, hdr, lds,
                                smem);
}

// Bracket task u of level l of pair P (one tile x one weight chunk of C::kJ
// weights; a chunk beyond a short last strip's weights does nothing).
template <class C, bool kCoop = false>
__device__ __forceinline__ void bracket_task(const BatchArgs &A, uint8_t *ws, const PairRec &P,
                                             int32_t l, int32_t u, BracketSmemT<C> &sm) {
    const CombineArgs c = pair_combine_args(P, ws, l, A.tile);
    const int32_t ntile = P.nanch - 1;
    const int32_t Hf = 2 * P.lev[l - 1].hfull + 1;  // weights of a full-height parent
    const int32_t nchl = imax(1, (Hf - 1 + C::kJ - 1) / C::kJ);
    const int32_t qt = u / nchl;
    const int32_t q = qt / ntile, tl = qt - q * ntile, ch = u - qt * nchl;
    const StripRef U = child_strip(c, 2 * q), L = child_strip(c, 2 * q + 1);
    int32_t *G = parent_strip(c, q);
    const int32_t H = U.h + L.h + 1;
    const int32_t nch = imax(1, (H - 1 + C::kJ - 1) / C::kJ);
    if (ch >= nch) return;
    const int32_t i0 = tl * A.tile;
    const int32_t len = imin(A.tile, P.n - i0);
    const int32_t *Ka = c.anch + ((size_t)q * c.nanch + tl) * (size_t)c.hs;
    const int32_t *Kb = c.anch + ((size_t)q * c.nanch + tl + 1) * (size_t)c.hs;
    const int32_t j0 = ch * C::kJ;
    const int32_t jn = (ch == nch - 1) ? H - j0 : C::kJ;
    bracket_block<C, kCoop>(U.d, U.h, L.d, L.h, G, P.n, i0, len, j0, jn, Ka, Kb, sm);
}

// One task of pair p (all threads of the work-group).  kAll: every table
// form and bracket shape, chosen at run time (the persistent and pair-queue
// kernels); otherwise the global-table base strips only (the step kernel,
// which the staged mode uses for them).
template <int H0, bool kAll = true>
__device__ __forceinline__ void exec_task(const BatchArgs &A, uint8_t *ws, int32_t p, int32_t kind,
                                          int32_t l, int32_t u, PersistentSmem &sm) {
    const PairRec &P = A.pairs[p];
    int32_t *hdr = reinterpret_cast<int32_t *>(ws + P.off_hdr);
    int32_t *nm = reinterpret_cast<int32_t *>(ws + P.off_nm);
    const uint8_t *a = A.symbols + P.a_off;
    const uint8_t *b = A.symbols + P.b_off;
    switch (kind) {
        case ST_EMPTY:
            if (threadIdx.x == 0) A.lengths[p] = 0;
            break;
        case ST_NM_SYM:
            if (u == 0)  // (the same work-group then checks b's symbols into hdr[0])
                for (int32_t i = threadIdx.x; i < kHeaderWords; i += kBlock) hdr[i] = 0;
            nextmatch_block(b, P.n, u, A.sigma, nm + (size_t)u * (size_t)(P.n + 2), sm.nm, hdr);
            break;
        case ST_BASE_BLK:
            if (kAll && A.base_mode == kBaseTab16Mode)
                base_task<H0, kBaseTab16Mode>(A, ws, P, u, sm.base,
                                              reinterpret_cast<uint8_t *>(sm.base));
            else
                base_task<H0, kBaseGlobal>(A, ws, P, u, sm.base, nullptr);
            break;
        case ST_ANCHOR: {
            const CombineArgs c = pair_combine_args(P, ws, l, A.tile);
            const int32_t q = u / P.nanch, an = u - q * P.nanch;
            const StripRef U = child_strip(c, 2 * q), L = child_strip(c, 2 * q + 1);
            int32_t *G = parent_strip(c, q);
            anchor_block(U.d, U.h, L.d, L.h, G, P.n, anchor_vertex(an, A.tile, P.n),
                         c.anch + ((size_t)q * c.nanch + an) * (size_t)c.hs, sm.anchor);
            if (an == c.nanch - 1) {
                const int32_t H = U.h + L.h + 1;
                int32_t *srow = G + (size_t)(P.n + 1) * H;
                for (int32_t j = threadIdx.x; j < H; j += kBlock) srow[j] = P.n + 1;
            }
            break;
        }
        case ST_BRACKET_CH:
            if (kAll && P.jchunk == BracketCfg16::kJ)
                bracket_task<BracketCfg16>(A, ws, P, l, u, sm.bracket16);
            else
                bracket_task<BracketCfg32>(A, ws, P, l, u, sm.bracket);
            break;
        case ST_LENGTH: {
            const LevelGeom &top = P.lev[P.nlev - 1];
            length_block(reinterpret_cast<const int32_t *>(ws + top.last_off), P.m, P.n, hdr,
                         reinterpret_cast<int4 *>(ws + P.node_off[P.nlev - 1]), sm.len);
            if (threadIdx.x == 0) A.lengths[p] = (hdr[0] & kErrSymbol) ? LCS_E_SYMBOL : hdr[1];
            break;
        }
        case ST_SPLIT: {
            const CombineArgs c = pair_combine_args(P, ws, l, A.tile);
            const int4 *nin = reinterpret_cast<const int4 *>(ws + P.node_off[l]);
            int4 *nout = reinterpret_cast<int4 *>(ws + P.node_off[l - 1]);
            const int4 node = nin[u];
            if (2 * u + 1 >= c.nc) {
                if (threadIdx.x == 0) nout[2 * u] = node;
            } else {
                const StripRef U = child_strip(c, 2 * u), L = child_strip(c, 2 * u + 1);
                trace_split_block(U.d, U.h, L.d, L.h, P.n, node, nout + 2 * u, nout + 2 * u + 1, hdr,
                                  sm.split);
            }
            break;
        }
        case ST_LEAF: {
            const LevelGeom &g = P.lev[0];
            const int32_t h = (u == g.nstrips - 1) ? g.hlast : H0;
            const int4 *nodes = reinterpret_cast<const int4 *>(ws + P.node_off[0]);
            trace_leaf_block<H0>(a + (size_t)u * H0, h, P.n, A.sigma, nm, nodes[u], u * H0,
                                 A.a_idx + P.wit_off, A.b_idx + P.wit_off, P.m < P.n ? P.m : P.n, hdr,
                                 sm.leaf);
            break;
        }
    }
}

// One kernel runs every kind of task, so it would carry the largest register
// allocation of them all (the base strip's, about 210 VGPRs: 2 waves per
// SIMD).  It is held to 4 waves per SIMD instead; the base-strip task then
// spills a little, and the latency-bound bracket tasks, most of the work,
// have twice the waves in flight.
template <int H0>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_persistent(BatchArgs A) {
    __shared__ PersistentSmem sm;
    __shared__ int32_t s_pair, s_stage, s_u0, s_cnt, s_ok;
    for (;;) {
        if (threadIdx.x == 0) {
            const long long g = (long long)atomicAdd(A.next, 1ull);
            s_cnt = 0;
            if (g < A.nchunks) {
                const Seg &sg = A.segs[find_seg(A.segs, A.nseg, g)];
                const int32_t u0 = (int32_t)(g - sg.start) * A.chunk;
                const int32_t cnt = imin(A.chunk, stage_tasks(A.pairs[sg.pair], sg.stage) - u0);
                // wait for the inputs of every task of the chunk (bounded); on a
                // timeout the chunk is skipped
                int32_t ok = 1;
                for (int32_t u = u0; u < u0 + cnt; ++u) {
                    const Task T = decode_task(A.pairs, A.slots, sg.pair, sg.stage, u);
                    for (int32_t w = 0; w < T.nwait; ++w)
                        ok &= wait_ge(A.ctr + T.wait_idx[w], T.wait_tgt[w], A.gerr);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                s_pair = sg.pair;
                s_stage = sg.stage;
                s_u0 = u0;
                s_cnt = cnt;
                s_ok = ok;
            }
        }
        __syncthreads();
        const int32_t cnt = uniform(s_cnt);
        if (cnt == 0) break;
        const int32_t p = uniform(s_pair), st = uniform(s_stage), u0 = uniform(s_u0);
        const PairRec &P = A.pairs[p];
        if (uniform(s_ok))
            for (int32_t u = u0; u < u0 + cnt; ++u) {
                exec_task<H0>(A, A.ws + P.ws_off, p, P.stage_kind[st], P.stage_level[st], u, sm);
                __syncthreads();
            }
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            // raise the chunk's counters, equal consecutive ones at once
            int32_t last = -1, run = 0;
            for (int32_t u = u0; u < u0 + cnt; ++u) {
                const Task T = decode_task(A.pairs, A.slots, p, st, u);
                for (int32_t i = 0; i < T.nsig; ++i) {
                    if (T.sig_idx[i] == last) {
                        ++run;
                        continue;
                    }
                    if (run) raise_ctr(A.ctr + last, run);
                    last = T.sig_idx[i];
                    run = 1;
                }
            }
            if (run) raise_ctr(A.ctr + last, run);
        }
        __syncthreads();
    }
}

// Pair queue: a work-group takes whole pairs from the queue A.next (in the
// host's order, largest first, for balance) and runs the stages of each in
// order, every task of a stage and every stage separated by a work-group
// barrier; all of a pair's matrices live in the work-group's own slot.
// Nothing waits on another work-group.
template <int H0>
__global__ void __launch_bounds__(kBlock) k_pair_queue(BatchArgs A, const int32_t *order,
                                                        int64_t off_slots, int64_t slot_bytes) {
    __shared__ PersistentSmem sm;
    __shared__ int32_t s_q;
    uint8_t *ws = A.ws + off_slots + (int64_t)blockIdx.x * slot_bytes;
    for (;;) {
        if (threadIdx.x == 0) s_q = (int32_t)atomicAdd(A.next, 1ull);
        __syncthreads();
        const int32_t q = uniform(s_q);
        __syncthreads();
        if (q >= A.npairs) break;
        const int32_t p = order[q];
        const PairRec &P = A.pairs[p];
        for (int32_t st = 0; st < P.nstages; ++st) {
            const int32_t kind = P.stage_kind[st], l = P.stage_level[st];
            const int32_t nu = P.stage_start[st + 1] - P.stage_start[st];
            for (int32_t u = 0; u < nu; ++u) {
                exec_task<H0>(A, ws, p, kind, l, u, sm);
                __syncthreads();
            }
        }
    }
}

// One step of the staged mode: the items of every participating pair, as a
// queue of work-groups.  Item t belongs to the pair j with
// first[j] <= t < first[j + 1] (stage_item below).
struct StageArgs {
    int32_t kind, level, npairs;
    int32_t jchunk;         // weights per bracket task (the bracket shape's kJ)
    int32_t cols;           // longest column string of the plan
    const int32_t *pair;    // participating pairs
    const int64_t *first;   // their first item, plus the total at [npairs]
};

// The pair of item t and t's index among that pair's items, found by the whole
// wave: each round loads 64 evenly spaced entries of first[] at once and keeps
// the last one <= t (first[] never decreases and first[0] = 0 <= t), so 4096
// pairs take two rounds of loads instead of a dozen dependent ones.  Every
// lane returns the same pair; t must be the same on every lane.
__device__ __forceinline__ int2 stage_item(const StageArgs &S, int64_t t) {
    const int32_t lane = __lane_id();
    int32_t lo = 0, cnt = S.npairs;
    while (cnt > 1) {
        const int32_t stride = (cnt + kWave - 1) / kWave;
        const int32_t off = lane * stride;
        const bool le = off < cnt && S.first[lo + off] <= t;
        const int32_t l = 63 - __clzll((long long)__ballot(le));
        lo = uniform(lo + l * stride);
        cnt = uniform(imin(stride, cnt - l * stride));
    }
    return make_int2(uniform(S.pair[lo]), uniform((int32_t)(t - S.first[lo])));
}

// Instantiated per step kind, so each step gets its own register allocation
// (a kernel that could run any step would carry the largest one everywhere).
template <int H0, int KIND>
__global__ void __launch_bounds__(kBlock) k_stage(BatchArgs A, StageArgs S) {
    __shared__ PersistentSmem sm;
    const int64_t t = blockIdx.x;
    const int2 pu = stage_item(S, t);
    const int32_t p = pu.x, u = pu.y;
    exec_task<H0, false>(A, A.ws + A.pairs[p].ws_off, p, KIND, S.level, u, sm);
}

// Staged base-strip tasks (one strip x one 256-vertex block each) with the
// next-match table window in LDS, as in the single-pair path.
template <int H0, int kMode>
__global__ void __launch_bounds__(kBlock) k_stage_base(BatchArgs A, StageArgs S) {
    static_assert(kMode == kBaseTab16Mode, "the global-table form runs in k_stage");
    __shared__ __align__(16) uint8_t smem[base_smem_bytes<H0, kMode>()];  // table, then transposition
    const int64_t t = blockIdx.x;
    const int2 pu = stage_item(S, t);
    const PairRec &P = A.pairs[pu.x];
    base_task<H0, kMode>(A, A.ws + P.ws_off, P, pu.y, reinterpret_cast<int32_t *>(smem), smem);
}

// Staged bracket tasks (one tile x one weight chunk each) in the bracket shape
// C: the 16-bit one (64 weights per task) when every pair of the plan fits
// 16-bit values, as in the single-pair path, with the same 64-VGPR limit.
template <int H0, class C, bool kCoop = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8)))
k_stage_bracket(BatchArgs A, StageArgs S) {
    __shared__ BracketSmemT<C> sm;
    const int64_t t = blockIdx.x;
    const int2 pu = stage_item(S, t);
    const PairRec &P = A.pairs[pu.x];
    bracket_task<C, kCoop>(A, A.ws + P.ws_off, P, S.level, pu.y, sm);
}

// Staged anchor search with the vertex's D_U row and k* row in dynamic LDS
// (the search's AnchorSmem, hc + 1 and 2 hc + 1 int32; hc = child strip height, the
// same for every pair at one level).
// (Left to itself the compiler gives this kernel 184 VGPRs, 2 waves per
// SIMD; the search fits in 80 without spills, as in the single-pair path.)
template <int H0>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6)))
k_stage_anchor_lds(BatchArgs A, StageArgs S, int32_t hc) {
    extern __shared__ unsigned long long dyn[];
    // neighbouring anchors on one XCD (see anchor_block_id in lcs_kernels.hip)
    const int64_t t = xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x, imax(1, (int32_t)gridDim.x / 8));
    const int2 pu = stage_item(S, t);
    const int32_t p = pu.x, u = pu.y;
    const PairRec &P = A.pairs[p];
    uint8_t *ws = A.ws + P.ws_off;
    const CombineArgs c = pair_combine_args(P, ws, S.level, A.tile);
    const int32_t q = u / P.nanch, an = u - q * P.nanch;
    const StripRef U = child_strip(c, 2 * q), L = child_strip(c, 2 * q + 1);
    int32_t *G = parent_strip(c, q);
    AnchorSmemBlock &sm = *reinterpret_cast<AnchorSmemBlock *>(dyn);
    int32_t *us = reinterpret_cast<int32_t *>(dyn + sizeof(AnchorSmemBlock) / 8);
    int32_t *ks = us + (hc + 1);
    anchor_block_t<true, kBlock, 4>(U.d, U.h, L.d, L.h, G, P.n, anchor_vertex(an, A.tile, P.n),
                                    c.anch + ((size_t)q * c.nanch + an) * (size_t)c.hs, sm, us, ks);
    if (an == c.nanch - 1) {
        const int32_t H = U.h + L.h + 1;
        int32_t *srow = G + (size_t)(P.n + 1) * H;
        for (int32_t j = threadIdx.x; j < H; j += kBlock) srow[j] = P.n + 1;
    }
}

// Staged anchor searches, one per wave, for short rows (hs = 2 hc + 1 <= 512
// weights): each wave finds its own task and has its own slice of dynamic
// LDS (`bytes`: the search's AnchorSmem, then hc + 1 and 2 hc + 1 int32); no
// block barrier is used, so a wave without a task simply exits.
template <int CPT>
__global__ void __launch_bounds__(kBlock) k_stage_anchor_wave(BatchArgs A, StageArgs S, int32_t hc,
                                                              int32_t bytes, int64_t items) {
    extern __shared__ unsigned long long dyn[];
    const int32_t wv = uniform((int32_t)threadIdx.x / kWave);  // the same on every lane of a wave
    const int64_t t = (int64_t)xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x,
                                         imax(1, (int32_t)gridDim.x / 8)) * kWaves + wv;
    if (t >= items) return;
    const int2 pu = stage_item(S, t);
    const int32_t p = pu.x, u = pu.y;
    const PairRec &P = A.pairs[p];
    uint8_t *ws = A.ws + P.ws_off;
    const CombineArgs c = pair_combine_args(P, ws, S.level, A.tile);
    const int32_t q = u / P.nanch, an = u - q * P.nanch;
    const StripRef U = child_strip(c, 2 * q), L = child_strip(c, 2 * q + 1);
    int32_t *G = parent_strip(c, q);
    unsigned long long *base = dyn + (size_t)wv * (size_t)(bytes / 8);
    AnchorSmem<kWave, CPT> &sm = *reinterpret_cast<AnchorSmem<kWave, CPT> *>(base);
    int32_t *us = reinterpret_cast<int32_t *>(base + sizeof(AnchorSmem<kWave, CPT>) / 8);
    int32_t *ks = us + (hc + 1);
    anchor_block_t<true, kWave, CPT>(U.d, U.h, L.d, L.h, G, P.n, anchor_vertex(an, A.tile, P.n),
                                     c.anch + ((size_t)q * c.nanch + an) * (size_t)c.hs, sm, us, ks);
    if (an == c.nanch - 1) {
        const int32_t H = U.h + L.h + 1;
        int32_t *srow = G + (size_t)(P.n + 1) * H;
        for (int32_t j = __lane_id(); j < H; j += kWave) srow[j] = P.n + 1;
    }
}

// Staged seaweed combing: one work-group per (pair, base strip), blockDim set
// by the plan's longest string (C columns per thread, as in the single-pair
// path).
template <int C, bool kPacked>
__global__ void __launch_bounds__(kCombMaxThreads) k_stage_comb(BatchArgs A, StageArgs S) {
    __shared__ int32_t lds[3 * kCombMaxRows + 4 * (kCombMaxThreads / kWave)];
    const int2 pu = stage_item(S, blockIdx.x);
    const PairRec &P = A.pairs[pu.x];
    uint8_t *ws = A.ws + P.ws_off;
    const LevelGeom &g = P.lev[0];
    const int32_t s = pu.y;
    const int32_t h = (s == g.nstrips - 1) ? g.hlast : P.h0;
    int32_t *cs = reinterpret_cast<int32_t *>(ws + P.off_comb) + (size_t)s * (size_t)P.comb_stride;
    comb_strip_block<kCombMaxThreads, C, kPacked>(A.symbols + P.a_off + (size_t)s * P.h0, h, A.symbols + P.b_off,
                                         P.n, A.sigma, cs, cs + P.n, cs + 2 * (size_t)P.n, lds,
                                         reinterpret_cast<int32_t *>(ws + P.off_hdr));
}

// The same as a pipeline of waves (the plan's longest string <= 32767): 64 C
// columns per wave, blockDim set by that string.
template <int C>
__global__ void __launch_bounds__(kCombPipeWaves * kWave) k_stage_comb_pipe(BatchArgs A, StageArgs S) {
    extern __shared__ int32_t lds[];  // (waves + 1) x base rows int32
    const int2 pu = stage_item(S, blockIdx.x);
    const PairRec &P = A.pairs[pu.x];
    uint8_t *ws = A.ws + P.ws_off;
    const LevelGeom &g = P.lev[0];
    const int32_t s = pu.y;
    const int32_t h = (s == g.nstrips - 1) ? g.hlast : P.h0;
    int32_t *cs = reinterpret_cast<int32_t *>(ws + P.off_comb) + (size_t)s * (size_t)P.comb_stride;
    comb_strip_pipe<C>(A.symbols + P.a_off + (size_t)s * P.h0, h, A.symbols + P.b_off, P.n, A.sigma, cs,
                       cs + P.n, cs + 2 * (size_t)P.n, lds, reinterpret_cast<int32_t *>(ws + P.off_hdr));
}

// Staged breakout-row generation: one wave per (pair, strip, run of
// kStageRun vertices), four per work-group (runs of one strip on one XCD).
constexpr int32_t kStageRun = 64;
template <int E>
__global__ void __launch_bounds__(kBlock) k_stage_dgen(BatchArgs A, StageArgs S, int64_t items) {
    __shared__ int32_t lst[kWaves][E * kWave];
    const int32_t wv = uniform((int32_t)threadIdx.x / kWave);
    const int64_t t = (int64_t)xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x,
                                         imax(1, (int32_t)gridDim.x / 8)) * kWaves + wv;
    if (t >= items) return;
    const int2 pu = stage_item(S, t);
    const PairRec &P = A.pairs[pu.x];
    uint8_t *ws = A.ws + P.ws_off;
    const LevelGeom &g = P.lev[0];
    const int32_t nrun = (P.n + 2 + kStageRun - 1) / kStageRun;
    const int32_t s = pu.y / nrun, ck = pu.y - s * nrun;
    const bool last = (s == g.nstrips - 1);
    const int32_t h = last ? g.hlast : P.h0;
    int32_t *out = reinterpret_cast<int32_t *>(ws + (last ? g.last_off : g.base)) +
                   (last ? 0 : (size_t)s * strip_elems(P.n, P.h0));
    const int32_t *cs = reinterpret_cast<const int32_t *>(ws + P.off_comb) + (size_t)s * (size_t)P.comb_stride;
    const int32_t i0 = ck * kStageRun;
    dgen_wave<E>(cs, cs + P.n, cs + 2 * (size_t)P.n, h, P.n, i0, imin(i0 + kStageRun, P.n + 2), out,
                 lst[wv]);
}

// Staged trace inside base strips of 128 to 512 rows: K waves per strip.
template <int Ew, int K>
__global__ void __launch_bounds__(K * kWave) k_stage_leaf_tall(BatchArgs A, StageArgs S, int32_t tabcap) {
    constexpr int E = Ew * K;
    extern __shared__ int32_t tab[];  // tabcap int32: the next-match window
    __shared__ int32_t mrow[E * kWave], xs[E * kWave];
    __shared__ int32_t ring[(K - 1) * E * kWave], sync[K + 2];
    const int2 pu = stage_item(S, blockIdx.x);
    const PairRec &P = A.pairs[pu.x];
    uint8_t *ws = A.ws + P.ws_off;
    const LevelGeom &g = P.lev[0];
    const int32_t u = pu.y;
    const int32_t h = (u == g.nstrips - 1) ? g.hlast : P.h0;
    const int4 *nodes = reinterpret_cast<const int4 *>(ws + P.node_off[0]);
    trace_leaf_pipe<Ew, K>(A.symbols + P.a_off + (size_t)u * P.h0, h, P.n, A.sigma,
                           reinterpret_cast<const int32_t *>(ws + P.off_nm), nodes[u], u * P.h0,
                           A.a_idx + P.wit_off, A.b_idx + P.wit_off, P.m < P.n ? P.m : P.n,
                           reinterpret_cast<int32_t *>(ws + P.off_hdr), tab, tabcap,
                           ws + P.off_leaf + (size_t)u * (size_t)P.leaf_stride, mrow, xs, ring, sync);
}

// dynamic LDS a staged anchor search may take: what one work-group of gfx950
// can hold (160 KB) minus room for the kernel's static LDS
constexpr size_t kStageMaxLds = 159 * 1024;

// Opt the staged anchor kernels in to more than 64 KB of dynamic LDS, once per
// device (also called at plan time, outside any graph capture).
static hipError_t opt_in_stage_lds() {
    static bool opted[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64 || opted[dev]) return hipSuccess;
    const void *fns[3] = {(const void *)k_stage_anchor_lds<16>, (const void *)k_stage_anchor_lds<32>,
                          (const void *)k_stage_anchor_lds<64>};
    for (const void *f : fns) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kStageMaxLds);
        if (e != hipSuccess) return e;
    }
    opted[dev] = true;
    return hipSuccess;
}

template <int H0>
static hipError_t launch_stage(const BatchArgs &A, const StageArgs &S, dim3 grid, hipStream_t st) {
    if (S.kind == ST_ANCHOR && S.level >= 1 && S.level < kMaxLev) {
        const int32_t hc = A.base_rows << (S.level - 1);
        const int32_t hs = 2 * hc + 1;
        if (hs <= 512) {  // short rows: one search per wave
            const int32_t per_wave = (int32_t)(((hs <= 256 ? sizeof(AnchorSmem<kWave, 4>)
                                                           : sizeof(AnchorSmem<kWave, 8>)) +
                                                4 * ((size_t)hc + 1 + (size_t)hs) + 7) & ~(size_t)7);
            const int64_t items = grid.x;
            const dim3 g((unsigned)((items + kWaves - 1) / kWaves));
            const size_t bytes = (size_t)per_wave * kWaves;
            if (hs <= 256)
                hipLaunchKernelGGL((k_stage_anchor_wave<4>), g, dim3(kBlock), bytes, st, A, S, hc,
                                   per_wave, items);
            else
                hipLaunchKernelGGL((k_stage_anchor_wave<8>), g, dim3(kBlock), bytes, st, A, S, hc,
                                   per_wave, items);
            return hipGetLastError();
        }
        const size_t bytes = sizeof(AnchorSmemBlock) + 4 * ((size_t)hc + 1 + 2 * (size_t)hc + 1);
        if (bytes <= kStageMaxLds) {
            const hipError_t e = opt_in_stage_lds();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_stage_anchor_lds<H0>), grid, dim3(kBlock), bytes, st, A, S, hc);
            return hipGetLastError();
        }
    }
    switch (S.kind) {
        case ST_EMPTY: hipLaunchKernelGGL((k_stage<H0, ST_EMPTY>), grid, dim3(kBlock), 0, st, A, S); break;
        case ST_NM_SYM: hipLaunchKernelGGL((k_stage<H0, ST_NM_SYM>), grid, dim3(kBlock), 0, st, A, S); break;
        case ST_BASE_BLK:
            // table form by the plan's longest string (every pair's n is at most that)
            if (A.base_mode == kBaseTab16Mode)
                hipLaunchKernelGGL((k_stage_base<H0, kBaseTab16Mode>), grid, dim3(kBlock), 0, st, A, S);
            else  // the generic step kernel keeps a smaller register allocation here
                hipLaunchKernelGGL((k_stage<H0, ST_BASE_BLK>), grid, dim3(kBlock), 0, st, A, S);
            break;
        case ST_ANCHOR: hipLaunchKernelGGL((k_stage<H0, ST_ANCHOR>), grid, dim3(kBlock), 0, st, A, S); break;
        case ST_BRACKET_CH:
            // the single-pair path's shape for the level's child strip height
            if (S.jchunk == BracketCfg16::kJ && S.level >= 1 && (A.base_rows << (S.level - 1)) >= kWideWindowMinH)
                hipLaunchKernelGGL((k_stage_bracket<H0, BracketCfg16Wide, true>), grid, dim3(kBlock), 0, st, A, S);
            else if (S.jchunk == BracketCfg16::kJ && S.level >= 1 && (A.base_rows << (S.level - 1)) >= kCoopPass2MinH)
                hipLaunchKernelGGL((k_stage_bracket<H0, BracketCfg16Mid, true>), grid, dim3(kBlock), 0, st, A, S);
            else if (S.jchunk == BracketCfg16::kJ)
                hipLaunchKernelGGL((k_stage_bracket<H0, BracketCfg16>), grid, dim3(kBlock), 0, st, A, S);
            else
                hipLaunchKernelGGL((k_stage_bracket<H0, BracketCfg32>), grid, dim3(kBlock), 0, st, A, S);
            break;
        case ST_LENGTH: hipLaunchKernelGGL((k_stage<H0, ST_LENGTH>), grid, dim3(kBlock), 0, st, A, S); break;
        case ST_SPLIT: hipLaunchKernelGGL((k_stage<H0, ST_SPLIT>), grid, dim3(kBlock), 0, st, A, S); break;
        case ST_LEAF: hipLaunchKernelGGL((k_stage<H0, ST_LEAF>), grid, dim3(kBlock), 0, st, A, S); break;
        case ST_COMB: {
            const int32_t C = comb_cols(S.cols);  // as in the single-pair path
            const int32_t thr = comb_threads(S.cols, C);
            const int32_t cp = comb_pipe_cols(S.cols);
            const int32_t waves = (S.cols + kWave * cp - 1) / (kWave * cp);
            const size_t bytes = 4 * (size_t)(waves + 1) * (size_t)A.base_rows;
            if (S.cols <= kCombPackedMaxN && bytes <= kCombPipeMaxLds) {  // the wave pipeline
                const dim3 blk((unsigned)(kWave * waves));  // (a pair's n may be below S.cols)
                if (cp == 4)
                    hipLaunchKernelGGL((k_stage_comb_pipe<4>), grid, blk, bytes, st, A, S);
                else if (cp == 8)
                    hipLaunchKernelGGL((k_stage_comb_pipe<8>), grid, blk, bytes, st, A, S);
                else if (cp == 16)
                    hipLaunchKernelGGL((k_stage_comb_pipe<16>), grid, blk, bytes, st, A, S);
                else
                    hipLaunchKernelGGL((k_stage_comb_pipe<32>), grid, blk, bytes, st, A, S);
            } else if (S.cols > kCombPackedMaxN)
                hipLaunchKernelGGL((k_stage_comb<16, false>), grid, dim3(thr), 0, st, A, S);
            else if (C == 4)
                hipLaunchKernelGGL((k_stage_comb<4, true>), grid, dim3(thr), 0, st, A, S);
            else if (C == 8)
                hipLaunchKernelGGL((k_stage_comb<8, true>), grid, dim3(thr), 0, st, A, S);
            else if (C == 16)
                hipLaunchKernelGGL((k_stage_comb<16, true>), grid, dim3(thr), 0, st, A, S);
            else
                hipLaunchKernelGGL((k_stage_comb<32, true>), grid, dim3(thr), 0, st, A, S);
            break;
        }
        case ST_DGEN: {
            const int64_t items = grid.x;
            const dim3 g((unsigned)((items + kWaves - 1) / kWaves));
            if (A.base_rows <= kWave)
                hipLaunchKernelGGL((k_stage_dgen<1>), g, dim3(kBlock), 0, st, A, S, items);
            else if (A.base_rows <= 2 * kWave)
                hipLaunchKernelGGL((k_stage_dgen<2>), g, dim3(kBlock), 0, st, A, S, items);
            else if (A.base_rows <= 4 * kWave)
                hipLaunchKernelGGL((k_stage_dgen<4>), g, dim3(kBlock), 0, st, A, S, items);
            else if (A.base_rows <= 8 * kWave)
                hipLaunchKernelGGL((k_stage_dgen<8>), g, dim3(kBlock), 0, st, A, S, items);
            else
                hipLaunchKernelGGL((k_stage_dgen<16>), g, dim3(kBlock), 0, st, A, S, items);
            break;
        }
        case ST_LEAF_TALL: {
            const int32_t tabcap = leaf_tab_cap(A.sigma, S.cols);  // by the plan's longest string
            const size_t bytes = 4 * (size_t)tabcap;
            if (A.base_rows <= 2 * kWave)
                hipLaunchKernelGGL((k_stage_leaf_tall<1, 2>), grid, dim3(2 * kWave), bytes, st, A, S, tabcap);
            else if (A.base_rows <= 4 * kWave)
                hipLaunchKernelGGL((k_stage_leaf_tall<1, 4>), grid, dim3(4 * kWave), bytes, st, A, S, tabcap);
            else if (A.base_rows <= 8 * kWave)
                hipLaunchKernelGGL((k_stage_leaf_tall<2, 4>), grid, dim3(4 * kWave), bytes, st, A, S, tabcap);
            else
                hipLaunchKernelGGL((k_stage_leaf_tall<2, 8>), grid, dim3(8 * kWave), bytes, st, A, S, tabcap);
            break;
        }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ void k_fill(int32_t *p, int64_t count, int32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_finish_pair(const int32_t *hdr, int32_t *len_out) {
    if (threadIdx.x == 0) *len_out = (hdr[0] & kErrSymbol) ? LCS_E_SYMBOL : hdr[1];
}

}  // namespace lcs

using namespace lcs;

struct lcs_batch_s {
    lcs_batch_desc d{};
    int64_t slot_bytes = 0;
    int32_t ctr_per_pair = 0;
    int64_t off_ctl = 0, off_pairs = 0, off_ctr = 0, off_slots = 0, total = 0;
    PairRec *host_pairs = nullptr;  // pinned staging of the pair records
    int32_t resident = 0;           // work-groups of the persistent kernel that fit at once
    int32_t resident_pq = 0;        // the same for the pair-queue kernel
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    uint64_t gkey = 0;
    hipEvent_t copied = nullptr;    // the last copy out of host_pairs has run
    int64_t off_stage = 0, stage_bytes = 0;
    uint8_t *host_stage = nullptr;  // pinned staging of the staged-mode item tables
};

// Weights per staged bracket task: the 16-bit bracket shape when every value
// of every pair of the plan fits in 16 bits (n + 1 <= 65535; strip heights
// are at most max_len), else the 32-bit one.
static int32_t stage_jchunk(int32_t max_len) {
    return (max_len + 1 <= 65535) ? BracketCfg16::kJ : BracketCfg32::kJ;
}

static int32_t counters_per_pair(int32_t max_len, int32_t h0) {
    // 2 + 3 * sum over levels of the strip count
    int32_t s = (max_len + h0 - 1) / h0, tot = 0;
    if (s < 1) s = 1;
    for (;;) {
        tot += s;
        if (s == 1) break;
        s = (s + 1) / 2;
    }
    return kCtrHead + 3 * tot;
}

// Sizes of a batch plan (no device calls).
static int32_t plan_sizes(const lcs_batch_desc *desc, lcs_batch_s *b) {
    lcs_batch_desc d = *desc;
    d.base_rows = resolve(d.base_rows, kDefaultBaseRows);
    d.tile = resolve(d.tile, kDefaultTile);
    if (d.max_pairs < 1 || d.max_len < 1 || d.alphabet < 1 || d.alphabet > 256 || d.flags != 0 ||
        d.slots < 0)
        return LCS_E_INVAL;
    // 128- to 1024-row base strips: staged and per-pair modes only (checked at submit)
    const bool tall = d.base_rows == 128 || d.base_rows == 256 || d.base_rows == 512 || d.base_rows == 1024;
    if (!valid_shape(tall ? 64 : d.base_rows, d.tile)) return LCS_E_INVAL;
    if (d.slots == 0 || d.slots > d.max_pairs) d.slots = d.max_pairs;
    Layout L;
    if (!make_layout(d.max_len, d.max_len, d.alphabet, d.base_rows, d.tile, L)) return LCS_E_TOO_BIG;
    if ((int32_t)L.lev.size() > kMaxLev) return LCS_E_TOO_BIG;
    b->d = d;
    b->slot_bytes = align256(L.total);
    b->ctr_per_pair = counters_per_pair(d.max_len, d.base_rows);
    int64_t off = 0;
    b->off_ctl = off;
    off += 256;
    b->off_pairs = off;
    off = align256(off + (int64_t)sizeof(PairRec) * d.max_pairs);
    b->off_ctr = off;
    off = align256(off + 4 * (int64_t)b->ctr_per_pair * d.max_pairs);
    // staged mode: per step, the participating pairs (int32) and their first
    // items (int64, one extra entry per wave)
    // a pair appears at most once per step; each listing costs 4 + 8 bytes, a
    // wave adds one 8-byte total and 8 bytes of alignment per step
    b->stage_bytes = (int64_t)kMaxStages * 32 * ((int64_t)d.max_pairs + 2) + 4096;
    b->off_stage = off;
    off = align256(off + b->stage_bytes);
    b->off_slots = off;
    off += b->slot_bytes * d.slots;
    b->total = off;
    return LCS_OK;
}

extern "C" int32_t lcs_batch_plan(const lcs_batch_desc *desc, lcs_batch_t *out, size_t *ws_bytes) {
    if (!desc || !out || !ws_bytes) return LCS_E_INVAL;
    *out = nullptr;
    lcs_batch_s *b = new (std::nothrow) lcs_batch_s();
    if (!b) return LCS_E_NOMEM;
    const int32_t rc = plan_sizes(desc, b);
    if (rc != LCS_OK) {
        delete b;
        return rc;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&b->host_pairs), sizeof(PairRec) * b->d.max_pairs,
                      hipHostMallocDefault) != hipSuccess) {
        delete b;
        return LCS_E_NOMEM;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&b->host_stage), b->stage_bytes, hipHostMallocDefault) !=
        hipSuccess) {
        hipHostFree(b->host_pairs);
        delete b;
        return LCS_E_NOMEM;
    }
    int dev = 0, ncu = 0, per = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e = hipSuccess;
    switch (b->d.base_rows) {
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<16>, kBlock, 0); break;
        case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<32>, kBlock, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persistent<64>, kBlock, 0); break;
    }
    if (e != hipSuccess || per < 1 || ncu < 1) {
        hipHostFree(b->host_stage);
        hipHostFree(b->host_pairs);
        delete b;
        return LCS_E_HIP;
    }
    b->resident = per * ncu;
    int per_pq = 0;
    switch (b->d.base_rows) {
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_pq, k_pair_queue<16>, kBlock, 0); break;
        case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_pq, k_pair_queue<32>, kBlock, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_pq, k_pair_queue<64>, kBlock, 0); break;
    }
    if (e != hipSuccess || per_pq < 1) {
        hipHostFree(b->host_stage);
        hipHostFree(b->host_pairs);
        delete b;
        return LCS_E_HIP;
    }
    b->resident_pq = per_pq * ncu;
    if (hipEventCreateWithFlags(&b->copied, hipEventDisableTiming) != hipSuccess) {
        hipHostFree(b->host_stage);
        hipHostFree(b->host_pairs);
        delete b;
        return LCS_E_HIP;
    }
    if (opt_in_stage_lds() != hipSuccess) {  // done here, outside any graph capture
        (void)hipGetLastError();
        hipEventDestroy(b->copied);
        hipHostFree(b->host_stage);
        hipHostFree(b->host_pairs);
        delete b;
        return LCS_E_HIP;
    }
    *ws_bytes = (size_t)b->total;
    *out = b;
    return LCS_OK;
}

extern "C" int32_t lcs_batch_destroy(lcs_batch_t b) {
    if (!b) return LCS_OK;
    if (b->gexec) hipGraphExecDestroy(b->gexec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->copied) {
        hipEventSynchronize(b->copied);
        hipEventDestroy(b->copied);
    }
    if (b->host_pairs) hipHostFree(b->host_pairs);
    if (b->host_stage) hipHostFree(b->host_stage);
    delete b;
    return LCS_OK;
}

// Pair record: layout inside the slot, counters and task stages.
static bool make_pair(const lcs_batch_s *B, const lcs_pair_desc &pd, int32_t p, int64_t wit_off,
                      PairRec &R) {
    memset(&R, 0, sizeof(R));
    Layout L;
    if (!make_layout(pd.m, pd.n, B->d.alphabet, B->d.base_rows, B->d.tile, L)) return false;
    if ((int32_t)L.lev.size() > kMaxLev) return false;
    R.ws_off = B->off_slots + (int64_t)(p % B->d.slots) * B->slot_bytes;
    R.a_off = pd.a_off;
    R.b_off = pd.b_off;
    R.wit_off = wit_off;
    R.off_hdr = L.off_hdr;
    R.off_nm = L.off_nm;
    R.total = L.total;
    R.m = pd.m;
    R.n = pd.n;
    R.nlev = (int32_t)L.lev.size();
    R.nanch = L.nanch;
    R.ctr_base = p * B->ctr_per_pair;
    R.sigma = B->d.alphabet;
    R.nvb = vertex_blocks_of(pd.n, kBlock);
    R.jchunk = stage_jchunk(B->d.max_len);
    R.h0 = B->d.base_rows;
    R.comb_stride = L.comb_stride;
    R.off_comb = L.off_comb;
    R.off_leaf = L.off_leaf;
    R.leaf_stride = L.leaf_stride;
    int32_t c = kCtrHead;
    for (int32_t l = 0; l < R.nlev; ++l) {
        R.lev[l] = L.lev[l];
        R.node_off[l] = L.node_off[l];
        R.anch_off[l] = L.anch_off[l];
        R.ctr_lev[l] = c;
        c += 3 * L.lev[l].nstrips;
    }
    int32_t ns = 0, start = 0;
    auto add = [&](int32_t kind, int32_t level, int32_t count) {
        R.stage_kind[ns] = kind;
        R.stage_level[ns] = level;
        R.stage_start[ns] = start;
        start += count;
        ++ns;
    };
    if (R.nlev == 0) {
        add(ST_EMPTY, 0, 1);
    } else {
        add(ST_NM_SYM, 0, R.sigma);
        add(ST_BASE_BLK, 0, L.lev[0].nstrips * R.nvb);
        for (int32_t l = 1; l < R.nlev; ++l) {
            add(ST_ANCHOR, l, L.lev[l].npairs * L.nanch);
            add(ST_BRACKET_CH, l, L.lev[l].npairs * (L.nanch - 1) * level_chunks_of(R, l));
        }
        add(ST_LENGTH, R.nlev - 1, 1);
        for (int32_t l = R.nlev - 1; l >= 1; --l) add(ST_SPLIT, l, L.lev[l].nstrips);
        add(ST_LEAF, 0, L.lev[0].nstrips);
    }
    R.stage_start[ns] = start;
    R.nstages = ns;
    R.ntasks = start;
    R.nctr = c;
    return R.nctr <= B->ctr_per_pair && R.total <= B->slot_bytes;
}

// Tasks per chunk of the persistent mode: a chunk pays one acquire and one
// release (each a maintenance of the die's whole L2) instead of one per task,
// and runs its tasks one after another in one work-group.
constexpr int32_t kPersistChunk = 16;

// Global task order of the persistent mode: for every wave of `slots` pairs,
// the steps of the method in order (step_rank), and for each step the stage
// of every pair of the wave that has it, cut into chunks of at most `chunk`
// tasks.  Writes the segments (at most cap) and returns their number, or -1;
// *nchunks and *ntasks = the totals.
static int64_t build_segments(const PairRec *R, int32_t count, int32_t slots, int32_t chunk, Seg *segs,
                              int64_t cap, int64_t *nchunks, int64_t *ntasks) {
    int64_t ns = 0, g = 0, t = 0;
    std::vector<int32_t> cur;
    for (int32_t p0 = 0; p0 < count; p0 += slots) {
        const int32_t p1 = std::min(count, p0 + slots);
        cur.assign((size_t)(p1 - p0), 0);
        for (int32_t r = 0; r <= step_rank(ST_LEAF, 0); ++r)
            for (int32_t p = p0; p < p1; ++p) {
                const PairRec &P = R[p];
                int32_t &st = cur[(size_t)(p - p0)];
                if (st >= P.nstages || step_rank(P.stage_kind[st], P.stage_level[st]) != r) continue;
                const int32_t c = stage_tasks(P, st);
                if (c > 0) {
                    if (ns >= cap) return -1;
                    segs[ns++] = Seg{g, p, st};
                    g += (c + chunk - 1) / chunk;
                    t += c;
                }
                ++st;
            }
        for (int32_t p = p0; p < p1; ++p)  // every stage placed (ranks increase along a pair)
            if (cur[(size_t)(p - p0)] != R[p].nstages) return -1;
    }
    *nchunks = g;
    *ntasks = t;
    return ns;
}

static uint64_t mix(uint64_t h, uint64_t v) { return (h ^ v) * 0x100000001b3ull; }

extern "C" int32_t lcs_batch_submit(lcs_batch_t B, const lcs_pair_desc *pairs, int32_t count,
                                    const uint8_t *symbols, int64_t symbols_len, int32_t *lengths,
                                    int32_t *a_idx, int32_t *b_idx, int64_t witness_capacity,
                                    void *workspace, size_t workspace_bytes, uint32_t mode,
                                    void *stream) {
    if (!B || (count > 0 && (!pairs || !lengths)) || count < 0 || !workspace) return LCS_E_INVAL;
    if (count > B->d.max_pairs) return LCS_E_TOO_BIG;
    {
        const uint32_t kinds = mode & (LCS_BATCH_PER_PAIR | LCS_BATCH_STAGED | LCS_BATCH_PAIR_QUEUE);
        if ((mode & ~(uint32_t)(LCS_BATCH_PER_PAIR | LCS_BATCH_GRAPH | LCS_BATCH_STAGED |
                                LCS_BATCH_PAIR_QUEUE)) != 0 ||
            (kinds & (kinds - 1)) != 0)  // at most one of them
            return LCS_E_INVAL;
    }
    // the persistent and pair-queue kernels append rows: base strips of at most 64 rows
    if (B->d.base_rows > kWave && !(mode & (LCS_BATCH_STAGED | LCS_BATCH_PER_PAIR))) return LCS_E_INVAL;
    if ((size_t)B->total > workspace_bytes) return LCS_E_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return LCS_E_INVAL;
    int64_t wit = 0;
    for (int32_t p = 0; p < count; ++p) {
        const lcs_pair_desc &pd = pairs[p];
        if (pd.m < 0 || pd.n < 0 || pd.a_off < 0 || pd.b_off < 0) return LCS_E_INVAL;
        if (pd.m > B->d.max_len || pd.n > B->d.max_len) return LCS_E_TOO_BIG;
        if (pd.a_off + pd.m > symbols_len || pd.b_off + pd.n > symbols_len) return LCS_E_INVAL;
        wit += pd.m < pd.n ? pd.m : pd.n;
    }
    if (wit > witness_capacity) return LCS_E_CAPACITY;
    if (wit > 0 && (!a_idx || !b_idx)) return LCS_E_INVAL;
    if (count > 0 && !symbols) return LCS_E_INVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    if (count == 0) return LCS_OK;

    if (mode & LCS_BATCH_PER_PAIR) {
        int64_t woff = 0;
        for (int32_t p = 0; p < count; ++p) {
            const lcs_pair_desc &pd = pairs[p];
            Layout L;
            if (!make_layout(pd.m, pd.n, B->d.alphabet, B->d.base_rows, B->d.tile, L)) return LCS_E_TOO_BIG;
            uint8_t *slot = ws + B->off_slots + (int64_t)(p % B->d.slots) * B->slot_bytes;
            int32_t rc = enqueue_build(L, slot, symbols + pd.a_off, symbols + pd.b_off, s, nullptr);
            if (rc == LCS_OK)
                rc = enqueue_trace(L, slot, symbols + pd.a_off, a_idx + woff, b_idx + woff, s, nullptr);
            if (rc != LCS_OK) return rc;
            hipLaunchKernelGGL(k_finish_pair, dim3(1), dim3(64), 0, s,
                               reinterpret_cast<const int32_t *>(slot + L.off_hdr), lengths + p);
            if (hipGetLastError() != hipSuccess) return LCS_E_HIP;
            woff += pd.m < pd.n ? pd.m : pd.n;
        }
        return LCS_OK;
    }

    // The previous submit's copy of the staging records must have run before
    // they are rewritten.
    if (hipEventSynchronize(B->copied) != hipSuccess) return LCS_E_HIP;
    int64_t woff = 0, tbase = 0, nseg = 0, nchunks = 0;
    uint64_t key = 0xcbf29ce484222325ull;  // graph key: the pairs' shapes, buffers and mode
    for (int32_t p = 0; p < count; ++p) {
        if (!make_pair(B, pairs[p], p, woff, B->host_pairs[p])) return LCS_E_TOO_BIG;
        woff += pairs[p].m < pairs[p].n ? pairs[p].m : pairs[p].n;
        tbase += B->host_pairs[p].ntasks;
        key = mix(mix(key, (uint64_t)pairs[p].m), (uint64_t)pairs[p].n);
    }
    if (!(mode & (LCS_BATCH_STAGED | LCS_BATCH_PAIR_QUEUE))) {  // persistent: the task order
        int64_t total = 0;
        nseg = build_segments(B->host_pairs, count, B->d.slots, kPersistChunk,
                              reinterpret_cast<Seg *>(B->host_stage), B->stage_bytes / (int64_t)sizeof(Seg),
                              &nchunks, &total);
        if (nseg < 1 || total != tbase) return LCS_E_TOO_BIG;
    }
    // staged mode: pack the pairs' layouts into the slot area in waves and
    // list, per step, the items of every pair of the wave
    struct StageLaunch {
        int32_t kind, level, npairs;
        int64_t pair_off, first_off, items;  // byte offsets in the stage tables
    };
    std::vector<StageLaunch> launches;
    if (mode & LCS_BATCH_STAGED) {
        const int64_t arena = B->slot_bytes * B->d.slots;
        std::vector<int32_t> wave_start(1, 0);
        int64_t used = 0;
        for (int32_t p = 0; p < count; ++p) {
            PairRec &R = B->host_pairs[p];
            const int64_t need = align256(R.total);
            if (used + need > arena) {
                wave_start.push_back(p);
                used = 0;
            }
            R.ws_off = B->off_slots + used;
            used += need;
        }
        wave_start.push_back(count);
        int64_t soff = 0;
        uint8_t *tab = B->host_stage;
        for (size_t w = 0; w + 1 < wave_start.size(); ++w) {
            const int32_t p0 = wave_start[w], p1 = wave_start[w + 1];
            int32_t lmax = 0;
            for (int32_t p = p0; p < p1; ++p) lmax = std::max(lmax, B->host_pairs[p].nlev - 1);
            auto add_stage = [&](int32_t kind, int32_t level, auto items_of) {
                std::vector<int32_t> ps;
                std::vector<int64_t> fs;
                int64_t tot = 0;
                for (int32_t p = p0; p < p1; ++p) {
                    const int64_t c = items_of(B->host_pairs[p]);
                    if (c <= 0) continue;
                    ps.push_back(p);
                    fs.push_back(tot);
                    tot += c;
                }
                if (ps.empty()) return;
                fs.push_back(tot);
                if (soff + 12 * (int64_t)ps.size() + 32 > B->stage_bytes) {
                    soff = B->stage_bytes + 1;  // reported after the loop; nothing written
                    return;
                }
                StageLaunch sl{kind, level, (int32_t)ps.size(), soff, 0, tot};
                memcpy(tab + soff, ps.data(), 4 * ps.size());
                soff = (soff + 4 * (int64_t)ps.size() + 7) & ~(int64_t)7;
                sl.first_off = soff;
                memcpy(tab + soff, fs.data(), 8 * fs.size());
                soff += 8 * (int64_t)fs.size();
                launches.push_back(sl);
            };
            const int32_t sig = B->d.alphabet;
            const int32_t sjc = stage_jchunk(B->d.max_len);
            add_stage(ST_EMPTY, 0, [](const PairRec &R) -> int64_t { return R.nlev == 0 ? 1 : 0; });
            add_stage(ST_NM_SYM, 0, [sig](const PairRec &R) -> int64_t { return R.nlev ? sig : 0; });
            // base strips by combing: one work-group per strip, one wave per
            // run of kStageRun vertices
            add_stage(ST_COMB, 0, [](const PairRec &R) -> int64_t { return R.nlev ? R.lev[0].nstrips : 0; });
            add_stage(ST_DGEN, 0, [](const PairRec &R) -> int64_t {
                return R.nlev ? (int64_t)R.lev[0].nstrips * ((R.n + 2 + kStageRun - 1) / kStageRun) : 0;
            });
            for (int32_t l = 1; l <= lmax; ++l) {
                add_stage(ST_ANCHOR, l, [l](const PairRec &R) -> int64_t {
                    return R.nlev > l ? (int64_t)R.lev[l].npairs * R.nanch : 0;
                });
                add_stage(ST_BRACKET_CH, l, [l, sjc](const PairRec &R) -> int64_t {
                    if (R.nlev <= l) return 0;
                    const int32_t H = 2 * R.lev[l - 1].hfull + 1;
                    const int32_t nch = std::max(1, (H - 1 + sjc - 1) / sjc);
                    return (int64_t)R.lev[l].npairs * (R.nanch - 1) * nch;
                });
            }
            add_stage(ST_LENGTH, 0, [](const PairRec &R) -> int64_t { return R.nlev ? 1 : 0; });
            for (int32_t l = lmax; l >= 1; --l)
                add_stage(ST_SPLIT, l, [l](const PairRec &R) -> int64_t {
                    return R.nlev > l ? R.lev[l].nstrips : 0;
                });
            add_stage(B->d.base_rows > kWave ? ST_LEAF_TALL : ST_LEAF, 0,
                      [](const PairRec &R) -> int64_t { return R.nlev ? R.lev[0].nstrips : 0; });
        }
        if (soff > B->stage_bytes) return LCS_E_TOO_BIG;
    }
    if (mode & LCS_BATCH_PAIR_QUEUE) {  // queue order: largest pair first
        if (4 * (int64_t)count > B->stage_bytes) return LCS_E_TOO_BIG;
        int32_t *order = reinterpret_cast<int32_t *>(B->host_stage);
        for (int32_t p = 0; p < count; ++p) order[p] = p;
        std::stable_sort(order, order + count, [&](int32_t x, int32_t y) {
            return (int64_t)pairs[x].m * pairs[x].n > (int64_t)pairs[y].m * pairs[y].n;
        });
    }
    BatchArgs A;
    A.pairs = reinterpret_cast<const PairRec *>(ws + B->off_pairs);
    A.npairs = count;
    A.slots = B->d.slots;
    A.nchunks = nchunks;
    A.chunk = kPersistChunk;
    A.ws = ws;
    A.symbols = symbols;
    A.lengths = lengths;
    A.a_idx = a_idx;
    A.b_idx = b_idx;
    A.ctr = reinterpret_cast<int32_t *>(ws + B->off_ctr);
    A.next = reinterpret_cast<unsigned long long *>(ws + B->off_ctl);
    A.gerr = reinterpret_cast<int32_t *>(ws + B->off_ctl + 8);
    A.sigma = B->d.alphabet;
    A.tile = B->d.tile;
    A.segs = reinterpret_cast<const Seg *>(ws + B->off_stage);
    A.nseg = nseg;
    A.base_rows = B->d.base_rows;
    switch (B->d.base_rows) {
        case 16: A.base_mode = base_tab_mode<16>(B->d.max_len, B->d.alphabet); break;
        case 32: A.base_mode = base_tab_mode<32>(B->d.max_len, B->d.alphabet); break;
        default: A.base_mode = base_tab_mode<64>(B->d.max_len, B->d.alphabet); break;
    }
    const int64_t nctr = (int64_t)B->ctr_per_pair * count;
    const int32_t grid = B->resident;

    auto enqueue = [&](hipStream_t st) -> int32_t {
        if (hipMemcpyAsync(ws + B->off_pairs, B->host_pairs, sizeof(PairRec) * count,
                           hipMemcpyHostToDevice, st) != hipSuccess)
            return LCS_E_HIP;
        if (mode & LCS_BATCH_STAGED) {
            int64_t tb = 0;
            for (const auto &sl : launches) tb = std::max(tb, sl.first_off + 8 * (int64_t)(sl.npairs + 1));
            if (tb > 0 && hipMemcpyAsync(ws + B->off_stage, B->host_stage, tb, hipMemcpyHostToDevice, st) !=
                              hipSuccess)
                return LCS_E_HIP;
            if (hipEventRecord(B->copied, st) != hipSuccess) return LCS_E_HIP;
            for (const auto &sl : launches) {
                StageArgs S;
                S.kind = sl.kind;
                S.level = sl.level;
                S.npairs = sl.npairs;
                S.jchunk = stage_jchunk(B->d.max_len);
                S.cols = B->d.max_len;
                S.pair = reinterpret_cast<const int32_t *>(ws + B->off_stage + sl.pair_off);
                S.first = reinterpret_cast<const int64_t *>(ws + B->off_stage + sl.first_off);
                if (sl.items >= (int64_t)1 << 31) return LCS_E_TOO_BIG;
                const dim3 grid((unsigned)sl.items);
                hipError_t e;
                switch (B->d.base_rows) {
                    case 16: e = launch_stage<16>(A, S, grid, st); break;
                    case 32: e = launch_stage<32>(A, S, grid, st); break;
                    default: e = launch_stage<64>(A, S, grid, st); break;
                }
                if (e != hipSuccess) return LCS_E_HIP;
            }
            return LCS_OK;
        }
        if (mode & LCS_BATCH_PAIR_QUEUE) {
            if (hipMemcpyAsync(ws + B->off_stage, B->host_stage, 4 * (size_t)count,
                               hipMemcpyHostToDevice, st) != hipSuccess)
                return LCS_E_HIP;
            if (hipEventRecord(B->copied, st) != hipSuccess) return LCS_E_HIP;
            hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st,
                               reinterpret_cast<int32_t *>(ws + B->off_ctl), (int64_t)16, 0);
            // one slot per work-group: at most `slots` of them
            const int32_t g = std::max(1, std::min(std::min(B->resident_pq, B->d.slots), count));
            const int32_t *order = reinterpret_cast<const int32_t *>(ws + B->off_stage);
            switch (B->d.base_rows) {
                case 16: hipLaunchKernelGGL(k_pair_queue<16>, dim3(g), dim3(kBlock), 0, st, A, order, B->off_slots, B->slot_bytes); break;
                case 32: hipLaunchKernelGGL(k_pair_queue<32>, dim3(g), dim3(kBlock), 0, st, A, order, B->off_slots, B->slot_bytes); break;
                default: hipLaunchKernelGGL(k_pair_queue<64>, dim3(g), dim3(kBlock), 0, st, A, order, B->off_slots, B->slot_bytes); break;
            }
            return hipGetLastError() == hipSuccess ? LCS_OK : LCS_E_HIP;
        }
        if (hipMemcpyAsync(ws + B->off_stage, B->host_stage, sizeof(Seg) * (size_t)nseg,
                           hipMemcpyHostToDevice, st) != hipSuccess)
            return LCS_E_HIP;
        if (hipEventRecord(B->copied, st) != hipSuccess) return LCS_E_HIP;
        hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, reinterpret_cast<int32_t *>(ws + B->off_ctl),
                           (int64_t)16, 0);
        hipLaunchKernelGGL(k_fill, dim3((unsigned)((nctr + 255) / 256 < 1024 ? (nctr + 255) / 256 : 1024)),
                           dim3(256), 0, st, A.ctr, nctr, 0);
        switch (B->d.base_rows) {
            case 16: hipLaunchKernelGGL(k_persistent<16>, dim3(grid), dim3(kBlock), 0, st, A); break;
            case 32: hipLaunchKernelGGL(k_persistent<32>, dim3(grid), dim3(kBlock), 0, st, A); break;
            default: hipLaunchKernelGGL(k_persistent<64>, dim3(grid), dim3(kBlock), 0, st, A); break;
        }
        return hipGetLastError() == hipSuccess ? LCS_OK : LCS_E_HIP;
    };

    if (!(mode & LCS_BATCH_GRAPH)) return enqueue(s);

    // graph: captured once per (count, buffers, tasks), replayed afterwards.
    // Every device pointer the captured kernels receive is part of the key.
    key = mix(key, (uint64_t)count);
    key = mix(key, (uint64_t)(uintptr_t)ws);
    key = mix(key, (uint64_t)(uintptr_t)symbols);
    key = mix(key, (uint64_t)(uintptr_t)lengths);
    key = mix(key, (uint64_t)(uintptr_t)a_idx);
    key = mix(key, (uint64_t)(uintptr_t)b_idx);
    key = mix(key, (uint64_t)tbase);
    key = mix(key, (uint64_t)mode);
    if (!B->gexec || B->gkey != key) {
        if (B->gexec) hipGraphExecDestroy(B->gexec);
        if (B->graph) hipGraphDestroy(B->graph);
        B->gexec = nullptr;
        B->graph = nullptr;
        hipStream_t cs;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return LCS_E_HIP;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            hipStreamDestroy(cs);
            return LCS_E_HIP;
        }
        const int32_t rc = enqueue(cs);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        hipStreamDestroy(cs);
        if (rc != LCS_OK || e != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return LCS_E_HIP;
        }
        if (hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(g);
            return LCS_E_HIP;
        }
        B->graph = g;
        B->gkey = key;
    }
    return hipGraphLaunch(B->gexec, s) == hipSuccess ? LCS_OK : LCS_E_HIP;
}

// status of the last persistent run (device word written by the kernel)
extern "C" int32_t lcs_batch_status(lcs_batch_t B, void *workspace, void *stream) {
    if (!B || !workspace) return LCS_E_INVAL;
    int32_t err = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(&err, static_cast<uint8_t *>(workspace) + B->off_ctl + 8, 4,
                       hipMemcpyDeviceToHost, s) != hipSuccess)
        return LCS_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return LCS_E_HIP;
    return err ? LCS_E_HIP : LCS_OK;
}

// Host simulation of the persistent schedule for a batch (no device work):
// builds the pair records exactly as lcs_batch_submit does, then checks that
//  - every counter index a task waits on or raises lies inside the counters of
//    its own pair (or, for the slot-reuse wait, of the pair it waits for);
//  - the task order's segments cover every stage of every pair once, in
//    order, each with the chunks it needs;
//  - run one stage at a time in that order, every wait of every task of the
//    stage is already met by earlier stages (so every dependency points to a
//    smaller chunk number and a chunk may wait for all its inputs before it
//    runs: the queue drains);
//  - every wait's target equals the total number of raises of its counter
//    (a met wait proves that all of its producers have finished);
//  - every task of a pair is an ancestor of that pair's finishing tasks, so
//    the slot-reuse wait orders ALL work of the previous occupant of a slot
//    before the new pair's first task;
//  - each pair's layout fits its slot.
// Returns LCS_OK or LCS_E_STATE (schedule defect), LCS_E_INVAL, LCS_E_TOO_BIG.
extern "C" int32_t lcs_batch_selftest(const lcs_batch_desc *desc, const lcs_pair_desc *pairs,
                                      int32_t count) {
    if (!desc || (count > 0 && !pairs) || count < 0) return LCS_E_INVAL;
    if (desc->base_rows > kWave) return LCS_E_INVAL;  // the persistent schedule appends rows (<= 64)
    lcs_batch_s b;
    const int32_t rc = plan_sizes(desc, &b);
    if (rc != LCS_OK) return rc;
    if (count > b.d.max_pairs) return LCS_E_TOO_BIG;
    std::vector<PairRec> R((size_t)count);
    int64_t woff = 0, tbase = 0;
    for (int32_t p = 0; p < count; ++p) {
        if (pairs[p].m < 0 || pairs[p].n < 0 || pairs[p].m > b.d.max_len || pairs[p].n > b.d.max_len)
            return LCS_E_TOO_BIG;
        if (!make_pair(&b, pairs[p], p, woff, R[p])) return LCS_E_STATE;
        woff += pairs[p].m < pairs[p].n ? pairs[p].m : pairs[p].n;
        tbase += R[p].ntasks;
    }
    std::vector<Seg> segs((size_t)count * kMaxStages + 1);
    int64_t ntot = 0, nch = 0;
    const int64_t nseg = count ? build_segments(R.data(), count, b.d.slots, kPersistChunk, segs.data(),
                                                (int64_t)segs.size(), &nch, &ntot)
                               : 0;
    if (nseg < 0 || ntot != tbase) return LCS_E_STATE;
    // every chunk number belongs to exactly one stage, in order, with the
    // chunks that stage needs
    for (int64_t i = 0; i < nseg; ++i) {
        const Seg &g = segs[(size_t)i];
        const int64_t end = i + 1 < nseg ? segs[(size_t)i + 1].start : nch;
        if (end - g.start != (stage_tasks(R[g.pair], g.stage) + kPersistChunk - 1) / kPersistChunk)
            return LCS_E_STATE;
    }
    // the tasks in the global order, stage by stage
    const int64_t nctr = (int64_t)b.ctr_per_pair * count;
    std::vector<int32_t> ctr((size_t)nctr, 0), total((size_t)nctr, 0);
    std::vector<Task> tasks((size_t)tbase);
    std::vector<int64_t> first((size_t)nseg + 1, 0);  // first task of each stage
    for (int64_t i = 0, t = 0; i < nseg; ++i) {
        const Seg &g = segs[(size_t)i];
        first[(size_t)i] = t;
        for (int32_t u = 0; u < stage_tasks(R[g.pair], g.stage); ++u)
            tasks[(size_t)t++] = decode_task(R.data(), b.d.slots, g.pair, g.stage, u);
        first[(size_t)i + 1] = t;
    }
    for (int64_t t = 0; t < tbase; ++t) {
        const Task &T = tasks[t];
        const PairRec &P = R[T.pair];
        for (int32_t i = 0; i < T.nsig; ++i) {
            const int32_t c = T.sig_idx[i];
            if (c < P.ctr_base || c >= P.ctr_base + P.nctr) return LCS_E_STATE;
            ++total[c];
        }
    }
    // consumers of each counter, for the ancestor check
    std::vector<std::vector<int64_t>> consumers((size_t)nctr);
    // run stage by stage: every wait of every task of a stage is met by the
    // stages before it (so a chunk may wait for all of its tasks' inputs
    // before it runs any of them), then the stage's raises are applied
    for (int64_t i = 0; i < nseg; ++i) {
        for (int64_t t = first[(size_t)i]; t < first[(size_t)i + 1]; ++t) {
            const Task &T = tasks[t];
            const PairRec &P = R[T.pair];
            for (int32_t w = 0; w < T.nwait; ++w) {
                const int32_t c = T.wait_idx[w];
                if (c < 0 || c >= nctr) return LCS_E_STATE;
                const bool own = c >= P.ctr_base && c < P.ctr_base + P.nctr;
                const bool prev = (T.kind == ST_NM_SYM || T.kind == ST_EMPTY) && T.pair >= b.d.slots &&
                                  c == R[T.pair - b.d.slots].ctr_base + kCtrLeaves;
                if (!own && !prev) return LCS_E_STATE;
                if (ctr[c] < T.wait_tgt[w]) return LCS_E_STATE;       // not met in stage order
                if (T.wait_tgt[w] != total[c]) return LCS_E_STATE;    // met before all producers ran
                if (own) consumers[c].push_back(t);
            }
        }
        for (int64_t t = first[(size_t)i]; t < first[(size_t)i + 1]; ++t)
            for (int32_t k = 0; k < tasks[t].nsig; ++k) ++ctr[tasks[t].sig_idx[k]];
    }
    // every task must lead (through its own pair's counters) to a finishing task
    std::vector<char> reach((size_t)tbase, 0);
    for (int64_t t = tbase - 1; t >= 0; --t) {
        const Task &T = tasks[t];
        if (T.kind == ST_LEAF || T.kind == ST_EMPTY) {
            reach[t] = 1;
            continue;
        }
        for (int32_t i = 0; i < T.nsig && !reach[t]; ++i)
            for (int64_t c : consumers[T.sig_idx[i]])
                if (reach[c]) {
                    reach[t] = 1;
                    break;
                }
        if (!reach[t]) return LCS_E_STATE;
    }
    return LCS_OK;
}
