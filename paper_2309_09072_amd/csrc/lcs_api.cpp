// C ABI of the single-pair path (include/lcs.h): planning, the breakout-matrix
// build, length, witness trace and matrix views.  Host code only; every step
// of the method runs in the kernels of lcs_kernels.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "lcs.h"
#include "lcs_launch.h"
#include "lcs_plan.h"

using namespace lcs;

namespace lcs {

// Optional per-launch timing: HIP events recorded around each launch.
struct Recorder {
    struct Rec {
        int32_t kind, level;
        int64_t bytes;
        hipEvent_t beg, end;
        bool ended;
    };
    static constexpr size_t kMaxRecords = 1 << 15;
    std::vector<hipEvent_t> pool;
    std::vector<Rec> recs;
    size_t used = 0;
    hipStream_t s = nullptr;
    bool on = false;

    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void reset(hipStream_t st) {
        recs.clear();
        used = 0;
        s = st;
    }
    void begin(int32_t kind, int32_t level, int64_t bytes) {
        if (!on || recs.size() >= kMaxRecords) return;
        Rec r{kind, level, bytes, take(), take(), false};
        if (r.beg) hipEventRecord(r.beg, s);
        recs.push_back(r);
    }
    void end() {
        if (!on || recs.empty() || recs.back().ended) return;
        recs.back().ended = true;
        if (recs.back().end) hipEventRecord(recs.back().end, s);
    }
    ~Recorder() {
        for (hipEvent_t e : pool) hipEventDestroy(e);
    }
};

}  // namespace lcs

struct lcs_plan_s {
    Recorder rec;
    lcs_plan_desc d{};
    Layout lay;
    bool built = false;
    bool empty = false;
    bool transposed = false;  // an oriented build of (rev b, rev a)
    int32_t m = 0, n = 0;     // sizes of the caller's a and b
    uint8_t *ws = nullptr;
    const uint8_t *a = nullptr;
    const uint8_t *b = nullptr;
};

// Layout of one build.  With LCS_PLAN_ORIENT and m > n the problem built is
// (rev b, rev a): layout (n, m) plus room for the two reversed strings.
static bool plan_layout(const lcs_plan_desc &d, int32_t m, int32_t n, Layout &L, bool *transposed) {
    *transposed = false;
    if ((d.flags & LCS_PLAN_ORIENT) && m > n &&
        make_layout(n, m, d.alphabet, d.base_rows, d.tile, L)) {
        L.off_rev = L.total;
        L.total = align256(L.total + align256(n) + m);
        *transposed = true;
        return true;
    }
    return make_layout(m, n, d.alphabet, d.base_rows, d.tile, L);
}

extern "C" const char *lcs_status_string(int32_t s) {
    switch (s) {
        case LCS_OK: return "LCS_OK";
        case LCS_E_INVAL: return "LCS_E_INVAL: invalid argument";
        case LCS_E_TOO_BIG: return "LCS_E_TOO_BIG: sizes exceed the plan or int32 indexing";
        case LCS_E_WORKSPACE: return "LCS_E_WORKSPACE: workspace too small";
        case LCS_E_HIP: return "LCS_E_HIP: HIP runtime error";
        case LCS_E_SYMBOL: return "LCS_E_SYMBOL: symbol outside the alphabet";
        case LCS_E_CAPACITY: return "LCS_E_CAPACITY: witness buffer too small";
        case LCS_E_STATE: return "LCS_E_STATE: call out of order";
        case LCS_E_NOMEM: return "LCS_E_NOMEM: host allocation failed";
        case LCS_E_BUDGET: return "LCS_E_BUDGET: request exceeds the memory budget";
        case LCS_E_AGAIN: return "LCS_E_AGAIN: queue full";
        default: return "unknown status";
    }
}

namespace lcs {

// shared with the batch and serving code
bool valid_shape(int32_t base_rows, int32_t tile) {
    if (base_rows != 16 && base_rows != 32 && base_rows != 64) return false;
    if (tile < 4 || tile > 32 || (tile & (tile - 1))) return false;
    return true;
}

// single-pair plans also take base strips of 128 to 1024 rows (their base
// strips are combed; the serving loop and the persistent batch modes append
// rows, up to 64)
static bool valid_pair_shape(int32_t base_rows, int32_t tile) {
    if (base_rows == 128 || base_rows == 256 || base_rows == 512 || base_rows == 1024)
        return valid_shape(64, tile);
    return valid_shape(base_rows, tile);
}

int32_t resolve(int32_t v, int32_t dflt) { return v == 0 ? dflt : v; }

static int32_t hip_status(hipError_t e) { return e == hipSuccess ? LCS_OK : LCS_E_HIP; }

// Enqueue the whole build for layout L on workspace ws.
// Algorithmic bytes of one combine level, split by parent rows: each row i of
// the parent costs row i of D_U and D_L (read) and row i of D_G (written).
static void level_bytes(const Layout &L, size_t l, int64_t *anchor, int64_t *bracket) {
    const LevelGeom &c = L.lev[l - 1];
    int64_t per_row = 0;  // summed over the pairs of the level
    for (int32_t p = 0; p < L.lev[l].npairs; ++p) {
        const int32_t hU = c.hfull;
        const int32_t hL = (2 * p + 1 == c.nstrips - 1) ? c.hlast : c.hfull;
        per_row += 4 * (int64_t)((hU + 1) + (hL + 1) + (hU + hL + 1));
    }
    *anchor = per_row * L.nanch;
    *bracket = per_row * (L.n + 2 - L.nanch);
}

int64_t build_bytes(const Layout &L) {
    if (L.lev.empty()) return 0;
    int64_t t = L.lev[0].bytes + L.m;
    for (size_t l = 1; l < L.lev.size(); ++l) {
        int64_t a, b;
        level_bytes(L, l, &a, &b);
        t += a + b;
    }
    return t;
}

int32_t enqueue_build(const Layout &L, uint8_t *ws, const uint8_t *a, const uint8_t *b,
                      hipStream_t s, Recorder *rec) {
    Recorder dummy;
    Recorder &R = rec ? *rec : dummy;
    int32_t *hdr = reinterpret_cast<int32_t *>(ws + L.off_hdr);
    int32_t *nm = reinterpret_cast<int32_t *>(ws + L.off_nm);
    hipError_t e = launch_clear(hdr, kHeaderWords, s);
    if (e != hipSuccess || L.lev.empty()) return hip_status(e);
    R.begin(LCS_PHASE_NEXTMATCH, 0, (int64_t)L.sigma * L.n + 4 * (int64_t)L.sigma * (L.n + 2));
    e = launch_nextmatch(b, L.n, L.sigma, nm, hdr, s);
    R.end();
    if (e != hipSuccess) return LCS_E_HIP;
    const LevelGeom &g0 = L.lev[0];
    R.begin(LCS_PHASE_BASE, 0, g0.bytes + L.m);
    e = launch_base_comb(L.h0, a, b, L.n, L.sigma, reinterpret_cast<int32_t *>(ws + g0.base),
                         reinterpret_cast<int32_t *>(ws + g0.last_off), g0.nstrips, g0.hlast,
                         reinterpret_cast<int32_t *>(ws + L.off_comb), L.comb_stride,
                         reinterpret_cast<int32_t *>(ws + L.off_rec), hdr, s);
    R.end();
    if (e != hipSuccess) return LCS_E_HIP;
    for (size_t l = 1; l < L.lev.size(); ++l) {
        int64_t ba, bb;
        level_bytes(L, l, &ba, &bb);
        const CombineArgs ca = combine_args(L, ws, l);
        R.begin(LCS_PHASE_ANCHOR, (int32_t)l, ba);
        e = launch_anchor(ca, L.lev[l].npairs, s);
        R.end();
        if (e != hipSuccess) return LCS_E_HIP;
        R.begin(LCS_PHASE_BRACKET, (int32_t)l, bb);
        e = launch_bracket(ca, L.lev[l].npairs, s);
        R.end();
        if (e != hipSuccess) return LCS_E_HIP;
    }
    const LevelGeom &top = L.lev.back();
    R.begin(LCS_PHASE_LENGTH, (int32_t)L.lev.size() - 1, 4 * (int64_t)(L.m + 1));
    e = launch_length(reinterpret_cast<const int32_t *>(ws + top.last_off), L.m, L.n, hdr,
                      reinterpret_cast<int4 *>(ws + L.node_off.back()), s);
    R.end();
    return hip_status(e);
}

// Enqueue the witness trace of a finished build.
int32_t enqueue_trace(const Layout &L, uint8_t *ws, const uint8_t *a, int32_t *a_idx,
                      int32_t *b_idx, hipStream_t s, Recorder *rec) {
    Recorder dummy;
    Recorder &R = rec ? *rec : dummy;
    if (L.lev.empty()) return LCS_OK;
    int32_t *hdr = reinterpret_cast<int32_t *>(ws + L.off_hdr);
    int32_t *nm = reinterpret_cast<int32_t *>(ws + L.off_nm);
    const size_t top = L.lev.size() - 1;
    if (top >= 1) {
        if (top >= (size_t)kTraceMaxLev) return LCS_E_TOO_BIG;
        TraceSplitArgs t{};
        int64_t bytes = 0;
        for (size_t l = 1; l <= top; ++l) {
            t.lev[l] = combine_args(L, ws, l);
            bytes += 8 * (int64_t)L.lev[l].nstrips * (L.lev[l - 1].hfull + 1);
        }
        for (size_t l = 0; l <= top; ++l) t.node[l] = reinterpret_cast<int4 *>(ws + L.node_off[l]);
        t.top = (int32_t)top;
        t.err = hdr;
        R.begin(LCS_PHASE_TRACE_SPLIT, (int32_t)top, bytes);
        hipError_t e = launch_trace_splits(t, s);
        R.end();
        if (e != hipSuccess) return LCS_E_HIP;
    }
    const LevelGeom &g0 = L.lev[0];
    R.begin(LCS_PHASE_TRACE_LEAF, 0, (int64_t)L.m + 8 * (int64_t)L.m);
    hipError_t e = launch_trace_leaf(L.h0, a, L.n, L.sigma, nm, g0.nstrips, g0.hlast,
                                     reinterpret_cast<const int4 *>(ws + L.node_off[0]), a_idx,
                                     b_idx, L.m < L.n ? L.m : L.n, hdr, ws + L.off_leaf, L.leaf_stride,
                                     s);
    R.end();
    return hip_status(e);
}

}  // namespace lcs

extern "C" int32_t lcs_plan(const lcs_plan_desc *desc, lcs_plan_t *out, size_t *workspace_bytes) {
    if (!desc || !out || !workspace_bytes) return LCS_E_INVAL;
    *out = nullptr;
    lcs_plan_desc d = *desc;
    if (d.base_rows == 0) {
        // Taller base strips replace combine levels; the trace inside a strip is
        // a chain of its rows, so they pay once there are rows for many strips
        // (measured on MI355X: 64 rows up to 2048 x 2048, 256 at 4096 x 4096,
        // 512 at 4096 x 16384, 512 and 1024 equal at 8192 x 8192, 1024 from
        // 12000 x 12000).
        const bool orient = (d.flags & LCS_PLAN_ORIENT) != 0;
        const int32_t rows = orient ? std::min(d.max_m, d.max_n) : d.max_m;
        const int32_t cols = orient ? std::max(d.max_m, d.max_n) : d.max_n;
        d.base_rows = rows >= 8192                                       ? 1024
                      : (rows >= 4096 && cols >= 8192)                   ? 512
                      : rows >= 4096                                     ? 256
                                                                         : kDefaultBaseRows;
    }
    d.tile = resolve(d.tile, kDefaultTile);
    if (d.max_m < 0 || d.max_n < 0 || d.alphabet < 1 || d.alphabet > 256 ||
        (d.flags & ~(LCS_PLAN_PROFILE | LCS_PLAN_ORIENT)) != 0)
        return LCS_E_INVAL;
    if (!valid_pair_shape(d.base_rows, d.tile)) return LCS_E_INVAL;
    if (d.max_n > 0x7ffffff0 || d.max_m > 0x7ffffff0) return LCS_E_TOO_BIG;
    Layout L;
    if (!make_layout(d.max_m, d.max_n, d.alphabet, d.base_rows, d.tile, L)) return LCS_E_TOO_BIG;
    int64_t total = L.total;
    if (d.flags & LCS_PLAN_ORIENT) {
        // an oriented build of (m, n) uses layout (n, m) (at most layout
        // (max_n, max_m): layouts grow with both sizes) plus the reversed strings
        Layout T;
        if (make_layout(d.max_n, d.max_m, d.alphabet, d.base_rows, d.tile, T)) {
            const int64_t t = align256(T.total + align256(d.max_n) + d.max_m);
            if (t > total) total = t;
        }
    }
    lcs_plan_s *p = new (std::nothrow) lcs_plan_s();
    if (!p) return LCS_E_NOMEM;
    p->d = d;
    p->rec.on = (d.flags & LCS_PLAN_PROFILE) != 0;
    *workspace_bytes = (size_t)total;
    *out = p;
    return LCS_OK;
}

extern "C" int32_t lcs_plan_describe(lcs_plan_t p, lcs_plan_desc *out) {
    if (!p || !out) return LCS_E_INVAL;
    *out = p->d;
    return LCS_OK;
}

extern "C" int32_t lcs_plan_workspace(lcs_plan_t p, int32_t m, int32_t n, size_t *bytes) {
    if (!p || !bytes || m < 0 || n < 0) return LCS_E_INVAL;
    if (m > p->d.max_m || n > p->d.max_n) return LCS_E_TOO_BIG;
    Layout L;
    bool tr = false;
    if (!plan_layout(p->d, m, n, L, &tr)) return LCS_E_TOO_BIG;
    *bytes = (size_t)L.total;
    return LCS_OK;
}

extern "C" int32_t lcs_plan_destroy(lcs_plan_t p) {
    delete p;
    return LCS_OK;
}

extern "C" int32_t lcs_dist_build(lcs_plan_t p, const uint8_t *a, int32_t m, const uint8_t *b,
                                  int32_t n, void *workspace, size_t workspace_bytes,
                                  void *stream) {
    if (!p) return LCS_E_INVAL;
    p->built = false;
    if (m < 0 || n < 0 || !workspace) return LCS_E_INVAL;
    if ((m > 0 && !a) || (n > 0 && !b)) return LCS_E_INVAL;
    if (m > p->d.max_m || n > p->d.max_n) return LCS_E_TOO_BIG;
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return LCS_E_INVAL;
    Layout L;
    bool tr = false;
    if (!plan_layout(p->d, m, n, L, &tr)) return LCS_E_TOO_BIG;
    if ((size_t)L.total > workspace_bytes) return LCS_E_WORKSPACE;
    p->lay = L;
    p->ws = static_cast<uint8_t *>(workspace);
    p->a = a;
    p->b = b;
    p->m = m;
    p->n = n;
    p->transposed = tr;
    p->empty = (m == 0 || n == 0);
    p->rec.s = static_cast<hipStream_t>(stream);
    if (tr) {  // rows: reversed b; columns: reversed a
        uint8_t *rb = p->ws + L.off_rev;
        uint8_t *ra = rb + align256(n);
        if (launch_reverse(b, n, rb, p->rec.s) != hipSuccess ||
            launch_reverse(a, m, ra, p->rec.s) != hipSuccess)
            return LCS_E_HIP;
        p->a = rb;
        p->b = ra;
    }
    const int32_t rc = enqueue_build(L, p->ws, p->a, p->b, static_cast<hipStream_t>(stream), &p->rec);
    if (rc != LCS_OK) return rc;
    p->built = true;
    return LCS_OK;
}

static int32_t read_header(lcs_plan_t p, hipStream_t s, int32_t out[3]) {
    if (hipMemcpyAsync(out, p->ws + p->lay.off_hdr, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
        hipSuccess)
        return LCS_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return LCS_E_HIP;
    if (out[0] & kErrSymbol) return LCS_E_SYMBOL;
    if (out[0] != 0) return LCS_E_HIP;
    return LCS_OK;
}

extern "C" int32_t lcs_length(lcs_plan_t p, int32_t *length_host, void *stream) {
    if (!p || !length_host) return LCS_E_INVAL;
    if (!p->built) return LCS_E_STATE;
    if (p->empty) {
        *length_host = 0;
        return LCS_OK;
    }
    int32_t h[3];
    const int32_t rc = read_header(p, static_cast<hipStream_t>(stream), h);
    if (rc != LCS_OK) return rc;
    *length_host = h[1];
    return LCS_OK;
}

extern "C" int32_t lcs_length_device(lcs_plan_t p, int32_t *length_dev, void *stream) {
    if (!p || !length_dev) return LCS_E_INVAL;
    if (!p->built) return LCS_E_STATE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // empty problems: header words were cleared by the build, hdr[1] == 0
    return launch_copy_len(reinterpret_cast<const int32_t *>(p->ws + p->lay.off_hdr), length_dev, s) ==
                   hipSuccess
               ? LCS_OK
               : LCS_E_HIP;
}

extern "C" int32_t lcs_semilocal(lcs_plan_t p, const int32_t *qi, const int32_t *qk, int32_t count,
                                 int32_t *out, void *stream) {
    if (!p || count < 0 || (count > 0 && (!qi || !qk || !out))) return LCS_E_INVAL;
    if (!p->built || p->transposed) return LCS_E_STATE;
    const int32_t *top = nullptr;
    int32_t m = 0;
    if (!p->empty) {
        top = reinterpret_cast<const int32_t *>(p->ws + p->lay.lev.back().last_off);
        m = p->lay.m;
    }
    return launch_semilocal(top, m, p->lay.n, qi, qk, count, out, static_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? LCS_OK
               : LCS_E_HIP;
}

extern "C" int32_t lcs_path(lcs_plan_t p, const int32_t *a_idx, const int32_t *b_idx,
                            const int32_t *length_dev, int32_t *col_in, int32_t *col_out,
                            void *stream) {
    if (!p || !length_dev || !col_in || !col_out) return LCS_E_INVAL;
    if (!p->built) return LCS_E_STATE;
    const int32_t cap = p->m < p->n ? p->m : p->n;
    if (cap > 0 && (!a_idx || !b_idx)) return LCS_E_INVAL;
    return launch_path(a_idx, b_idx, length_dev, cap, p->m, p->n, col_in, col_out,
                       static_cast<hipStream_t>(stream)) == hipSuccess
               ? LCS_OK
               : LCS_E_HIP;
}

extern "C" int32_t lcs_trace(lcs_plan_t p, int32_t *a_idx, int32_t *b_idx, int32_t capacity,
                             int32_t *length_host, void *stream) {
    if (!p || !length_host) return LCS_E_INVAL;
    if (!p->built) return LCS_E_STATE;
    const int32_t need = p->lay.m < p->lay.n ? p->lay.m : p->lay.n;
    if (capacity < need) return LCS_E_CAPACITY;
    if (p->empty) {
        *length_host = 0;
        return LCS_OK;
    }
    if (!a_idx || !b_idx) return LCS_E_INVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    p->rec.s = s;
    const int32_t rc = enqueue_trace(p->lay, p->ws, p->a, a_idx, b_idx, s, &p->rec);
    if (rc != LCS_OK) return rc;
    if (p->transposed &&
        launch_unflip(reinterpret_cast<const int32_t *>(p->ws + p->lay.off_hdr), a_idx, b_idx,
                      capacity, p->m, p->n, s) != hipSuccess)
        return LCS_E_HIP;
    int32_t h[3];
    const int32_t rc2 = read_header(p, s, h);
    if (rc2 != LCS_OK) return rc2;
    *length_host = h[1];
    return LCS_OK;
}

extern "C" int32_t lcs_plan_levels(lcs_plan_t p, int32_t *levels, int32_t *strips) {
    if (!p || !levels) return LCS_E_INVAL;
    if (!p->built) return LCS_E_STATE;
    *levels = (int32_t)p->lay.lev.size();
    if (strips)
        for (size_t l = 0; l < p->lay.lev.size(); ++l) strips[l] = p->lay.lev[l].nstrips;
    return LCS_OK;
}

extern "C" int32_t lcs_dist_view(lcs_plan_t p, int32_t level, int32_t strip, const int32_t **matrix,
                                 int32_t *rows, int32_t *cols, int32_t *row0) {
    if (!p || !matrix || !rows || !cols || !row0) return LCS_E_INVAL;
    if (!p->built || p->empty) return LCS_E_STATE;
    if (level < 0 || level >= (int32_t)p->lay.lev.size()) return LCS_E_INVAL;
    const LevelGeom &g = p->lay.lev[level];
    if (strip < 0 || strip >= g.nstrips) return LCS_E_INVAL;
    const bool last = strip == g.nstrips - 1;
    const int64_t off = last ? g.last_off : g.base + 4 * (int64_t)strip * (int64_t)strip_elems(p->lay.n, g.hfull);
    *matrix = reinterpret_cast<const int32_t *>(p->ws + off);
    *rows = p->lay.n + 2;
    *cols = (last ? g.hlast : g.hfull) + 1;
    *row0 = strip * g.hfull;
    return LCS_OK;
}

extern "C" int32_t lcs_trace_device(lcs_plan_t p, int32_t *a_idx, int32_t *b_idx, int32_t capacity,
                                    int32_t *length_dev, void *stream) {
    if (!p || !length_dev) return LCS_E_INVAL;
    if (!p->built) return LCS_E_STATE;
    const int32_t need = p->lay.m < p->lay.n ? p->lay.m : p->lay.n;
    if (capacity < need) return LCS_E_CAPACITY;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!p->empty) {
        if (!a_idx || !b_idx) return LCS_E_INVAL;
        p->rec.s = s;
        const int32_t rc = enqueue_trace(p->lay, p->ws, p->a, a_idx, b_idx, s, &p->rec);
        if (rc != LCS_OK) return rc;
        if (p->transposed &&
            launch_unflip(reinterpret_cast<const int32_t *>(p->ws + p->lay.off_hdr), a_idx, b_idx,
                          capacity, p->m, p->n, s) != hipSuccess)
            return LCS_E_HIP;
    }
    return launch_copy_len(reinterpret_cast<const int32_t *>(p->ws + p->lay.off_hdr), length_dev, s) ==
                   hipSuccess
               ? LCS_OK
               : LCS_E_HIP;
}

extern "C" int32_t lcs_plan_profile(lcs_plan_t p, lcs_phase_time *out, int32_t max, int32_t *count) {
    if (!p || !count || (max > 0 && !out)) return LCS_E_INVAL;
    if (!p->rec.on) return LCS_E_STATE;
    const int32_t nrec = (int32_t)p->rec.recs.size();
    *count = nrec;
    for (int32_t i = 0; i < nrec && i < max; ++i) {
        const Recorder::Rec &r = p->rec.recs[i];
        float ms = 0.f;
        if (!r.beg || !r.end) return LCS_E_HIP;
        if (hipEventSynchronize(r.end) != hipSuccess) return LCS_E_HIP;
        if (hipEventElapsedTime(&ms, r.beg, r.end) != hipSuccess) return LCS_E_HIP;
        out[i].kind = r.kind;
        out[i].level = r.level;
        out[i].ms = ms;
        out[i].bytes = r.bytes;
    }
    if (max >= nrec) p->rec.reset(p->rec.s);  // every record delivered: start afresh
    return LCS_OK;
}
