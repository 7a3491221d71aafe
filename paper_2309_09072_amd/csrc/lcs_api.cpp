// C ABI of the single-pair path (include/lcs.h): planning, the breakout-matrix
// build, length, witness trace and matrix views.  Host code only; every step
// of the method runs in the kernels of lcs_kernels.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <new>

#include "lcs.h"
#include "lcs_launch.h"
#include "lcs_plan.h"

using namespace lcs;

struct lcs_plan_s {
    lcs_plan_desc d{};
    Layout lay;
    bool built = false;
    bool empty = false;
    uint8_t *ws = nullptr;
    const uint8_t *a = nullptr;
    const uint8_t *b = nullptr;
};

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
    if (tile < 4 || tile > 64 || (tile & (tile - 1))) return false;
    return true;
}

int32_t resolve(int32_t v, int32_t dflt) { return v == 0 ? dflt : v; }

static int32_t hip_status(hipError_t e) { return e == hipSuccess ? LCS_OK : LCS_E_HIP; }

// Enqueue the whole build for layout L on workspace ws.
int32_t enqueue_build(const Layout &L, uint8_t *ws, const uint8_t *a, const uint8_t *b,
                      hipStream_t s) {
    int32_t *hdr = reinterpret_cast<int32_t *>(ws + L.off_hdr);
    int32_t *nm = reinterpret_cast<int32_t *>(ws + L.off_nm);
    hipError_t e = launch_clear(hdr, kHeaderWords, s);
    if (e != hipSuccess || L.lev.empty()) return hip_status(e);
    e = launch_nextmatch(b, L.n, L.sigma, nm, s);
    if (e != hipSuccess) return LCS_E_HIP;
    const LevelGeom &g0 = L.lev[0];
    e = launch_base(L.h0, a, L.n, L.sigma, nm, reinterpret_cast<int32_t *>(ws + g0.base),
                    reinterpret_cast<int32_t *>(ws + g0.last_off), g0.nstrips, g0.hlast, hdr, s);
    if (e != hipSuccess) return LCS_E_HIP;
    for (size_t l = 1; l < L.lev.size(); ++l) {
        e = launch_combine(combine_args(L, ws, l), L.lev[l].npairs, s);
        if (e != hipSuccess) return LCS_E_HIP;
    }
    const LevelGeom &top = L.lev.back();
    e = launch_length(reinterpret_cast<const int32_t *>(ws + top.last_off), L.m, L.n, hdr,
                      reinterpret_cast<int4 *>(ws + L.node_off.back()), s);
    return hip_status(e);
}

// Enqueue the witness trace of a finished build.
int32_t enqueue_trace(const Layout &L, uint8_t *ws, const uint8_t *a, int32_t *a_idx,
                      int32_t *b_idx, hipStream_t s) {
    if (L.lev.empty()) return LCS_OK;
    int32_t *hdr = reinterpret_cast<int32_t *>(ws + L.off_hdr);
    int32_t *nm = reinterpret_cast<int32_t *>(ws + L.off_nm);
    for (size_t l = L.lev.size() - 1; l >= 1; --l) {
        hipError_t e = launch_trace_split(combine_args(L, ws, l), L.lev[l].nstrips,
                                          reinterpret_cast<const int4 *>(ws + L.node_off[l]),
                                          reinterpret_cast<int4 *>(ws + L.node_off[l - 1]), hdr, s);
        if (e != hipSuccess) return LCS_E_HIP;
    }
    const LevelGeom &g0 = L.lev[0];
    hipError_t e = launch_trace_leaf(L.h0, a, L.n, L.sigma, nm, g0.nstrips, g0.hlast,
                                     reinterpret_cast<const int4 *>(ws + L.node_off[0]), a_idx,
                                     b_idx, hdr, s);
    return hip_status(e);
}

}  // namespace lcs

extern "C" int32_t lcs_plan(const lcs_plan_desc *desc, lcs_plan_t *out, size_t *workspace_bytes) {
    if (!desc || !out || !workspace_bytes) return LCS_E_INVAL;
    *out = nullptr;
    lcs_plan_desc d = *desc;
    d.base_rows = resolve(d.base_rows, kDefaultBaseRows);
    d.tile = resolve(d.tile, kDefaultTile);
    if (d.max_m < 0 || d.max_n < 0 || d.alphabet < 1 || d.alphabet > 256 || d.flags != 0)
        return LCS_E_INVAL;
    if (!valid_shape(d.base_rows, d.tile)) return LCS_E_INVAL;
    if (d.max_n > 0x7ffffff0 || d.max_m > 0x7ffffff0) return LCS_E_TOO_BIG;
    Layout L;
    if (!make_layout(d.max_m, d.max_n, d.alphabet, d.base_rows, d.tile, L)) return LCS_E_TOO_BIG;
    lcs_plan_s *p = new (std::nothrow) lcs_plan_s();
    if (!p) return LCS_E_NOMEM;
    p->d = d;
    *workspace_bytes = (size_t)L.total;
    *out = p;
    return LCS_OK;
}

extern "C" int32_t lcs_plan_workspace(lcs_plan_t p, int32_t m, int32_t n, size_t *bytes) {
    if (!p || !bytes || m < 0 || n < 0) return LCS_E_INVAL;
    if (m > p->d.max_m || n > p->d.max_n) return LCS_E_TOO_BIG;
    Layout L;
    if (!make_layout(m, n, p->d.alphabet, p->d.base_rows, p->d.tile, L)) return LCS_E_TOO_BIG;
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
    if (!make_layout(m, n, p->d.alphabet, p->d.base_rows, p->d.tile, L)) return LCS_E_TOO_BIG;
    if ((size_t)L.total > workspace_bytes) return LCS_E_WORKSPACE;
    p->lay = L;
    p->ws = static_cast<uint8_t *>(workspace);
    p->a = a;
    p->b = b;
    p->empty = (m == 0 || n == 0);
    const int32_t rc = enqueue_build(L, p->ws, a, b, static_cast<hipStream_t>(stream));
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
    const int32_t rc = enqueue_trace(p->lay, p->ws, p->a, a_idx, b_idx, s);
    if (rc != LCS_OK) return rc;
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
