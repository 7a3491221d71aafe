// Per-level kernels of the single-pair path: every launch covers one step of
// the strip recursion for all strips of a level.  The work-group bodies are in
// lcs_device.h and are shared with the persistent batch kernel.
#include "lcs_device.h"
#include "lcs_launch.h"

namespace lcs {

__global__ void __launch_bounds__(kBlock) k_clear(int32_t *words, int32_t count) {
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) words[i] = 0;
}

__global__ void __launch_bounds__(kBlock) k_nextmatch(const uint8_t *b, int32_t n, int32_t sigma,
                                                      int32_t *nm, int32_t *err) {
    __shared__ int32_t lds[kWaves];
    const int32_t x = blockIdx.x;
    nextmatch_block(b, n, x, sigma, nm + (size_t)x * (size_t)(n + 2), lds, err);
}

template <int H0, int kMode>
__global__ void __launch_bounds__(kBlock) k_base(const uint8_t *a, int32_t n, int32_t sigma,
                                                 const int32_t *nm, int32_t *base0, int32_t *last,
                                                 int32_t nstrips, int32_t hlast, int32_t *err) {
    __shared__ __align__(16) uint8_t smem[base_smem_bytes<H0, kMode>()];  // table, then transposition
    const int32_t s = blockIdx.y;
    const bool is_last = (s == nstrips - 1);
    const int32_t h = is_last ? hlast : H0;
    int32_t *out = is_last ? last : base0 + (size_t)s * strip_elems(n, H0);
    base_strip_block<H0, kMode>(a + (size_t)s * H0, h, n, sigma, nm, out, (int32_t)blockIdx.x * kBlock,
                                err, reinterpret_cast<int32_t *>(smem), smem);
}

// Seaweed combing of every base strip, one work-group (NT threads, fewer
// for narrow strings) per strip; region comb holds comb_stride int32 per strip.
template <int NT, int C, bool kPacked>
__global__ void __launch_bounds__(NT) k_comb(const uint8_t *a, const uint8_t *b, int32_t n,
                                             int32_t sigma, int32_t h0, int32_t nstrips,
                                             int32_t hlast, int32_t *comb, int32_t cstride,
                                             int32_t *err) {
    __shared__ int32_t lds[3 * kCombMaxRows + 4 * (NT / kWave)];
    const int32_t s = blockIdx.x;
    const int32_t h = (s == nstrips - 1) ? hlast : h0;
    int32_t *cs = comb + (size_t)s * (size_t)cstride;
    comb_strip_block<NT, C, kPacked>(a + (size_t)s * h0, h, b, n, sigma, cs, cs + n, cs + 2 * (size_t)n,
                                     lds, err);
}

// The same as a pipeline of waves (n <= 32767): 64 C columns per wave.
template <int C>
__global__ void __launch_bounds__(kCombPipeWaves * kWave) k_comb_pipe(const uint8_t *a, const uint8_t *b,
                                                                       int32_t n, int32_t sigma, int32_t h0,
                                                                       int32_t nstrips, int32_t hlast,
                                                                       int32_t *comb, int32_t cstride,
                                                                       int32_t *err) {
    extern __shared__ int32_t lds[];  // (waves + 1) x h0 int32
    const int32_t s = blockIdx.x;
    const int32_t h = (s == nstrips - 1) ? hlast : h0;
    int32_t *cs = comb + (size_t)s * (size_t)cstride;
    comb_strip_pipe<C>(a + (size_t)s * h0, h, b, n, sigma, cs, cs + n, cs + 2 * (size_t)n, lds, err);
}

// The same split into G column segments per strip, one work-group (KW waves of
// C columns per lane: 64 C KW columns) each; work-group s G + g is segment g
// of strip s, so a segment's predecessor is always dispatched before it.
template <int C, int KW>
__global__ void __launch_bounds__(KW * kWave) k_comb_seg(const uint8_t *a, const uint8_t *b, int32_t n,
                                                        int32_t sigma, int32_t h0, int32_t nstrips,
                                                        int32_t hlast, int32_t *comb, int32_t cstride,
                                                        unsigned long long *rec, int32_t G, int32_t *err) {
    extern __shared__ int32_t lds[];  // (KW + 1) x h0 int32
    const int32_t s = (int32_t)blockIdx.x / G, g = (int32_t)blockIdx.x - s * G;
    const int32_t h = (s == nstrips - 1) ? hlast : h0;
    int32_t *cs = comb + (size_t)s * (size_t)cstride;
    unsigned long long *rs = rec + (size_t)s * (size_t)(G - 1) * (size_t)h0;
    comb_strip_seg<C>(a + (size_t)s * h0, h, b, n, sigma, g * KW * kWave * C, g == 0, g == G - 1,
                      g > 0 ? rs + (size_t)(g - 1) * h0 : nullptr, g < G - 1 ? rs + (size_t)g * h0 : nullptr,
                      cs, cs + n, cs + 2 * (size_t)n, lds, err);
}

// Breakout rows of every base strip from its combing: one wave per run of
// `chunk` consecutive vertices of one strip (runs of a strip on one XCD).
template <int E>
__global__ void __launch_bounds__(kBlock) k_dgen(const int32_t *comb, int32_t cstride, int32_t n,
                                                 int32_t h0, int32_t nstrips, int32_t hlast,
                                                 int32_t *base0, int32_t *last, int32_t chunk,
                                                 int32_t nchunks) {
    __shared__ int32_t lst[kWaves][E * kWave];
    const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)threadIdx.x / kWave);
    const int64_t g = (int64_t)xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x,
                                         imax(1, (int32_t)gridDim.x / 8)) * kWaves + wv;
    if (g >= (int64_t)nstrips * nchunks) return;
    const int32_t s = (int32_t)(g / nchunks), ck = (int32_t)(g - (int64_t)s * nchunks);
    const bool is_last = (s == nstrips - 1);
    const int32_t h = is_last ? hlast : h0;
    int32_t *out = is_last ? last : base0 + (size_t)s * strip_elems(n, h0);
    const int32_t *cs = comb + (size_t)s * (size_t)cstride;
    const int32_t i0 = ck * chunk;
    dgen_wave<E>(cs, cs + n, cs + 2 * (size_t)n, h, n, i0, imin(i0 + chunk, n + 2), out, lst[wv]);
}

// Anchor searches of neighbouring vertices gather from nearly the same rows
// and columns of D_L, and those gathers are one cache line each (the anchor
// kernels move ~25x their algorithmic bytes).  The launch is remapped so that
// each XCD runs one contiguous range of (pair, anchor) blocks: a line then
// comes into one L2 and serves the neighbours there.
__device__ __forceinline__ int32_t anchor_block_id() {
    const int32_t N = (int32_t)(gridDim.x * gridDim.y);
    return xcd_block((int32_t)(blockIdx.x + blockIdx.y * gridDim.x), N, imax(1, N / 8));
}

// Anchor search with the D_U row and the k* row of the vertex in LDS
// (dynamic: the search's AnchorSmem, then hc + 1 and 2 hc + 1 values of KT).
template <int NT, int CPT, typename KT>
__global__ void __launch_bounds__(NT) k_anchor_lds(CombineArgs c) {
    extern __shared__ unsigned long long dyn[];
    const int32_t lb = anchor_block_id();
    const int32_t p = lb / (int32_t)gridDim.x, a = lb - p * (int32_t)gridDim.x;
    const StripRef U = child_strip(c, 2 * p), L = child_strip(c, 2 * p + 1);
    int32_t *G = parent_strip(c, p);
    const int32_t vtx = anchor_vertex(a, c.tile, c.n);
    int32_t *Krow = c.anch + ((size_t)p * c.nanch + a) * (size_t)c.hs;
    AnchorSmem<NT, CPT> &sm = *reinterpret_cast<AnchorSmem<NT, CPT> *>(dyn);
    KT *us = reinterpret_cast<KT *>(dyn + sizeof(AnchorSmem<NT, CPT>) / 8);
    KT *ks = us + (c.hc + 1);
    anchor_block_t<true, NT, CPT, KT>(U.d, U.h, L.d, L.h, G, c.n, vtx, Krow, sm, us, ks);
    if (a == c.nanch - 1) {  // sentinel row n + 1
        const int32_t H = U.h + L.h + 1;
        int32_t *srow = G + (size_t)(c.n + 1) * H;
        for (int32_t j = threadIdx.x; j < H; j += NT) srow[j] = c.n + 1;
    }
}

// One anchor search per wave (levels with many short anchor rows): each wave
// has its own slice of dynamic LDS (the search's AnchorSmem, then hc + 1 and
// 2 hc + 1 int32, `bytes` in all) and no block barrier is used, so a wave
// without an anchor simply exits.
template <int CPT>
__global__ void __launch_bounds__(kBlock) k_anchor_wave(CombineArgs c, int32_t bytes) {
    extern __shared__ unsigned long long dyn[];
    const int32_t wv = (int32_t)threadIdx.x / kWave;
    const int32_t lb = anchor_block_id();
    const int32_t p = lb / (int32_t)gridDim.x, a = (lb - p * (int32_t)gridDim.x) * kWaves + wv;
    if (a >= c.nanch) return;
    const StripRef U = child_strip(c, 2 * p), L = child_strip(c, 2 * p + 1);
    int32_t *G = parent_strip(c, p);
    const int32_t vtx = anchor_vertex(a, c.tile, c.n);
    int32_t *Krow = c.anch + ((size_t)p * c.nanch + a) * (size_t)c.hs;
    unsigned long long *base = dyn + (size_t)wv * (size_t)(bytes / 8);
    AnchorSmem<kWave, CPT> &sm = *reinterpret_cast<AnchorSmem<kWave, CPT> *>(base);
    int32_t *us = reinterpret_cast<int32_t *>(base + sizeof(AnchorSmem<kWave, CPT>) / 8);
    int32_t *ks = us + (c.hc + 1);
    anchor_block_t<true, kWave, CPT>(U.d, U.h, L.d, L.h, G, c.n, vtx, Krow, sm, us, ks);
    if (a == c.nanch - 1) {  // sentinel row n + 1
        const int32_t H = U.h + L.h + 1;
        int32_t *srow = G + (size_t)(c.n + 1) * H;
        for (int32_t j = __lane_id(); j < H; j += kWave) srow[j] = c.n + 1;
    }
}

// Anchor search with both rows in global memory (rows too long for LDS).
template <int NT, int CPT>
__global__ void __launch_bounds__(NT) k_anchor(CombineArgs c) {
    __shared__ AnchorSmem<NT, CPT> sm;
    const int32_t lb = anchor_block_id();
    const int32_t p = lb / (int32_t)gridDim.x, a = lb - p * (int32_t)gridDim.x;
    const StripRef U = child_strip(c, 2 * p), L = child_strip(c, 2 * p + 1);
    int32_t *G = parent_strip(c, p);
    const int32_t vtx = anchor_vertex(a, c.tile, c.n);
    int32_t *Krow = c.anch + ((size_t)p * c.nanch + a) * (size_t)c.hs;
    anchor_block_t<false, NT, CPT, int32_t>(U.d, U.h, L.d, L.h, G, c.n, vtx, Krow, sm, nullptr, nullptr);
    if (a == c.nanch - 1) {  // sentinel row n + 1
        const int32_t H = U.h + L.h + 1;
        int32_t *srow = G + (size_t)(c.n + 1) * H;
        for (int32_t j = threadIdx.x; j < H; j += NT) srow[j] = c.n + 1;
    }
}

// At most 64 VGPRs (8 waves per SIMD): with its ~18 KB of LDS eight
// work-groups fit on a CU, and the kernel is bound by dependent round trips
// per work-group, so work-groups in flight count more than a few spills.
template <class C, bool kCoop>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) k_bracket(CombineArgs c) {
    __shared__ BracketSmemT<C> sm;
    const int32_t p = blockIdx.y;
    const int32_t tile = blockIdx.x / c.nchunks, chunk = blockIdx.x - tile * c.nchunks;
    const StripRef U = child_strip(c, 2 * p), L = child_strip(c, 2 * p + 1);
    const int32_t H = U.h + L.h + 1;
    const int32_t nch = imax(1, (H - 1 + c.jchunk - 1) / c.jchunk);
    if (chunk >= nch) return;
    const int32_t j0 = chunk * c.jchunk;
    const int32_t jn = (chunk == nch - 1) ? H - j0 : c.jchunk;
    const int32_t i0 = tile * c.tile;
    const int32_t len = imin(c.tile, c.n - i0);
    int32_t *G = parent_strip(c, p);
    const int32_t *Ka = c.anch + ((size_t)p * c.nanch + tile) * (size_t)c.hs;
    const int32_t *Kb = c.anch + ((size_t)p * c.nanch + tile + 1) * (size_t)c.hs;
    bracket_block<C, kCoop>(U.d, U.h, L.d, L.h, G, c.n, i0, len, j0, jn, Ka, Kb, sm);
}

__global__ void __launch_bounds__(kBlock) k_length(const int32_t *top, int32_t m, int32_t n,
                                                   int32_t *hdr, int4 *root) {
    __shared__ int32_t lds[1];
    length_block(top, m, n, hdr, root, lds);
}

// Every split level of the trace in one work-group (Section II-C: the
// cross column of the node's combine, the smallest k with
// D_L(D_U(s, k), w - k) == e).  Level by level from the top, each parent node
// gets g threads; each thread takes every g-th k of the node's range, R at a
// time with the D_U loads, then the D_L loads, all in flight, and stops at its
// first hit; the hits meet in an LDS minimum.  A level's children are read by
// the next level after a barrier of the same work-group, so one launch
// replaces one launch per level; the nodes of the inner levels stay in LDS
// (up to kSplitNodes per level; only level 0's go to memory, for the leaves).
constexpr int32_t kSplitThreads = 1024;
constexpr int32_t kSplitNodes = 1024;
__global__ void __launch_bounds__(kSplitThreads) k_trace_splits(TraceSplitArgs A) {
    constexpr int32_t R = 4;
    __shared__ int32_t found[kSplitThreads];
    __shared__ int4 nbuf[2][kSplitNodes];
    const int32_t tid = threadIdx.x;
    bool in_lds = false;  // this level's nodes are in nbuf[cur]
    int32_t cur = 0;
    for (int32_t l = A.top; l >= 1; --l) {
        const CombineArgs &c = A.lev[l];
        const bool out_lds = l > 1 && c.nc <= kSplitNodes;
        const int4 *nin = in_lds ? nbuf[cur] : A.node[l];
        int4 *nout = out_lds ? nbuf[cur ^ 1] : A.node[l - 1];
        const int32_t np = c.np, n = c.n;
        int32_t g = kSplitThreads;  // threads per node (power of two)
        while (g > 1 && (int64_t)g * np > kSplitThreads) g >>= 1;
        const int32_t per = kSplitThreads / g;
        for (int32_t b0 = 0; b0 < np; b0 += per) {
            const int32_t pl = tid / g, sub = tid - pl * g, p = b0 + pl;
            if (sub == 0) found[pl] = 0x7fffffff;
            __syncthreads();
            int4 node = make_int4(0, 0, 0, 0);
            bool split = false;
            int32_t s = 0, w = 0, e = 0;
            const int32_t *urow = nullptr;
            StripRef U{}, L{};
            if (p < np) {
                node = nin[p];
                if (2 * p + 1 < c.nc) {
                    split = true;
                    U = child_strip(c, 2 * p);
                    L = child_strip(c, 2 * p + 1);
                    s = umin(node.x, n);
                    w = node.y;
                    e = node.z;
                    urow = U.d + (size_t)s * (U.h + 1);
                    const int32_t lo = imax(0, w - L.h), hi = imin(w, U.h);
                    const int32_t ldL = L.h + 1;
                    bool hit = false;
                    for (int32_t kb = lo + sub; kb <= hi && !hit; kb += g * R) {
                        int32_t xs[R], vs[R];
#pragma unroll
                        for (int t = 0; t < R; ++t) xs[t] = urow[imin(kb + t * g, hi)];
#pragma unroll
                        for (int t = 0; t < R; ++t) {
                            const int32_t k = imin(kb + t * g, hi);
                            vs[t] = ((uint32_t)xs[t] <= (uint32_t)n) ? L.d[(size_t)xs[t] * ldL + (w - k)] : -1;
                        }
#pragma unroll
                        for (int t = 0; t < R; ++t) {
                            const int32_t k = kb + t * g;
                            if (!hit && k <= hi && vs[t] == e) {
                                atomicMin(&found[pl], k);
                                hit = true;
                            }
                        }
                    }
                }
            }
            __syncthreads();
            if (p < np && sub == 0) {
                if (!split) {
                    nout[2 * p] = node;  // carried-up strip: same node one level down
                } else {
                    const int32_t k = found[pl];
                    if (k == 0x7fffffff) {
                        atomicOr(A.err, kErrTrace);
                        nout[2 * p] = make_int4(s, 0, s, node.w);
                        nout[2 * p + 1] = make_int4(s, 0, s, node.w);
                    } else {
                        const int32_t x = umin(urow[k], n);
                        nout[2 * p] = make_int4(s, k, x, node.w);
                        nout[2 * p + 1] = make_int4(x, w - k, e, node.w + k);
                    }
                }
            }
            __syncthreads();
        }
        in_lds = out_lds;
        if (out_lds) cur ^= 1;
    }
}

constexpr int32_t kLeafTab = 4096;  // next-match table entries a leaf block keeps in LDS
template <int H0>
__global__ void __launch_bounds__(kWave) k_trace_leaf(const uint8_t *a, int32_t n, int32_t sigma,
                                                       const int32_t *nm, int32_t nstrips,
                                                       int32_t hlast, const int4 *nodes,
                                                       int32_t *a_idx, int32_t *b_idx,
                                                       int32_t wcap, int32_t *err) {
    __shared__ int32_t lds[(H0 + 1) * (H0 + 1)];
    __shared__ int32_t tab[kLeafTab];
    const int32_t s = blockIdx.x;
    const int32_t h = (s == nstrips - 1) ? hlast : H0;
    trace_leaf_block<H0, true>(a + (size_t)s * H0, h, n, sigma, nm, nodes[s], s * H0, a_idx, b_idx,
                               wcap, err, lds, tab, kLeafTab);
}

// Base strips of 128 to 1024 rows (Ew K = 2, 4, 8, 16 registers of columns): K
// waves per strip; TT: the next-match window's entries.
template <int Ew, int K, typename TT>
__global__ void __launch_bounds__(K * kWave) k_trace_leaf_pipe(const uint8_t *a, int32_t n,
                                                                int32_t sigma, const int32_t *nm,
                                                                int32_t h0, int32_t nstrips,
                                                                int32_t hlast, const int4 *nodes,
                                                                int32_t *a_idx, int32_t *b_idx,
                                                                int32_t wcap, int32_t *err,
                                                                int32_t tabcap, uint8_t *leaf,
                                                                int64_t leaf_stride) {
    constexpr int E = Ew * K;
    extern __shared__ int32_t dyn_tab[];  // tabcap entries of TT: the next-match window
    TT *tab = reinterpret_cast<TT *>(dyn_tab);
    __shared__ int32_t mrow[E * kWave], xs[E * kWave];
    __shared__ int32_t ring[(K - 1) * E * kWave], sync[K + 2];
    const int32_t s = blockIdx.x;
    const int32_t h = (s == nstrips - 1) ? hlast : h0;
    trace_leaf_pipe<Ew, K, TT>(a + (size_t)s * h0, h, n, sigma, nm, nodes[s], s * h0, a_idx, b_idx, wcap,
                           err, tab, tabcap, leaf + (size_t)s * (size_t)leaf_stride, mrow, xs, ring,
                           sync);
}

__global__ void __launch_bounds__(kBlock) k_semilocal(const int32_t *top, int32_t m, int32_t n,
                                                      const int32_t *qi, const int32_t *qk,
                                                      int32_t count, int32_t *out) {
    for (int32_t q = blockIdx.x * kBlock + threadIdx.x; q < count; q += gridDim.x * kBlock)
        out[q] = semilocal_query(top, m, n, qi[q], qk[q]);
}
__global__ void __launch_bounds__(kBlock) k_reverse(const uint8_t *src, int32_t len, uint8_t *dst) {
    for (int32_t t = blockIdx.x * kBlock + threadIdx.x; t < len; t += gridDim.x * kBlock)
        dst[t] = src[len - 1 - t];
}
// Witness of the built problem (rows: reversed b, columns: reversed a), read
// backwards and mapped to indices of a and b.  Thread t swaps entries t and
// L - 1 - t.  L comes from the header (device), clamped to the capacity.
__global__ void __launch_bounds__(kBlock) k_unflip(const int32_t *hdr, int32_t *a_idx, int32_t *b_idx,
                                                   int32_t capacity, int32_t m, int32_t n) {
    const int32_t L = imin(imax(hdr[1], 0), capacity);
    for (int32_t t = blockIdx.x * kBlock + threadIdx.x; 2 * t < L; t += gridDim.x * kBlock) {
        const int32_t u = L - 1 - t;
        const int32_t rt = a_idx[t], ct = b_idx[t], ru = a_idx[u], cu = b_idx[u];
        a_idx[t] = m - 1 - cu;
        b_idx[t] = n - 1 - ru;
        a_idx[u] = m - 1 - ct;
        b_idx[u] = n - 1 - rt;
    }
}
__global__ void __launch_bounds__(kBlock) k_path(const int32_t *a_idx, const int32_t *b_idx,
                                                 const int32_t *length, int32_t cap, int32_t m,
                                                 int32_t n, int32_t *col_in, int32_t *col_out) {
    const int32_t L = imin(imax(*length, 0), cap);
    for (int32_t r = blockIdx.x * kBlock + threadIdx.x; r <= m; r += gridDim.x * kBlock)
        path_row(a_idx, b_idx, L, m, n, r, col_in + r, col_out + r);
}
__global__ void k_copy_len(const int32_t *hdr, int32_t *dst) {
    if (threadIdx.x == 0) *dst = hdr[1];
}

// ------------------------------------------------------------------ launchers

hipError_t launch_clear(int32_t *words, int32_t count, hipStream_t s) {
    const int32_t blocks = imin(1024, (count + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_clear, dim3(imax(blocks, 1)), dim3(kBlock), 0, s, words, count);
    return hipGetLastError();
}

hipError_t launch_nextmatch(const uint8_t *b, int32_t n, int32_t sigma, int32_t *nm, int32_t *err,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_nextmatch, dim3(sigma), dim3(kBlock), 0, s, b, n, sigma, nm, err);
    return hipGetLastError();
}

template <int H0>
static void launch_base_h(dim3 grid, hipStream_t s, const uint8_t *a, int32_t n, int32_t sigma,
                          const int32_t *nm, int32_t *base0, int32_t *last, int32_t nstrips,
                          int32_t hlast, int32_t *err) {
    switch (base_tab_mode<H0>(n, sigma)) {
        case kBaseTab16Mode:
            hipLaunchKernelGGL((k_base<H0, kBaseTab16Mode>), grid, dim3(kBlock), 0, s, a, n, sigma, nm,
                               base0, last, nstrips, hlast, err);
            break;
        default:
            hipLaunchKernelGGL((k_base<H0, kBaseGlobal>), grid, dim3(kBlock), 0, s, a, n, sigma, nm,
                               base0, last, nstrips, hlast, err);
    }
}

hipError_t launch_base(int32_t h0, const uint8_t *a, int32_t n, int32_t sigma, const int32_t *nm,
                       int32_t *base0, int32_t *last, int32_t nstrips, int32_t hlast, int32_t *err,
                       hipStream_t s) {
    const dim3 grid((n + 2 + kBlock - 1) / kBlock, nstrips);
    switch (h0) {
        case 16: launch_base_h<16>(grid, s, a, n, sigma, nm, base0, last, nstrips, hlast, err); break;
        case 32: launch_base_h<32>(grid, s, a, n, sigma, nm, base0, last, nstrips, hlast, err); break;
        case 64: launch_base_h<64>(grid, s, a, n, sigma, nm, base0, last, nstrips, hlast, err); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_base_comb(int32_t h0, const uint8_t *a, const uint8_t *b, int32_t n,
                            int32_t sigma, int32_t *base0, int32_t *last, int32_t nstrips,
                            int32_t hlast, int32_t *comb, int32_t comb_stride, int32_t *rec,
                            int32_t *err, hipStream_t s) {
    if (h0 < 1 || h0 > kCombMaxRows) return hipErrorInvalidValue;
    const int32_t G = comb_segments(n, nstrips, h0);
    // Columns per thread: the row's scan over the threads costs about as much
    // per thread as 16 packed columns, so a work-group of ~512 threads (two
    // waves per SIMD) with up to 32 columns each; labels fit 16 bits up to
    // 32767 columns (the packed form), past that 16 unpacked columns per thread
    // and several tiles.
    const int32_t C = comb_cols(n);
    const int32_t thr = comb_threads(n, C);
    // the wave pipeline: labels in 16 bits, its ring and row symbols in 64 KB of LDS
    const int32_t cp = comb_pipe_cols(n);
    const int32_t waves = (n + kWave * cp - 1) / (kWave * cp);
    const size_t bytes = 4 * (size_t)(waves + 1) * (size_t)h0;
    if (G > 1) {  // tall, few strips: several work-groups per strip (records cleared first)
        const hipError_t e = launch_clear(rec, 2 * nstrips * (G - 1) * h0, s);
        if (e != hipSuccess) return e;
        // 1024 columns per segment (comb_segments)
        constexpr int kSegC = 4, kSegW = 4;  // waves x columns per lane, measured at 16384² (base strips with their rows): 2 x 8 0.797, 4 x 4 0.750, 8 x 2 0.787 ms
        static_assert(kSegC * kSegW * kWave == 1024, "segment width");
        hipLaunchKernelGGL((k_comb_seg<kSegC, kSegW>), dim3((unsigned)(nstrips * G)), dim3(kSegW * kWave),
                           4 * (kSegW + 1) * (size_t)h0, s, a, b, n, sigma, h0, nstrips, hlast, comb,
                           comb_stride, reinterpret_cast<unsigned long long *>(rec), G, err);
    } else if (n >= 1 && n <= kCombPackedMaxN && bytes <= kCombPipeMaxLds) {
        const dim3 blk((unsigned)(kWave * waves));
        if (cp == 4)
            hipLaunchKernelGGL((k_comb_pipe<4>), dim3(nstrips), blk, bytes, s, a, b, n, sigma, h0, nstrips,
                               hlast, comb, comb_stride, err);
        else if (cp == 8)
            hipLaunchKernelGGL((k_comb_pipe<8>), dim3(nstrips), blk, bytes, s, a, b, n, sigma, h0, nstrips,
                               hlast, comb, comb_stride, err);
        else if (cp == 16)
            hipLaunchKernelGGL((k_comb_pipe<16>), dim3(nstrips), blk, bytes, s, a, b, n, sigma, h0, nstrips,
                               hlast, comb, comb_stride, err);
        else
            hipLaunchKernelGGL((k_comb_pipe<32>), dim3(nstrips), blk, bytes, s, a, b, n, sigma, h0, nstrips,
                               hlast, comb, comb_stride, err);
    } else if (n > kCombPackedMaxN)
        hipLaunchKernelGGL((k_comb<kCombMaxThreads, 16, false>), dim3(nstrips), dim3(thr), 0, s, a, b, n,
                           sigma, h0, nstrips, hlast, comb, comb_stride, err);
    else if (C == 4)
        hipLaunchKernelGGL((k_comb<kCombMaxThreads, 4, true>), dim3(nstrips), dim3(thr), 0, s, a, b, n,
                           sigma, h0, nstrips, hlast, comb, comb_stride, err);
    else if (C == 8)
        hipLaunchKernelGGL((k_comb<kCombMaxThreads, 8, true>), dim3(nstrips), dim3(thr), 0, s, a, b, n,
                           sigma, h0, nstrips, hlast, comb, comb_stride, err);
    else if (C == 16)
        hipLaunchKernelGGL((k_comb<kCombMaxThreads, 16, true>), dim3(nstrips), dim3(thr), 0, s, a, b, n,
                           sigma, h0, nstrips, hlast, comb, comb_stride, err);
    else
        hipLaunchKernelGGL((k_comb<kCombMaxThreads, 32, true>), dim3(nstrips), dim3(thr), 0, s, a, b, n,
                           sigma, h0, nstrips, hlast, comb, comb_stride, err);
    // runs short enough that the waves fill the chip, long enough to amortise
    // the scan for the first vertex of each run
    int32_t chunk = 256;
    while (chunk > 32 && (int64_t)nstrips * ((n + 2 + chunk - 1) / chunk) < 16384) chunk /= 2;
    const int32_t nchunks = (n + 2 + chunk - 1) / chunk;
    const int64_t runs = (int64_t)nstrips * nchunks;  // one wave each
    const dim3 grid((uint32_t)((runs + kWaves - 1) / kWaves));
    if (h0 <= kWave)
        hipLaunchKernelGGL((k_dgen<1>), grid, dim3(kBlock), 0, s, comb, comb_stride, n, h0, nstrips,
                           hlast, base0, last, chunk, nchunks);
    else if (h0 <= 2 * kWave)
        hipLaunchKernelGGL((k_dgen<2>), grid, dim3(kBlock), 0, s, comb, comb_stride, n, h0, nstrips,
                           hlast, base0, last, chunk, nchunks);
    else if (h0 <= 4 * kWave)
        hipLaunchKernelGGL((k_dgen<4>), grid, dim3(kBlock), 0, s, comb, comb_stride, n, h0, nstrips,
                           hlast, base0, last, chunk, nchunks);
    else if (h0 <= 8 * kWave)
        hipLaunchKernelGGL((k_dgen<8>), grid, dim3(kBlock), 0, s, comb, comb_stride, n, h0, nstrips,
                           hlast, base0, last, chunk, nchunks);
    else
        hipLaunchKernelGGL((k_dgen<16>), grid, dim3(kBlock), 0, s, comb, comb_stride, n, h0, nstrips,
                           hlast, base0, last, chunk, nchunks);
    return hipGetLastError();
}

// LDS available to one work-group on gfx950
constexpr size_t kMaxGroupLds = 160 * 1024;

// Compute units of the current device (cached per device; 256 if unknown).
static int64_t device_cus() {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] <= 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

// Opt a kernel in to more than 64 KB of dynamic LDS, once per device.
template <int NT, int CPT, typename KT>
static hipError_t opt_in_anchor_lds() {
    static bool opted[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64 || opted[dev]) return hipSuccess;
    e = hipFuncSetAttribute((const void *)k_anchor_lds<NT, CPT, KT>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxGroupLds);
    if (e != hipSuccess) return e;
    opted[dev] = true;
    return hipSuccess;
}

template <int NT, int CPT, typename KT>
static bool try_anchor_lds_t(const CombineArgs &c, int32_t npairs, hipStream_t s, hipError_t &e) {
    const size_t bytes = sizeof(AnchorSmem<NT, CPT>) + sizeof(KT) * ((size_t)c.hc + 1 + (size_t)c.hs);
    if (bytes > kMaxGroupLds) return false;
    e = opt_in_anchor_lds<NT, CPT, KT>();
    if (e == hipSuccess) {
        hipLaunchKernelGGL((k_anchor_lds<NT, CPT, KT>), dim3(c.nanch, npairs), dim3(NT), bytes, s, c);
        e = hipGetLastError();
    }
    return true;
}

// 16-bit rows when every value and k* + 1 fits (half the LDS, so more
// work-groups per CU: the search is bound by dependent depth rounds).
template <int NT, int CPT>
static bool try_anchor_lds(const CombineArgs &c, int32_t npairs, hipStream_t s, hipError_t &e) {
    if (c.n + 1 <= 65535 && c.hc <= 65533) return try_anchor_lds_t<NT, CPT, uint16_t>(c, npairs, s, e);
    return try_anchor_lds_t<NT, CPT, int32_t>(c, npairs, s, e);
}

hipError_t launch_anchor(const CombineArgs &c, int32_t npairs, hipStream_t s) {
    // Few anchors (the top levels) get many threads each, so that a depth's
    // candidates take fewer rounds, but never so many that the work-groups
    // stop fitting on the chip at once (one 1024-thread or about three
    // 512-thread work-groups per CU).  The search is bound by dependent
    // depth rounds, so LDS per work-group sets the speed: below the fewest-
    // anchor case two columns per thread per segment (half the search state)
    // let, with 16-bit rows, two 512-thread work-groups share a CU at the
    // 16384-row top level and 7 to 8 256-thread ones at the 2048-row level
    // (measured at 16384²: anchors 1.81 -> 1.69 ms per build).
    const int64_t blocks = (int64_t)c.nanch * npairs;
    const int64_t cus = device_cus();
    hipError_t e = hipSuccess;
    if (blocks <= cus) {
        if (try_anchor_lds<1024, 4>(c, npairs, s, e) || try_anchor_lds<1024, 2>(c, npairs, s, e))
            return e;
        hipLaunchKernelGGL((k_anchor<1024, 2>), dim3(c.nanch, npairs), dim3(1024), 0, s, c);
        return hipGetLastError();
    }
    // 512 threads up to three work-groups per CU, and for long rows up to
    // five (16384², the 4096-row level's 1026 anchors of 8193 weights: 0.42
    // -> 0.39 ms; short rows lose: 4096², 1032 anchors of 513 weights: 0.029
    // -> 0.038 ms)
    if (blocks <= 3 * cus || (blocks <= 5 * cus && c.hs > 2048)) {
        if (try_anchor_lds<512, 2>(c, npairs, s, e)) return e;
        hipLaunchKernelGGL((k_anchor<512, 4>), dim3(c.nanch, npairs), dim3(512), 0, s, c);
        return hipGetLastError();
    }
    // many short rows: one search per wave (measured: faster up to 512
    // weights, slower at 1024, where the wave's smaller candidate budget per
    // depth needs more depths)
    if (c.hs <= 512) {
        const int32_t per_wave = (int32_t)(((c.hs <= 256 ? sizeof(AnchorSmem<kWave, 4>)
                                                         : sizeof(AnchorSmem<kWave, 8>)) +
                                            4 * ((size_t)c.hc + 1 + (size_t)c.hs) + 7) & ~(size_t)7);
        const dim3 grid((c.nanch + kWaves - 1) / kWaves, npairs);
        const size_t bytes = (size_t)per_wave * kWaves;
        if (c.hs <= 256)
            hipLaunchKernelGGL((k_anchor_wave<4>), grid, dim3(kBlock), bytes, s, c, per_wave);
        else
            hipLaunchKernelGGL((k_anchor_wave<8>), grid, dim3(kBlock), bytes, s, c, per_wave);
        return hipGetLastError();
    }
    if (try_anchor_lds<kBlock, 2>(c, npairs, s, e)) return e;
    hipLaunchKernelGGL((k_anchor<kBlock, 4>), dim3(c.nanch, npairs), dim3(kBlock), 0, s, c);
    return hipGetLastError();
}

// bracket shape of the 16-bit state
using NarrowBracket = BracketCfg16;
template <class C, class Mid, class Wide>
static void launch_bracket_cfg(const CombineArgs &c, dim3 grid, hipStream_t s) {
    // The cooperative pass 2 is compiled only into the kernels for tall
    // strips, so that the others keep their register allocation.  The top
    // combine (one parent strip) of strips of kWideWindowMinH rows and more
    // takes the shape with the wider D_U window: there k* moves furthest
    // across a block (with the narrow window 27% of the top level's live
    // blocks read D_U from global memory, two round trips per batch), which
    // is worth one work-group per CU less.  Below the top the narrow window
    // still holds about 95% of the live blocks and the eighth work-group per
    // CU wins (measured at 16384²: 9% less time in the 2048- and 4096-row
    // combines).
    if (c.hc >= kWideWindowMinH && grid.y == 1)
        hipLaunchKernelGGL((k_bracket<Wide, true>), grid, dim3(kBlock), 0, s, c);
    else if (c.hc >= kCoopPass2MinH)
        hipLaunchKernelGGL((k_bracket<Mid, true>), grid, dim3(kBlock), 0, s, c);
    else
        hipLaunchKernelGGL((k_bracket<C, false>), grid, dim3(kBlock), 0, s, c);
}

hipError_t launch_bracket(const CombineArgs &c0, int32_t npairs, hipStream_t s) {
    const int32_t ntiles = (c0.n + c0.tile - 1) / c0.tile;
    if (ntiles <= 0) return hipSuccess;
    // 16-bit state (64 weights per work-group) when every value fits
    const bool narrow = (c0.n + 1 <= 65535) && (c0.hc <= 65534);
    CombineArgs c = c0;
    c.jchunk = narrow ? NarrowBracket::kJ : BracketCfg32::kJ;
    c.nchunks = imax(1, (c.hs - 1 + c.jchunk - 1) / c.jchunk);  // hs = 2 hc + 1 weights
    const dim3 grid(ntiles * c.nchunks, npairs);
    if (narrow)
        launch_bracket_cfg<NarrowBracket, BracketCfg16Mid, BracketCfg16Wide>(c, grid, s);
    else
        launch_bracket_cfg<BracketCfg32, BracketCfg32, BracketCfg32>(c, grid, s);
    return hipGetLastError();
}

hipError_t launch_length(const int32_t *top, int32_t m, int32_t n, int32_t *hdr, int4 *root,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_length, dim3(1), dim3(kBlock), 0, s, top, m, n, hdr, root);
    return hipGetLastError();
}

hipError_t launch_trace_splits(const TraceSplitArgs &t, hipStream_t s) {
    if (t.top < 1) return hipSuccess;
    if (t.top >= kTraceMaxLev) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_trace_splits, dim3(1), dim3(kSplitThreads), 0, s, t);
    return hipGetLastError();
}

template <typename TT>
static hipError_t launch_trace_leaf_tall(int32_t h0, const uint8_t *a, int32_t n, int32_t sigma,
                                         const int32_t *nm, int32_t nstrips, int32_t hlast,
                                         const int4 *nodes, int32_t *a_idx, int32_t *b_idx,
                                         int32_t wcap, int32_t *err, uint8_t *leaf,
                                         int64_t leaf_stride, hipStream_t s) {
    // the next-match window: no more than the tables hold, so that short
    // strings leave LDS for more leaves per CU
    const int32_t tabcap = leaf_tab_cap(sigma, n, (int32_t)sizeof(TT));
    const size_t bytes = sizeof(TT) * (size_t)tabcap;
    switch (h0) {
        case 128:
            hipLaunchKernelGGL((k_trace_leaf_pipe<1, 2, TT>), dim3(nstrips), dim3(2 * kWave), bytes, s, a, n,
                               sigma, nm, h0, nstrips, hlast, nodes, a_idx, b_idx, wcap, err, tabcap,
                               leaf, leaf_stride);
            break;
        case 256:
            hipLaunchKernelGGL((k_trace_leaf_pipe<1, 4, TT>), dim3(nstrips), dim3(4 * kWave), bytes, s, a, n,
                               sigma, nm, h0, nstrips, hlast, nodes, a_idx, b_idx, wcap, err, tabcap,
                               leaf, leaf_stride);
            break;
        case 512:
            hipLaunchKernelGGL((k_trace_leaf_pipe<2, 4, TT>), dim3(nstrips), dim3(4 * kWave), bytes, s, a, n,
                               sigma, nm, h0, nstrips, hlast, nodes, a_idx, b_idx, wcap, err, tabcap,
                               leaf, leaf_stride);
            break;
        case 1024:
            hipLaunchKernelGGL((k_trace_leaf_pipe<2, 8, TT>), dim3(nstrips), dim3(8 * kWave), bytes, s, a, n,
                               sigma, nm, h0, nstrips, hlast, nodes, a_idx, b_idx, wcap, err, tabcap,
                               leaf, leaf_stride);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_trace_leaf(int32_t h0, const uint8_t *a, int32_t n, int32_t sigma,
                             const int32_t *nm, int32_t nstrips, int32_t hlast, const int4 *nodes,
                             int32_t *a_idx, int32_t *b_idx, int32_t wcap, int32_t *err,
                             uint8_t *leaf, int64_t leaf_stride, hipStream_t s) {
    switch (h0) {
        case 16:
            hipLaunchKernelGGL(k_trace_leaf<16>, dim3(nstrips), dim3(kWave), 0, s, a, n, sigma, nm,
                               nstrips, hlast, nodes, a_idx, b_idx, wcap, err);
            break;
        case 32:
            hipLaunchKernelGGL(k_trace_leaf<32>, dim3(nstrips), dim3(kWave), 0, s, a, n, sigma, nm,
                               nstrips, hlast, nodes, a_idx, b_idx, wcap, err);
            break;
        case 64:
            hipLaunchKernelGGL(k_trace_leaf<64>, dim3(nstrips), dim3(kWave), 0, s, a, n, sigma, nm,
                               nstrips, hlast, nodes, a_idx, b_idx, wcap, err);
            break;
        case 128:
        case 256:
        case 512:
        case 1024:
            if (n + 1 <= 65535)
                return launch_trace_leaf_tall<uint16_t>(h0, a, n, sigma, nm, nstrips, hlast, nodes, a_idx,
                                                        b_idx, wcap, err, leaf, leaf_stride, s);
            return launch_trace_leaf_tall<int32_t>(h0, a, n, sigma, nm, nstrips, hlast, nodes, a_idx,
                                                   b_idx, wcap, err, leaf, leaf_stride, s);
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_copy_len(const int32_t *hdr, int32_t *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_len, dim3(1), dim3(64), 0, s, hdr, dst);
    return hipGetLastError();
}

hipError_t launch_semilocal(const int32_t *top, int32_t m, int32_t n, const int32_t *qi,
                            const int32_t *qk, int32_t count, int32_t *out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int32_t blocks = (count + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_semilocal, dim3(blocks < 4096 ? blocks : 4096), dim3(kBlock), 0, s, top, m,
                       n, qi, qk, count, out);
    return hipGetLastError();
}

hipError_t launch_reverse(const uint8_t *src, int32_t len, uint8_t *dst, hipStream_t s) {
    if (len <= 0) return hipSuccess;
    const int32_t blocks = (len + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_reverse, dim3(blocks < 4096 ? blocks : 4096), dim3(kBlock), 0, s, src, len,
                       dst);
    return hipGetLastError();
}

hipError_t launch_unflip(const int32_t *hdr, int32_t *a_idx, int32_t *b_idx, int32_t capacity,
                         int32_t m, int32_t n, hipStream_t s) {
    const int32_t half = (imin(m, n) + 1) / 2;
    const int32_t blocks = imax(1, (half + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_unflip, dim3(blocks < 4096 ? blocks : 4096), dim3(kBlock), 0, s, hdr, a_idx,
                       b_idx, capacity, m, n);
    return hipGetLastError();
}

hipError_t launch_path(const int32_t *a_idx, const int32_t *b_idx, const int32_t *length,
                       int32_t cap, int32_t m, int32_t n, int32_t *col_in, int32_t *col_out,
                       hipStream_t s) {
    const int32_t blocks = (m + 1 + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_path, dim3(blocks < 4096 ? blocks : 4096), dim3(kBlock), 0, s, a_idx, b_idx,
                       length, cap, m, n, col_in, col_out);
    return hipGetLastError();
}

}  // namespace lcs
