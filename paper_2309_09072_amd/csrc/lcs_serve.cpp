// Continuous-batching LCS server (lcs_server_*): a FIFO of waiting requests on
// the host, a first-fit allocator over the caller's device arena, and `slots`
// HIP streams.  The head of the queue is admitted as soon as a slot is idle and
// its footprint fits the arena; admitted requests run concurrently, each on
// its slot's stream (the same per-level kernels as lcs_dist_build/lcs_trace),
// so new arrivals join requests already on the device.  Completion is observed
// with events in lcs_server_poll, which never blocks.
//
// The admission policy (queue + arena) is shared with lcs_server_simulate,
// which replays it under a virtual clock without a device.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "lcs.h"
#include "lcs_plan.h"

namespace lcs {

bool valid_shape(int32_t base_rows, int32_t tile);
int32_t resolve(int32_t v, int32_t dflt);

// First-fit allocator over [0, cap) in 256-byte units, coalescing on free.
class Arena {
   public:
    explicit Arena(size_t cap = 0) : cap_(cap & ~(size_t)255) {
        if (cap_) free_[0] = cap_;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                if (used_ > peak_) peak_ = used_;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

   private:
    size_t cap_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

static size_t footprint(int32_t m, int32_t n, int32_t sigma, int32_t h0, int32_t tile) {
    Layout L;
    if (!make_layout(m, n, sigma, h0, tile, L)) return 0;
    return (size_t)(align256(m) + align256(n) + L.total);
}

}  // namespace lcs

using namespace lcs;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    int64_t tag;
    std::vector<uint8_t> a, b;
    int32_t sigma;  // the request's own alphabet: its next-match tables and symbol check
    int32_t *ai, *bi;
    double t_submit;
    size_t foot;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    lcs_plan_t plan = nullptr;  // planned per admitted request (host memory only)
    uint8_t *pin_a = nullptr, *pin_b = nullptr;
    int32_t *pin_hdr = nullptr;  // err bits, length, end column
    bool busy = false;
    Request req;
    size_t off = 0;
    double t_admit = 0;
    int32_t launch_status = LCS_OK;
};

}  // namespace

struct lcs_server_s {
    lcs_server_desc d{};
    uint8_t *arena = nullptr;
    Arena alloc;
    std::deque<Request> queue;
    std::vector<Slot> slots;
    std::deque<lcs_result> finished;
    Clock::time_point t0;
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

static void destroy_server(lcs_server_s *S) {
    for (Slot &s : S->slots) {
        if (s.stream) hipStreamSynchronize(s.stream);
        if (s.done) hipEventDestroy(s.done);
        if (s.stream) hipStreamDestroy(s.stream);
        if (s.plan) lcs_plan_destroy(s.plan);
        if (s.pin_a) hipHostFree(s.pin_a);
        if (s.pin_b) hipHostFree(s.pin_b);
        if (s.pin_hdr) hipHostFree(s.pin_hdr);
    }
    delete S;
}

extern "C" int32_t lcs_server_open(const lcs_server_desc *desc, void *arena, size_t arena_bytes,
                                   lcs_server_t *out) {
    if (!desc || !arena || !out) return LCS_E_INVAL;
    *out = nullptr;
    lcs_server_desc d = *desc;
    d.base_rows = resolve(d.base_rows, kDefaultBaseRows);
    d.tile = resolve(d.tile, kDefaultTile);
    if (d.max_len < 1 || d.alphabet < 1 || d.alphabet > 256 || d.slots < 1 || d.slots > 64 ||
        d.max_queue < 1 || d.flags != 0 || !valid_shape(d.base_rows, d.tile))
        return LCS_E_INVAL;
    if (reinterpret_cast<uintptr_t>(arena) & 255) return LCS_E_INVAL;
    lcs_server_s *S = new (std::nothrow) lcs_server_s();
    if (!S) return LCS_E_NOMEM;
    S->d = d;
    S->arena = static_cast<uint8_t *>(arena);
    S->alloc = Arena(arena_bytes);
    S->t0 = Clock::now();
    S->slots.resize(d.slots);
    for (Slot &s : S->slots) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&s.pin_a), (size_t)d.max_len + 1, 0) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&s.pin_b), (size_t)d.max_len + 1, 0) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&s.pin_hdr), 4 * sizeof(int32_t), 0) != hipSuccess) {
            destroy_server(S);
            return LCS_E_HIP;
        }
    }
    *out = S;
    return LCS_OK;
}

extern "C" int32_t lcs_server_footprint(lcs_server_t S, int32_t m, int32_t n, size_t *bytes) {
    if (!S || !bytes || m < 0 || n < 0) return LCS_E_INVAL;
    if (m > S->d.max_len || n > S->d.max_len) return LCS_E_TOO_BIG;
    *bytes = footprint(m, n, S->d.alphabet, S->d.base_rows, S->d.tile);  // largest alphabet
    return *bytes ? LCS_OK : LCS_E_TOO_BIG;
}

extern "C" int32_t lcs_server_submit(lcs_server_t S, int64_t tag, const uint8_t *a, int32_t m,
                                     const uint8_t *b, int32_t n, int32_t alphabet, int32_t *a_idx,
                                     int32_t *b_idx) {
    if (!S || m < 0 || n < 0 || (m > 0 && !a) || (n > 0 && !b)) return LCS_E_INVAL;
    if ((a_idx == nullptr) != (b_idx == nullptr)) return LCS_E_INVAL;
    if (alphabet < 1 || alphabet > S->d.alphabet) return LCS_E_INVAL;
    if (m > S->d.max_len || n > S->d.max_len) return LCS_E_TOO_BIG;
    const size_t foot = footprint(m, n, alphabet, S->d.base_rows, S->d.tile);
    if (!foot) return LCS_E_TOO_BIG;
    if (foot > S->alloc.capacity()) return LCS_E_BUDGET;
    if ((int32_t)S->queue.size() >= S->d.max_queue) return LCS_E_AGAIN;
    Request r;
    r.tag = tag;
    r.a.assign(a, a + m);
    r.b.assign(b, b + n);
    r.sigma = alphabet;
    r.ai = a_idx;
    r.bi = b_idx;
    r.t_submit = S->now();
    r.foot = foot;
    S->queue.push_back(std::move(r));
    return LCS_OK;
}

// Enqueue the device work of request r on slot s (memory at arena offset off).
static int32_t start(lcs_server_s *S, Slot &s) {
    Request &r = s.req;
    const int32_t m = (int32_t)r.a.size(), n = (int32_t)r.b.size();
    uint8_t *base = S->arena + s.off;
    uint8_t *ad = base, *bd = base + align256(m), *ws = base + align256(m) + align256(n);
    const size_t wsb = r.foot - (size_t)(align256(m) + align256(n));
    // a plan of the request's exact sizes and alphabet (host memory only)
    if (s.plan) lcs_plan_destroy(s.plan);
    s.plan = nullptr;
    lcs_plan_desc pd{m, n, r.sigma, S->d.base_rows, S->d.tile, 0};
    size_t need = 0;
    if (lcs_plan(&pd, &s.plan, &need) != LCS_OK) return LCS_E_NOMEM;
    if (need > wsb) return LCS_E_WORKSPACE;
    if (m) memcpy(s.pin_a, r.a.data(), m);
    if (n) memcpy(s.pin_b, r.b.data(), n);
    if (m && hipMemcpyAsync(ad, s.pin_a, m, hipMemcpyHostToDevice, s.stream) != hipSuccess) return LCS_E_HIP;
    if (n && hipMemcpyAsync(bd, s.pin_b, n, hipMemcpyHostToDevice, s.stream) != hipSuccess) return LCS_E_HIP;
    int32_t rc = lcs_dist_build(s.plan, ad, m, bd, n, ws, wsb, s.stream);
    if (rc != LCS_OK) return rc;
    if (r.ai) {
        // the length also lands in the header's word 1, read back below
        rc = lcs_trace_device(s.plan, r.ai, r.bi, m < n ? m : n, reinterpret_cast<int32_t *>(ws) + 3,
                              s.stream);
        if (rc != LCS_OK) return rc;
    }
    if (hipMemcpyAsync(s.pin_hdr, ws, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s.stream) != hipSuccess)
        return LCS_E_HIP;
    return hipEventRecord(s.done, s.stream) == hipSuccess ? LCS_OK : LCS_E_HIP;
}

extern "C" int32_t lcs_server_poll(lcs_server_t S, lcs_result *results, int32_t max_results,
                                   int32_t *count) {
    if (!S || !count || (max_results > 0 && !results)) return LCS_E_INVAL;
    // 1. completions
    for (Slot &s : S->slots) {
        if (!s.busy) continue;
        if (s.launch_status == LCS_OK) {
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) s.launch_status = LCS_E_HIP;
        } else {
            hipStreamSynchronize(s.stream);
        }
        lcs_result res;
        res.tag = s.req.tag;
        res.t_submit = s.req.t_submit;
        res.t_admit = s.t_admit;
        res.t_done = S->now();
        res.status = s.launch_status;
        res.length = 0;
        if (res.status == LCS_OK) {
            if (s.pin_hdr[0] & kErrSymbol)
                res.status = LCS_E_SYMBOL;
            else if (s.pin_hdr[0] != 0)
                res.status = LCS_E_HIP;
            res.length = s.pin_hdr[1];
        }
        S->finished.push_back(res);
        S->alloc.release(s.off, s.req.foot);
        s.busy = false;
        s.req = Request();
    }
    // 2. admissions, in arrival order
    for (Slot &s : S->slots) {
        if (S->queue.empty()) break;
        if (s.busy) continue;
        size_t off = 0;
        if (!S->alloc.alloc(S->queue.front().foot, &off)) break;
        s.req = std::move(S->queue.front());
        S->queue.pop_front();
        s.off = off;
        s.busy = true;
        s.t_admit = S->now();
        s.pin_hdr[0] = s.pin_hdr[1] = s.pin_hdr[2] = 0;
        s.launch_status = start(S, s);
    }
    // 3. results
    int32_t c = 0;
    while (c < max_results && !S->finished.empty()) {
        results[c++] = S->finished.front();
        S->finished.pop_front();
    }
    *count = c;
    return LCS_OK;
}

extern "C" int32_t lcs_server_pending(lcs_server_t S, int32_t *running, int32_t *waiting,
                                      size_t *used, size_t *peak) {
    if (!S) return LCS_E_INVAL;
    int32_t r = 0;
    for (const Slot &s : S->slots) r += s.busy ? 1 : 0;
    if (running) *running = r;
    if (waiting) *waiting = (int32_t)S->queue.size();
    if (used) *used = S->alloc.used();
    if (peak) *peak = S->alloc.peak();
    return LCS_OK;
}

extern "C" int32_t lcs_server_close(lcs_server_t S) {
    if (!S) return LCS_OK;
    destroy_server(S);
    return LCS_OK;
}

// Virtual-clock replay of the admission policy: the same queue order and the
// same first-fit arena, with simulated completions instead of device work.
extern "C" int32_t lcs_server_simulate(size_t arena_bytes, int32_t slots, int32_t count,
                                       const double *arrival, const size_t *foot,
                                       const double *service, double *t_admit, double *t_done,
                                       size_t *peak) {
    if (slots < 1 || count < 0 || (count > 0 && (!arrival || !foot || !service || !t_admit || !t_done)))
        return LCS_E_INVAL;
    for (int32_t i = 0; i < count; ++i) {
        if (foot[i] > (arena_bytes & ~(size_t)255)) return LCS_E_BUDGET;
        if (i > 0 && arrival[i] < arrival[i - 1]) return LCS_E_INVAL;
    }
    Arena A(arena_bytes);
    std::deque<int32_t> q;
    struct Run {
        int32_t id;
        size_t off;
        double end;
    };
    std::vector<Run> run;
    int32_t next = 0, finished = 0;
    double t = 0;
    while (finished < count) {
        // next event: the earliest completion or arrival
        double tn = 1e300;
        for (const Run &r : run) tn = r.end < tn ? r.end : tn;
        if (next < count && arrival[next] < tn) tn = arrival[next];
        t = tn;
        for (size_t k = 0; k < run.size();) {
            if (run[k].end <= t) {
                A.release(run[k].off, foot[run[k].id]);
                ++finished;
                run[k] = run.back();
                run.pop_back();
            } else {
                ++k;
            }
        }
        while (next < count && arrival[next] <= t) q.push_back(next++);
        while (!q.empty() && (int32_t)run.size() < slots) {
            size_t off = 0;
            if (!A.alloc(foot[q.front()], &off)) break;
            const int32_t id = q.front();
            q.pop_front();
            t_admit[id] = t;
            t_done[id] = t + service[id];
            run.push_back(Run{id, off, t_done[id]});
        }
    }
    if (peak) *peak = A.peak();
    return LCS_OK;
}
