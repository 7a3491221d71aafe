// Host-code driver for the sanitizer test (tests/test_host_sanitizers.py):
// runs every host-only path of the C ABI -- planning and workspace sizes, the
// batch schedule builder and its simulation (lcs_batch_selftest), the serving
// admission policy and arena (lcs_server_simulate), argument validation --
// in a library whose host code is built with AddressSanitizer and
// UndefinedBehaviorSanitizer.  No call here reaches a device.  Prints "ok"
// and returns 0 when every status is the expected one.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "lcs.h"

static int failures = 0;
#define EXPECT(cond)                                                      \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static void plans(std::mt19937_64 &g) {
    for (int32_t s = -12; s <= 2; ++s) EXPECT(lcs_status_string(s) != nullptr);
    const int32_t rows[] = {16, 32, 64, 0, 8, 48};
    const int32_t tiles[] = {4, 8, 16, 32, 0, 3, 64};
    for (int rep = 0; rep < 300; ++rep) {
        lcs_plan_desc d{};
        d.max_m = (int32_t)(g() % 5000) - 2;
        d.max_n = (int32_t)(g() % 5000) - 2;
        d.alphabet = (int32_t)(g() % 260);
        d.base_rows = rows[g() % 6];
        d.tile = tiles[g() % 7];
        d.flags = (uint32_t)(g() % 5);
        lcs_plan_t p = nullptr;
        size_t ws = 0;
        const int32_t rc = lcs_plan(&d, &p, &ws);
        const bool ok = d.max_m >= 0 && d.max_n >= 0 && d.alphabet >= 1 && d.alphabet <= 256 &&
                        d.base_rows != 8 && d.base_rows != 48 && d.tile != 3 && d.tile != 64 &&
                        d.flags <= 3;
        EXPECT((rc == LCS_OK) == ok);
        if (rc != LCS_OK) continue;
        for (int k = 0; k < 20; ++k) {
            const int32_t m = d.max_m ? (int32_t)(g() % (d.max_m + 1)) : 0;
            const int32_t n = d.max_n ? (int32_t)(g() % (d.max_n + 1)) : 0;
            size_t w = 0;
            EXPECT(lcs_plan_workspace(p, m, n, &w) == LCS_OK && w <= ws);
        }
        size_t w = 0;
        EXPECT(lcs_plan_workspace(p, d.max_m + 1, 0, &w) == LCS_E_TOO_BIG);
        int32_t len = 0;
        EXPECT(lcs_length(p, &len, nullptr) == LCS_E_STATE);
        EXPECT(lcs_dist_build(p, nullptr, 1, nullptr, 1, nullptr, 0, nullptr) == LCS_E_INVAL);
        EXPECT(lcs_plan_destroy(p) == LCS_OK);
    }
    lcs_plan_desc big{4096, 4096, 4, 64, 32, 0};
    lcs_plan_t p = nullptr;
    size_t ws = 0;
    EXPECT(lcs_plan(&big, &p, &ws) == LCS_OK);
    EXPECT(lcs_dist_build_noalloc(p, nullptr, 4096, nullptr, 4096, nullptr) == LCS_E_WORKSPACE);
    lcs_plan_destroy(p);
    lcs_plan_desc huge{70000, 70000, 4, 64, 32, 0};
    EXPECT(lcs_plan(&huge, &p, &ws) == LCS_E_TOO_BIG);
}

static void schedules(std::mt19937_64 &g) {
    const int32_t rows[] = {16, 32, 64};
    const int32_t tiles[] = {4, 8, 16, 32};
    for (int rep = 0; rep < 60; ++rep) {
        const int32_t count = 1 + (int32_t)(g() % 48);
        lcs_batch_desc d{};
        d.max_pairs = count;
        d.max_len = 1 + (int32_t)(g() % 900);
        d.alphabet = 1 + (int32_t)(g() % 20);
        d.base_rows = rows[g() % 3];
        d.tile = tiles[g() % 4];
        d.slots = (int32_t)(g() % (count + 1));
        std::vector<lcs_pair_desc> pairs(count);
        int64_t off = 0;
        for (auto &pd : pairs) {
            pd.m = (g() % 7 == 0) ? 0 : (int32_t)(g() % (d.max_len + 1));
            pd.n = (g() % 7 == 0) ? 0 : (int32_t)(g() % (d.max_len + 1));
            pd.a_off = off;
            pd.b_off = off + pd.m;
            off += pd.m + pd.n;
        }
        EXPECT(lcs_batch_selftest(&d, pairs.data(), count) == LCS_OK);
        pairs[0].m = d.max_len + 1;
        EXPECT(lcs_batch_selftest(&d, pairs.data(), count) == LCS_E_TOO_BIG);
    }
}

static void serving(std::mt19937_64 &g) {
    for (int rep = 0; rep < 40; ++rep) {
        const int32_t count = (int32_t)(g() % 300);
        const size_t arena = ((size_t)1 << 20) * (1 + g() % 64);
        const int32_t slots = 1 + (int32_t)(g() % 16);
        std::vector<double> arr(count), svc(count), ta(count), td(count);
        std::vector<size_t> foot(count);
        double t = 0;
        for (int32_t i = 0; i < count; ++i) {
            t += (double)(g() % 1000) * 1e-5;
            arr[i] = t;
            svc[i] = (double)(1 + g() % 1000) * 1e-5;
            foot[i] = 256 + (size_t)(g() % (arena / 2));
        }
        size_t peak = 0;
        EXPECT(lcs_server_simulate(arena, slots, count, arr.data(), foot.data(), svc.data(),
                                   ta.data(), td.data(), &peak) == LCS_OK);
        EXPECT(peak <= arena);
        for (int32_t i = 0; i < count; ++i) EXPECT(ta[i] >= arr[i] && td[i] >= ta[i] + svc[i] - 1e-12);
        if (count > 0) {
            foot[0] = arena + 1024;
            EXPECT(lcs_server_simulate(arena, slots, count, arr.data(), foot.data(), svc.data(),
                                       ta.data(), td.data(), &peak) == LCS_E_BUDGET);
        }
    }
}

int main() {
    std::mt19937_64 g(2309090720ull);
    plans(g);
    schedules(g);
    serving(g);
    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
