// server_host_check.cpp -- host-only checks of the frame server's bookkeeping
// (built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py; no GPU is used).
//
// The server source is included whole so that its internal classes can be
// exercised directly:
//   * the first-fit device-arena allocator: random allocations and releases
//     checked against a byte-level occupancy map (no overlap, every range inside
//     the arena, the largest free range and the peak as stated, full coalescing
//     once everything is released);
//   * the re-basing of a batch's inlier mask to one frame: every frame offset
//     and length against a bit-by-bit reference;
//   * the server entry points' argument checks (NULL server, bad sizes).
// The estimate entry points the server calls are replaced by stubs that must
// never run here.
#include "../paper_2012_12618_amd/csrc/rv_server.cpp"

#include <stdarg.h>

#include <stdio.h>
#include <stdlib.h>

#include <random>

namespace rv_internal {
thread_local char g_error[512] = "";
int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
    return code;
}
}  // namespace rv_internal

extern "C" {
size_t rv_batch_workspace_bytes(int64_t, int64_t n_clusters, int64_t n_points, int32_t) {
    return (size_t)(28 * n_points + 40 * n_clusters + 2560);
}
void rv_tuning_default(rv_tuning_t *t) { memset(t, 0, sizeof *t); }
int rv_estimate_velocity_batch(const float *, const float *, const int32_t *, const int32_t *,
                               const uint64_t *, int64_t, int64_t, int64_t, int32_t, float, float *,
                               float *, float *, int32_t *, uint8_t *, int32_t *, uint32_t *,
                               int32_t *, int32_t *, const rv_tuning_t *, void *, size_t, void *) {
    fprintf(stderr, "the estimate must not run in the host check\n");
    abort();
}
size_t rv_workspace_bytes(int64_t n_clusters, int64_t n_points, int32_t) {
    return (size_t)(20 * n_points + 12 * n_clusters + 1536);
}
int rv_estimate_velocity(const float *, const float *, const int32_t *, int64_t, int64_t, int32_t,
                         float, uint64_t, float *, float *, float *, int32_t *, uint8_t *,
                         int32_t *, uint32_t *, int32_t *, int32_t *, void *, size_t, void *) {
    fprintf(stderr, "the estimate must not run in the host check\n");
    abort();
}
}

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static void check_arena() {
    const size_t unit = kAlign, size = 4096 * unit;
    Arena a;
    a.reset(size);
    std::vector<int> owner(size / unit, -1);
    std::vector<std::pair<size_t, size_t>> live;  // (offset, bytes)
    std::mt19937_64 rng(7);
    size_t used = 0, peak = 0;
    for (int step = 0; step < 20000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t n = 1 + rng() % (64 * unit);
            // the largest free range, computed from the occupancy map
            size_t best = 0, run = 0;
            for (int o : owner) {
                run = o < 0 ? run + unit : 0;
                best = std::max(best, run);
            }
            CHECK(a.largest_free() == best);
            const size_t off = a.alloc(n);
            const size_t len = align_up(n);
            if (off == kNone) {
                CHECK(len > best);
                continue;
            }
            CHECK(off % unit == 0 && off + len <= size);
            for (size_t u = off / unit; u < (off + len) / unit; ++u) {
                CHECK(owner[u] < 0);
                owner[u] = step;
            }
            live.emplace_back(off, n);
            used += len;
            peak = std::max(peak, used);
        } else {
            const size_t i = rng() % live.size();
            const auto r = live[i];
            live[i] = live.back();
            live.pop_back();
            a.release(r.first, r.second);
            for (size_t u = r.first / unit; u < (r.first + align_up(r.second)) / unit; ++u) owner[u] = -1;
            used -= align_up(r.second);
        }
    }
    CHECK(a.peak() == peak);
    for (const auto &r : live) a.release(r.first, r.second);
    CHECK(a.largest_free() == size);
    CHECK(a.alloc(size) == 0);
}

static void check_extract_bits() {
    std::mt19937 rng(11);
    const int64_t n_batch = 1000;
    std::vector<uint32_t> w((n_batch + 31) / 32);
    for (auto &x : w) x = rng();
    if (n_batch % 32) w.back() &= (1u << (n_batch % 32)) - 1u;  // as the kernels leave it
    for (int64_t p0 = 0; p0 <= n_batch; ++p0) {
        for (int64_t n : {(int64_t)0, (int64_t)1, (int64_t)31, (int64_t)32, (int64_t)33,
                          (int64_t)64, (int64_t)97, n_batch - p0}) {
            if (p0 + n > n_batch || n < 0) continue;
            std::vector<uint32_t> out((n + 31) / 32 + 1, 0xDEADBEEFu);
            extract_bits(w.data(), w.size(), p0, n, out.data());
            for (int64_t q = 0; q < ((n + 31) / 32) * 32; ++q) {
                const int64_t p = p0 + q;
                const uint32_t want = q < n ? (w[p >> 5] >> (p & 31)) & 1u : 0u;
                CHECK(((out[q >> 5] >> (q & 31)) & 1u) == want);
            }
            CHECK(out[(n + 31) / 32] == 0xDEADBEEFu);  // nothing written past the frame
        }
    }
}

static void check_entry_points() {
    rv_server_config_t cfg;
    rv_server_config_default(&cfg);
    CHECK(cfg.keep_inlier_bits == 0 && cfg.n_hyp == 512);
    CHECK(rv_server_frame_bytes(&cfg, 700, 146000) > 0);
    cfg.keep_inlier_bits = 1;
    CHECK(rv_server_frame_bytes(&cfg, 700, 146000) >= 146000 / 8);
    CHECK(rv_server_frame_bytes(nullptr, 1, 1) == 0);
    uint64_t t = 0;
    CHECK(rv_server_submit(nullptr, nullptr, nullptr, nullptr, 0, 0, 1, &t) == RV_ERR_INVALID_ARG);
    CHECK(rv_server_wait(nullptr, 1, 0) == RV_ERR_INVALID_ARG);
    CHECK(rv_server_result(nullptr, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr) == RV_ERR_INVALID_ARG);
    rv_server_stats_t st;
    CHECK(rv_server_stats(nullptr, &st) == RV_ERR_INVALID_ARG);
    rv_server_t *s = nullptr;
    cfg.n_streams = 9;
    CHECK(rv_server_create(&cfg, &s) == RV_ERR_INVALID_ARG && s == nullptr);
    rv_server_destroy(nullptr);
}

int main() {
    check_arena();
    check_extract_bits();
    check_entry_points();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("server host checks passed\n");
    return 0;
}
