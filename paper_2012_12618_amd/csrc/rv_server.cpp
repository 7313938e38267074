// rv_server.cpp -- the frame server declared in include/rv.h: a request queue
// with admission by a device-memory budget, continuous batching over launch
// slots, and pinned host staging.  Host code only; every estimate runs through
// rv_estimate_velocity_batch.

#include <hip/hip_runtime_api.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <system_error>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rv.h"
#include "rv_internal.h"

using rv_internal::fail;
using rv_internal::g_error;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kNone = ~(size_t)0;
constexpr int kMaxStreams = 8;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator of kAlign-multiple ranges of [0, size); freed ranges are
// merged with their free neighbours.
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        size_ = size;
        used_ = peak_ = 0;
        if (size > 0) free_[0] = size;
    }
    size_t alloc(size_t n) {
        n = align_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return kNone;
    }
    void release(size_t off, size_t n) {
        n = align_up(n);
        used_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &r : free_) m = std::max(m, r.second);
        return m;
    }
    size_t size() const { return size_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

// Pinned host buffers reused by power-of-two capacity class.
class PinnedPool {
  public:
    void *get(size_t n, size_t *cap) {
        size_t c = 4096;
        while (c < n) c <<= 1;
        {
            std::lock_guard<std::mutex> lock(mu_);
            auto it = free_.find(c);
            if (it != free_.end()) {
                void *p = it->second;
                free_.erase(it);
                *cap = c;
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> lock(mu_);
        held_ += c;
        *cap = c;
        return p;
    }
    void put(void *p, size_t cap) {
        if (p == nullptr) return;
        std::lock_guard<std::mutex> lock(mu_);
        free_.emplace(cap, p);
    }
    size_t held() {
        std::lock_guard<std::mutex> lock(mu_);
        return held_;
    }
    // Frees the buffers returned so far (all of them, once nothing is in use).
    void clear() {
        std::lock_guard<std::mutex> lock(mu_);
        for (auto &b : free_) {
            (void)hipHostFree(b.second);
            held_ -= b.first;
        }
        free_.clear();
    }

  private:
    std::mutex mu_;
    std::multimap<size_t, void *> free_;
    size_t held_ = 0;
};

// Arena layout of one batch.  The first meta_bytes (cluster offsets, frame
// offsets, seeds) are staged in pinned memory with the same layout and copied
// in one transfer; the outputs form one block copied back in one transfer.
struct BatchPlan {
    size_t offsets, frame_off, seeds, meta_bytes;
    size_t theta, vd, ws, ws_bytes;
    size_t out, out_bytes;                      // outputs block, and within it:
    size_t o_vx, o_vy, o_heading, o_inl, o_near, o_best, o_bits, o_status;
    size_t bits_words;                          // 0 unless the inlier mask is kept
    size_t total;
};

BatchPlan plan_batch(int64_t F, int64_t K, int64_t N, int32_t H, bool bits) {
    BatchPlan p;
    size_t at = 0;
    p.offsets = at; at = align_up(at + (size_t)(K + 1) * 4);
    p.frame_off = at; at = align_up(at + (size_t)(F + 1) * 4);
    p.seeds = at; at = align_up(at + (size_t)F * 8);
    p.meta_bytes = at;
    p.theta = at; at = align_up(at + (size_t)N * 4);
    p.vd = at; at = align_up(at + (size_t)N * 4);
    p.ws = at;
    p.ws_bytes = rv_batch_workspace_bytes(F, K, N, H);
    at = align_up(at + p.ws_bytes);
    p.out = at;
    size_t o = 0;
    p.o_vx = o; o = align_up(o + (size_t)K * 4);
    p.o_vy = o; o = align_up(o + (size_t)K * 4);
    p.o_heading = o; o = align_up(o + (size_t)K * 4);
    p.o_inl = o; o = align_up(o + (size_t)K * 4);
    p.o_near = o; o = align_up(o + (size_t)K * 4);
    p.o_best = o; o = align_up(o + (size_t)K * 4);
    p.bits_words = bits ? ((size_t)N + 31) / 32 : 0;
    p.o_bits = o; o = align_up(o + p.bits_words * 4);
    p.o_status = o; o = align_up(o + (size_t)K);
    p.out_bytes = o;
    p.total = at + o;
    return p;
}

enum FrameState { kWaiting = 0, kLaunched = 1, kDone = 2, kFailed = 3 };

struct Frame {
    int64_t K = 0, N = 0;
    uint64_t seed = 0;
    void *in = nullptr;  // the server's pinned copy: theta[N] | vd[N] | offsets[K + 1];
    size_t in_cap = 0;   // null when the frame is read from the caller's pinned arrays
    const float *src_theta = nullptr, *src_vd = nullptr;  // where the frame is read from
    const int32_t *src_off = nullptr;
    int64_t c0 = 0, p0 = 0;  // first cluster and point in its batch
    int state = kWaiting;
    rv_frame_times_t times{};
    std::vector<float> vx, vy, heading;
    std::vector<int32_t> n_inliers, n_near, best;
    std::vector<uint8_t> status;
    std::vector<uint32_t> bits;  // its inlier mask, when the server keeps masks

    const float *theta() const { return src_theta; }
    const float *vd() const { return src_vd; }
    const int32_t *offsets() const { return src_off; }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *meta = nullptr, *result = nullptr;  // pinned staging
    size_t meta_cap = 0, result_cap = 0;
    bool busy = false;
    size_t arena_off = 0;
    BatchPlan plan{};
    int64_t K = 0, N = 0;
    std::vector<Frame *> frames;
    int rc = RV_OK;
};

}  // namespace

struct rv_server {
    rv_server_config_t cfg{};
    int device = 0;
    char *arena_base = nullptr;
    Arena arena;
    PinnedPool pool;
    Slot slots[kMaxStreams];
    std::deque<Frame *> waiting;
    std::deque<int> inflight;  // slot indices in launch order
    std::unordered_map<uint64_t, Frame *> frames;
    uint64_t next_ticket = 1;
    int64_t reserved = 0;  // submits between their queue check and their push
    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_ready;
    bool stopping = false, sched_done = false;
    std::thread scheduler, completer;
    std::chrono::steady_clock::time_point t0;
    rv_server_stats_t st{};

    int64_t now() const {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(
                   std::chrono::steady_clock::now() - t0)
            .count();
    }
};

namespace {

int free_slot(const rv_server *s) {
    for (int i = 0; i < s->cfg.n_streams; ++i)
        if (!s->slots[i].busy) return i;
    return -1;
}

BatchPlan plan_for(const rv_server *s, int64_t F, int64_t K, int64_t N) {
    return plan_batch(F, K, N, s->cfg.n_hyp, s->cfg.keep_inlier_bits != 0);
}

bool head_fits(const rv_server *s) {
    const Frame *f = s->waiting.front();
    return plan_for(s, 1, f->K, f->N).total <= s->arena.largest_free();
}

// Bits [p0, p0 + n) of a batch's inlier mask (n_words words), re-based to start
// at bit 0 of out[ceil(n / 32)]; bits of the next frame in the last word are
// cleared.
void extract_bits(const uint32_t *w, size_t n_words, int64_t p0, int64_t n, uint32_t *out) {
    const int64_t nw = (n + 31) / 32;
    const int sh = (int)(p0 & 31);
    const size_t base = (size_t)(p0 >> 5);
    for (int64_t i = 0; i < nw; ++i) {
        const size_t a = base + (size_t)i;
        const uint64_t lo = a < n_words ? w[a] : 0u;
        const uint64_t hi = a + 1 < n_words ? w[a + 1] : 0u;
        out[i] = (uint32_t)(((hi << 32) | lo) >> sh);
    }
    if ((n & 31) != 0) out[nw - 1] &= (1u << (n & 31)) - 1u;
}

bool ensure_pinned(PinnedPool &pool, void **p, size_t *cap, size_t need) {
    if (*p != nullptr && *cap >= need) return true;
    pool.put(*p, *cap);
    *p = pool.get(need, cap);
    return *p != nullptr;
}

// Host staging and the enqueue of one batch on its slot's stream (no lock held).
int launch_slot(rv_server *s, Slot &sl) {
    const BatchPlan &p = sl.plan;
    const int64_t F = (int64_t)sl.frames.size();
    char *meta = (char *)sl.meta;
    int32_t *off = (int32_t *)(meta + p.offsets);
    int32_t *fo = (int32_t *)(meta + p.frame_off);
    uint64_t *seeds = (uint64_t *)(meta + p.seeds);
    int64_t cb = 0, pb = 0;
    for (int64_t i = 0; i < F; ++i) {
        Frame *f = sl.frames[i];
        f->c0 = cb;
        f->p0 = pb;
        fo[i] = (int32_t)cb;
        seeds[i] = f->seed;
        const int32_t *lo = f->offsets();
        for (int64_t k = 0; k < f->K; ++k) off[cb + k] = (int32_t)(pb + lo[k]);
        cb += f->K;
        pb += f->N;
    }
    off[cb] = (int32_t)pb;
    fo[F] = (int32_t)cb;

    char *d = s->arena_base + sl.arena_off;
    hipStream_t st = sl.stream;
    hipError_t e = hipMemcpyAsync(d, meta, p.meta_bytes, hipMemcpyHostToDevice, st);
    for (int64_t i = 0; i < F && e == hipSuccess; ++i) {
        const Frame *f = sl.frames[i];
        if (f->N == 0) continue;
        e = hipMemcpyAsync(d + p.theta + 4 * f->p0, f->theta(), 4 * (size_t)f->N,
                           hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d + p.vd + 4 * f->p0, f->vd(), 4 * (size_t)f->N,
                               hipMemcpyHostToDevice, st);
    }
    if (e != hipSuccess) return fail(RV_ERR_HIP, "hipMemcpyAsync failed: %s", hipGetErrorString(e));
    char *o = d + p.out;
    int rc;
    // A batch of one frame in float32 takes the single-frame launch sequence
    // (three kernels, or one for a small frame, against the batched form's
    // six): the same results bit for bit, fewer launches on the frame's path.
    // Its workspace fits in the batched one (fewer bytes per cluster).
    if (F == 1 && s->cfg.tuning.fp16_min_points == 0 &&
        rv_workspace_bytes(sl.K, sl.N, s->cfg.n_hyp) <= p.ws_bytes)
        rc = rv_estimate_velocity(
            (const float *)(d + p.theta), (const float *)(d + p.vd),
            (const int32_t *)(d + p.offsets), sl.K, sl.N, s->cfg.n_hyp, s->cfg.tau,
            sl.frames[0]->seed, (float *)(o + p.o_vx), (float *)(o + p.o_vy),
            (float *)(o + p.o_heading), (int32_t *)(o + p.o_inl), (uint8_t *)(o + p.o_status),
            (int32_t *)(o + p.o_near), p.bits_words > 0 ? (uint32_t *)(o + p.o_bits) : nullptr,
            nullptr, (int32_t *)(o + p.o_best), d + p.ws, p.ws_bytes, st);
    else
        rc = rv_estimate_velocity_batch(
            (const float *)(d + p.theta), (const float *)(d + p.vd),
            (const int32_t *)(d + p.offsets), (const int32_t *)(d + p.frame_off),
            (const uint64_t *)(d + p.seeds), F, sl.K, sl.N, s->cfg.n_hyp, s->cfg.tau,
            (float *)(o + p.o_vx), (float *)(o + p.o_vy), (float *)(o + p.o_heading),
            (int32_t *)(o + p.o_inl), (uint8_t *)(o + p.o_status), (int32_t *)(o + p.o_near),
            p.bits_words > 0 ? (uint32_t *)(o + p.o_bits) : nullptr, nullptr,
            (int32_t *)(o + p.o_best), &s->cfg.tuning, d + p.ws, p.ws_bytes, st);
    if (rc != RV_OK) return rc;
    if (sl.K > 0) {
        e = hipMemcpyAsync(sl.result, o, p.out_bytes, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess)
            return fail(RV_ERR_HIP, "hipMemcpyAsync failed: %s", hipGetErrorString(e));
    }
    e = hipEventRecord(sl.done, st);
    if (e != hipSuccess) return fail(RV_ERR_HIP, "hipEventRecord failed: %s", hipGetErrorString(e));
    return RV_OK;
}

void scheduler_loop(rv_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_sched.wait(lk, [&] {
            if (s->waiting.empty()) return s->stopping;
            return free_slot(s) >= 0 && head_fits(s);
        });
        if (s->waiting.empty()) break;  // stopping, and nothing left to launch
        const int si = free_slot(s);
        Slot &sl = s->slots[si];
        // Arrival order: the longest prefix of waiting frames that fits the
        // arena's largest free range and the frame limit.
        const size_t room = s->arena.largest_free();
        int64_t F = 0, K = 0, N = 0;
        for (const Frame *f : s->waiting) {
            if (F >= s->cfg.max_batch_frames) break;
            const int64_t K2 = K + f->K, N2 = N + f->N;
            if (K2 > INT32_MAX || N2 > INT32_MAX) break;
            if (plan_for(s, F + 1, K2, N2).total > room) break;
            ++F;
            K = K2;
            N = N2;
        }
        sl.plan = plan_for(s, F, K, N);
        sl.arena_off = s->arena.alloc(sl.plan.total);  // fits: total <= room
        sl.K = K;
        sl.N = N;
        sl.busy = true;
        sl.frames.assign(s->waiting.begin(), s->waiting.begin() + F);
        s->waiting.erase(s->waiting.begin(), s->waiting.begin() + F);
        lk.unlock();
        int rc = RV_OK;
        if (!ensure_pinned(s->pool, &sl.meta, &sl.meta_cap, sl.plan.meta_bytes) ||
            !ensure_pinned(s->pool, &sl.result, &sl.result_cap, sl.plan.out_bytes))
            rc = fail(RV_ERR_HIP, "pinned host allocation failed");
        if (rc == RV_OK) rc = launch_slot(s, sl);
        const int64_t t = s->now();
        lk.lock();
        sl.rc = rc;
        for (Frame *f : sl.frames) {
            f->state = kLaunched;
            f->times.launched_ns = t;
            f->times.batch_frames = (int32_t)F;
            f->times.slot = si;
        }
        s->inflight.push_back(si);
        s->st.batches += 1;
        s->st.max_batch_frames_seen = std::max<int64_t>(s->st.max_batch_frames_seen, F);
        s->cv_done.notify_one();
    }
}

void completer_loop(rv_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_done.wait(lk, [&] { return !s->inflight.empty() || s->sched_done; });
        if (s->inflight.empty()) break;  // the scheduler has finished and nothing is in flight
        const int si = s->inflight.front();
        Slot &sl = s->slots[si];
        lk.unlock();
        bool ok = sl.rc == RV_OK && hipEventSynchronize(sl.done) == hipSuccess;
        // After a failed enqueue, wait for whatever did reach the stream before
        // the frames' pinned inputs go back to the pool.
        if (!ok) (void)hipStreamSynchronize(sl.stream);
        const int64_t t = s->now();
        if (ok) {
            const char *r = (const char *)sl.result;
            const BatchPlan &p = sl.plan;
            for (Frame *f : sl.frames) {
                const size_t K = (size_t)f->K, c0 = (size_t)f->c0;
                f->vx.assign((const float *)(r + p.o_vx) + c0, (const float *)(r + p.o_vx) + c0 + K);
                f->vy.assign((const float *)(r + p.o_vy) + c0, (const float *)(r + p.o_vy) + c0 + K);
                f->heading.assign((const float *)(r + p.o_heading) + c0,
                                  (const float *)(r + p.o_heading) + c0 + K);
                f->n_inliers.assign((const int32_t *)(r + p.o_inl) + c0,
                                    (const int32_t *)(r + p.o_inl) + c0 + K);
                f->n_near.assign((const int32_t *)(r + p.o_near) + c0,
                                 (const int32_t *)(r + p.o_near) + c0 + K);
                f->status.assign((const uint8_t *)(r + p.o_status) + c0,
                                 (const uint8_t *)(r + p.o_status) + c0 + K);
                f->best.assign((const int32_t *)(r + p.o_best) + c0,
                               (const int32_t *)(r + p.o_best) + c0 + K);
                if (p.bits_words > 0) {
                    f->bits.resize(((size_t)f->N + 31) / 32);
                    extract_bits((const uint32_t *)(r + p.o_bits), p.bits_words, f->p0, f->N,
                                 f->bits.data());
                }
            }
        }
        lk.lock();
        for (Frame *f : sl.frames) {
            f->state = ok ? kDone : kFailed;
            f->times.done_ns = t;
            s->pool.put(f->in, f->in_cap);
            f->in = nullptr;
        }
        s->st.frames_done += (int64_t)sl.frames.size();
        s->arena.release(sl.arena_off, sl.plan.total);
        sl.frames.clear();
        sl.busy = false;
        s->inflight.pop_front();
        s->cv_ready.notify_all();
        s->cv_sched.notify_one();
    }
}

int check_config(const rv_server_config_t *c) {
    if (c == nullptr) return fail(RV_ERR_INVALID_ARG, "config is NULL");
    if (c->n_hyp < 1 || c->n_hyp > RV_MAX_HYP)
        return fail(RV_ERR_INVALID_ARG, "n_hyp must be in [1, %d]", RV_MAX_HYP);
    if (!(c->tau > 0.0f) || !(c->tau < __builtin_inff()))
        return fail(RV_ERR_INVALID_ARG, "tau must be finite and > 0");
    if (c->hbm_budget_bytes < ((size_t)1 << 20))
        return fail(RV_ERR_INVALID_ARG, "hbm_budget_bytes must be >= 1 MiB");
    if (c->max_batch_frames < 1) return fail(RV_ERR_INVALID_ARG, "max_batch_frames must be >= 1");
    if (c->n_streams < 1 || c->n_streams > kMaxStreams)
        return fail(RV_ERR_INVALID_ARG, "n_streams must be in [1, %d]", kMaxStreams);
    if (c->max_waiting_frames < 1)
        return fail(RV_ERR_INVALID_ARG, "max_waiting_frames must be >= 1");
    for (int b = 0; b < RV_TUNE_BUCKETS; ++b)
        if (c->tuning.rows_max[b] < 1 || c->tuning.rows_max[b] > 16)
            return fail(RV_ERR_INVALID_ARG, "tuning.rows_max must be in [1, 16]");
    if (c->tuning.blocks_per_cu < 0 || c->tuning.blocks_per_cu > 64)
        return fail(RV_ERR_INVALID_ARG, "tuning.blocks_per_cu must be in [0, 64]");
    if (c->tuning.fp16_min_points < 0)
        return fail(RV_ERR_INVALID_ARG, "tuning.fp16_min_points must be >= 0");
    if (c->tuning.lanes_max_points < 0 || c->tuning.lanes_max_points > 256)
        return fail(RV_ERR_INVALID_ARG, "tuning.lanes_max_points must be in [0, 256]");
    return RV_OK;
}

void release_all(rv_server *s) {
    for (auto &kv : s->frames) {
        s->pool.put(kv.second->in, kv.second->in_cap);
        delete kv.second;
    }
    s->frames.clear();
    for (Slot &sl : s->slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        s->pool.put(sl.meta, sl.meta_cap);
        s->pool.put(sl.result, sl.result_cap);
        sl = Slot();
    }
    s->pool.clear();
    if (s->arena_base) (void)hipFree(s->arena_base);
    s->arena_base = nullptr;
}

}  // namespace

namespace {

// Queues a frame read from the server's pinned copy (copy = true) or straight
// from the caller's arrays.  The caller's arrays are not checked for being
// pinned: a pointer query per array costs the runtime's lock, which the
// scheduler and completion threads also take; pageable arrays are still copied
// correctly, only synchronously.
int submit_frame(rv_server *s, const float *theta, const float *vd,
                 const int32_t *cluster_offsets, int64_t n_clusters, int64_t n_points,
                 uint64_t seed, uint64_t *ticket, bool copy) {
    g_error[0] = '\0';
    if (s == nullptr || ticket == nullptr) return fail(RV_ERR_INVALID_ARG, "server or ticket is NULL");
    if (n_clusters < 0 || n_clusters > INT32_MAX || n_points < 0 || n_points > INT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "n_clusters and n_points must be in [0, 2^31 - 1]");
    if (cluster_offsets == nullptr || (n_points > 0 && (theta == nullptr || vd == nullptr)))
        return fail(RV_ERR_INVALID_ARG, "theta, vd or cluster_offsets is NULL");
    if (cluster_offsets[0] != 0 || cluster_offsets[n_clusters] != n_points)
        return fail(RV_ERR_INVALID_ARG, "cluster_offsets must start at 0 and end at n_points");
    for (int64_t k = 0; k < n_clusters; ++k)
        if (cluster_offsets[k + 1] < cluster_offsets[k])
            return fail(RV_ERR_INVALID_ARG, "cluster_offsets must be non-decreasing");
    const size_t need = plan_for(s, 1, n_clusters, n_points).total;
    if (need > s->cfg.hbm_budget_bytes)
        return fail(RV_ERR_INVALID_ARG, "frame needs %zu bytes of device memory, budget is %zu",
                    need, s->cfg.hbm_budget_bytes);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int64_t)s->waiting.size() + s->reserved >= s->cfg.max_waiting_frames) {
            s->st.busy_rejections += 1;
            return fail(RV_ERR_BUSY, "%d frames are waiting", s->cfg.max_waiting_frames);
        }
        s->reserved += 1;
    }
    Frame *f = new Frame;
    f->K = n_clusters;
    f->N = n_points;
    f->seed = seed;
    if (copy) {
        const size_t bytes = 8 * (size_t)n_points + 4 * (size_t)(n_clusters + 1);
        f->in = s->pool.get(bytes, &f->in_cap);
        if (f->in == nullptr) {
            delete f;
            std::lock_guard<std::mutex> lk(s->mu);
            s->reserved -= 1;
            return fail(RV_ERR_HIP, "pinned host allocation of %zu bytes failed", bytes);
        }
        float *in = (float *)f->in;
        if (n_points > 0) {
            memcpy(in, theta, 4 * (size_t)n_points);
            memcpy(in + n_points, vd, 4 * (size_t)n_points);
        }
        memcpy(in + 2 * n_points, cluster_offsets, 4 * (size_t)(n_clusters + 1));
        f->src_theta = in;
        f->src_vd = in + n_points;
        f->src_off = (const int32_t *)(in + 2 * n_points);
    } else {
        f->src_theta = theta;
        f->src_vd = vd;
        f->src_off = cluster_offsets;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->reserved -= 1;
        f->times.submitted_ns = s->now();
        f->times.slot = -1;
        *ticket = s->next_ticket++;
        s->frames[*ticket] = f;
        s->waiting.push_back(f);
        s->st.frames_submitted += 1;
    }
    s->cv_sched.notify_one();
    return RV_OK;
}

}  // namespace

extern "C" {

void rv_server_config_default(rv_server_config_t *cfg) {
    if (cfg == nullptr) return;
    memset(cfg, 0, sizeof *cfg);
    cfg->n_hyp = 512;
    cfg->tau = 0.15f;
    cfg->hbm_budget_bytes = (size_t)16 << 30;
    cfg->max_batch_frames = 64;
    cfg->n_streams = 2;
    cfg->max_waiting_frames = 1024;
    rv_tuning_default(&cfg->tuning);
}

size_t rv_server_frame_bytes(const rv_server_config_t *cfg, int64_t n_clusters, int64_t n_points) {
    if (cfg == nullptr || n_clusters < 0 || n_points < 0 || n_clusters > INT32_MAX ||
        n_points > INT32_MAX || cfg->n_hyp < 1)
        return 0;
    return plan_batch(1, n_clusters, n_points, cfg->n_hyp, cfg->keep_inlier_bits != 0).total;
}

int rv_server_create(const rv_server_config_t *cfg, rv_server_t **server) {
    g_error[0] = '\0';
    if (server == nullptr) return fail(RV_ERR_INVALID_ARG, "server is NULL");
    *server = nullptr;
    if (int rc = check_config(cfg)) return rc;
    rv_server *s = new rv_server;
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    int rc = RV_OK;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc((void **)&s->arena_base, cfg->hbm_budget_bytes);
    if (e != hipSuccess) {
        rc = fail(RV_ERR_HIP, "device arena of %zu bytes: %s", cfg->hbm_budget_bytes,
                  hipGetErrorString(e));
        s->arena_base = nullptr;
    }
    s->arena.reset(cfg->hbm_budget_bytes);
    for (int i = 0; i < cfg->n_streams && rc == RV_OK; ++i) {
        if (hipStreamCreateWithFlags(&s->slots[i].stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s->slots[i].done, hipEventDisableTiming) != hipSuccess)
            rc = fail(RV_ERR_HIP, "stream or event creation failed");
    }
    if (rc == RV_OK) {
        try {
            s->scheduler = std::thread(scheduler_loop, s);
            s->completer = std::thread(completer_loop, s);
        } catch (const std::system_error &) {
            rc = fail(RV_ERR_HIP, "could not start the server threads");
        }
    }
    if (rc != RV_OK) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stopping = true;
        }
        s->cv_sched.notify_all();
        if (s->scheduler.joinable()) s->scheduler.join();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->sched_done = true;
        }
        s->cv_done.notify_all();
        if (s->completer.joinable()) s->completer.join();
        release_all(s);
        delete s;
        return rc;
    }
    s->st.arena_bytes = (int64_t)cfg->hbm_budget_bytes;
    *server = s;
    return RV_OK;
}

int rv_server_submit(rv_server_t *s, const float *theta, const float *vd,
                     const int32_t *cluster_offsets, int64_t n_clusters, int64_t n_points,
                     uint64_t seed, uint64_t *ticket) {
    return submit_frame(s, theta, vd, cluster_offsets, n_clusters, n_points, seed, ticket, true);
}

int rv_server_submit_pinned(rv_server_t *s, const float *theta, const float *vd,
                            const int32_t *cluster_offsets, int64_t n_clusters, int64_t n_points,
                            uint64_t seed, uint64_t *ticket) {
    return submit_frame(s, theta, vd, cluster_offsets, n_clusters, n_points, seed, ticket, false);
}

int rv_server_wait(rv_server_t *s, uint64_t ticket, int64_t timeout_ms) {
    g_error[0] = '\0';
    if (s == nullptr) return fail(RV_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] {
        auto it = s->frames.find(ticket);
        return it == s->frames.end() || it->second->state >= kDone;
    };
    if (timeout_ms < 0)
        s->cv_ready.wait(lk, ready);
    else
        s->cv_ready.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    auto it = s->frames.find(ticket);
    if (it == s->frames.end()) return fail(RV_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second->state == kFailed) return fail(RV_ERR_HIP, "the batch of ticket %llu failed", (unsigned long long)ticket);
    return it->second->state == kDone ? 1 : 0;
}

int rv_server_result(rv_server_t *s, uint64_t ticket, float *vx, float *vy, float *heading,
                     int32_t *n_inliers, uint8_t *status, int32_t *n_near_tau, int32_t *best_hyp,
                     uint32_t *inlier_bits, rv_frame_times_t *times) {
    g_error[0] = '\0';
    if (s == nullptr) return fail(RV_ERR_INVALID_ARG, "server is NULL");
    Frame *f = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->frames.find(ticket);
        if (it == s->frames.end())
            return fail(RV_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
        f = it->second;
        if (f->state < kDone) return fail(RV_ERR_BUSY, "ticket %llu is not ready", (unsigned long long)ticket);
        if (f->K > 0 && (vx == nullptr || vy == nullptr || heading == nullptr ||
                         n_inliers == nullptr || status == nullptr))
            return fail(RV_ERR_INVALID_ARG, "a required output is NULL");
        if (inlier_bits != nullptr && s->cfg.keep_inlier_bits == 0)
            return fail(RV_ERR_INVALID_ARG, "inlier_bits requested from a server that keeps no masks");
        s->frames.erase(it);
    }
    int rc = RV_OK;
    if (f->state == kFailed) {
        rc = fail(RV_ERR_HIP, "the batch of ticket %llu failed", (unsigned long long)ticket);
    } else if (f->K > 0) {
        const size_t K = (size_t)f->K;
        memcpy(vx, f->vx.data(), 4 * K);
        memcpy(vy, f->vy.data(), 4 * K);
        memcpy(heading, f->heading.data(), 4 * K);
        memcpy(n_inliers, f->n_inliers.data(), 4 * K);
        memcpy(status, f->status.data(), K);
        if (n_near_tau) memcpy(n_near_tau, f->n_near.data(), 4 * K);
        if (best_hyp) memcpy(best_hyp, f->best.data(), 4 * K);
    }
    if (f->state != kFailed && inlier_bits != nullptr && !f->bits.empty())
        memcpy(inlier_bits, f->bits.data(), 4 * f->bits.size());
    if (times) *times = f->times;
    delete f;
    return rc;
}

int rv_server_stats(rv_server_t *s, rv_server_stats_t *stats) {
    g_error[0] = '\0';
    if (s == nullptr || stats == nullptr) return fail(RV_ERR_INVALID_ARG, "server or stats is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *stats = s->st;
    stats->arena_peak_bytes = (int64_t)s->arena.peak();
    stats->pinned_bytes = (int64_t)s->pool.held();
    stats->waiting_frames = (int64_t)s->waiting.size();
    stats->inflight_batches = (int64_t)s->inflight.size();
    return RV_OK;
}

void rv_server_destroy(rv_server_t *s) {
    if (s == nullptr) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_sched.notify_all();
    if (s->scheduler.joinable()) s->scheduler.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->sched_done = true;
    }
    s->cv_done.notify_all();
    if (s->completer.joinable()) s->completer.join();
    release_all(s);
    delete s;
}

}  // extern "C"
