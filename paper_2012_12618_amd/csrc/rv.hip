// rv.hip -- gfx950 kernels and host entry points of the per-cluster RANSAC
// velocity and heading estimator declared in include/rv.h.
//
// A single-frame call enqueues three kernels on the caller's stream:
//   prep    one thread per point: FP64 sincos of the azimuth; stages float32
//           (cos, sin) and v_d for scoring and the float32 low parts of the
//           FP64 (cos, sin) for the solves and the refit;
//           clears the optional frame-wide inlier bitmask and the per-cluster
//           best keys.  Its first workgroup plans the dispatch order: clusters
//           by decreasing size.
//   score   the hot loop.  Workgroup = (cluster, block of 256 hypotheses).
//           Each thread draws one Philox4x32-10 seed pair and solves the 2x2
//           system in FP64 (Sec. 3.1, Alg. 1: seeds, slope and intercept, as the
//           velocity profile of Sec. 3.2, Eq. 6); the float32 (vx, vy) go to LDS.
//           Each wave then owns 64 hypotheses: lanes hold the cluster's points in
//           registers (rows of 64 points), every lane reads the same hypothesis
//           from LDS, and per point two float32 FMAs and one compare produce a
//           64-lane ballot that the scalar unit popcounts (Alg. 1's distance test
//           and inlier count).  The last n mod 64 points of a cluster, when
//           fewer than 32, and whole clusters of at most 64 points are scored
//           with lanes = hypotheses instead (points broadcast from LDS, each
//           lane counting its own inliers; same arithmetic, same counts).  The
//           best (count, lowest index) key of the block is merged per cluster
//           with a 64-bit atomic maximum (Sec. 3.1: the trial with the most
//           inliers is kept).
//   refit   one wave per cluster, or the whole workgroup for clusters of
//           1024 points or more: FP64 re-classification under the kept
//           hypothesis, FP64 normal-equation sums in a fixed reduction tree,
//           2x2 solve (Sec. 3.2, Eq. 7, Alg. 2) and atan2 heading (Eq. 8).
// Small frames without an inlier mask take one launch (small_frame_kernel)
// that runs the same three steps per cluster in one workgroup.  A part of a
// frame (its clusters drawing with their whole-frame indexes, its points found
// through the frame's offsets minus a point base) runs the same kernels; a
// frame in host memory can be copied and estimated part by part.  The batched
// form stages, orders and describes the clusters of many frames, scores them
// from per-XCD work queues in one persistent launch (optionally in the FP16
// residual form) and refits them in one more launch.
//
// No floating-point atomics and fixed reduction orders: results are bitwise
// reproducible run to run and independent of the other clusters in the frame.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "rv.h"
#include "rv_device.h"
#include "rv_internal.h"

// v_writelane_b32: write a wave-uniform value into one lane of a VGPR (the
// LLVM intrinsic; clang exposes no builtin for it).
__device__ int amdgcn_writelane(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// Error text shared by every translation unit of the library.
namespace rv_internal {
thread_local char g_error[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
    return code;
}

// Stage timing (rv_stage_timing / rv_stage_times): events recorded around the
// kernels of a call.
std::mutex g_timing_mutex;
bool g_timing = false;
std::vector<TimedCall> g_pending;   // recorded, not yet read
std::vector<TimedCall> g_free;      // reusable event sets

bool take_timed_call(TimedCall &tc) {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    if (!g_timing) return false;
    if (!g_free.empty()) {
        tc = g_free.back();
        g_free.pop_back();
        return true;
    }
    for (int i = 0; i <= kStages; ++i)
        if (hipEventCreate(&tc.ev[i]) != hipSuccess) return false;
    return true;
}

void keep_timed_call(const TimedCall &tc) {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    g_pending.push_back(tc);
}
}  // namespace rv_internal

namespace {

constexpr int kScoreBlock = 256;        // score: 4 waves x 64 hypotheses, one per thread
constexpr int kRefitBlock = 256;
constexpr int kRefitWaves = kRefitBlock / 64;  // clusters per refit workgroup
constexpr int kRefitBigClass = 41;             // size class of 1024 points: a workgroup each
constexpr int kXcds = 8;                // MI355X: 8 XCDs, workgroups dealt round-robin
constexpr int kPrepBlock = 256;
constexpr int kRowsMax = 16;            // rows of 64 points held in registers per pass
constexpr int kHypGroup = 4;            // hypotheses per LDS fetch in the scoring loop
constexpr int kSizeClasses = 128;       // quarter-octave size classes for the dispatch order
constexpr int64_t kPlanMaxClusters = 1 << 16;  // above this, clusters run in index order
// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Staged points: float32 (cos, sin) and v_d for scoring (v_d = +inf marks a
// point whose azimuth or Doppler value is not finite), the float32 low parts of
// the FP64 (cos, sin) for the solves and the refit (cs64() below), and the
// caller's azimuths for the seed-separation test.
struct Points {
    const float2 *cs32;
    const float *v32;
    const float2 *cslo;
    const float *theta;
};

// FP64 (cos, sin) of a staged point: the float32 value plus its float32 low
// part, c = hi + lo (an exact FP64 sum), within 2^-49 of the FP64 sincos.
// Staging 8 bytes per point for the low parts instead of 16 for the FP64 pair
// shortens the staging kernel, which is bound by its bytes.
__device__ __forceinline__ double2 cs64(float2 hi, float2 lo) {
    return make_double2((double)hi.x + (double)lo.x, (double)hi.y + (double)lo.y);
}

struct Hypothesis {
    double vx, vy;
    bool valid;
};

// Hypothesis h of cluster k: seed pair, validity and the FP64 2x2 solve of
// v_d = vx cos + vy sin at the two seeds (Cramer's rule).
__device__ __forceinline__ Hypothesis make_hypothesis(const Points &pts, Span sp, uint32_t h,
                                                      uint32_t k, uint32_t key0, uint32_t key1) {
    const uint4 u = philox4x32_10(make_uint4(h, k, 0u, 0u), key0, key1);
    uint32_t i, j;
    seed_pair(u.x, u.y, (uint32_t)sp.n, i, j);
    const int64_t pi = sp.lo + i, pj = sp.lo + j;
    // No branch before the solve: all six loads are in flight together, and
    // an invalid pair's solve (possibly inf or NaN) is replaced by NaN.
    const float vi = pts.v32[pi], vj = pts.v32[pj];
    const float ti = pts.theta[pi], tj = pts.theta[pj];
    const double2 ai = cs64(pts.cs32[pi], pts.cslo[pi]), bj = cs64(pts.cs32[pj], pts.cslo[pj]);
    Hypothesis hy;
    hy.valid = ((int)isfinite(vi) & (int)isfinite(vj) &
                (int)(fabs((double)tj - (double)ti) >= RV_MIN_SEED_SEPARATION)) != 0;
    const double ci = ai.x, si = ai.y, cj = bj.x, sj = bj.y;
    const double dvi = vi, dvj = vj;
    const double inv_det = 1.0 / (ci * sj - si * cj);
    const double vx = (dvi * sj - dvj * si) * inv_det;
    const double vy = (ci * dvj - cj * dvi) * inv_det;
    hy.vx = hy.valid ? vx : __builtin_nan("");
    hy.vy = hy.valid ? vy : __builtin_nan("");
    return hy;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Size class of a cluster for the dispatch order: quarter-octave buckets of n,
// larger n -> larger class; clusters with fewer than two points get class 0.
__device__ __forceinline__ int size_class(int64_t n) {
    if (n < 2) return 0;
    const uint32_t u = n > 0x7FFFFFFF ? 0x7FFFFFFFu : (uint32_t)n;
    const int e = 31 - __builtin_clz(u);                      // floor(log2 n) >= 1
    const int frac = e >= 2 ? (int)((u >> (e - 2)) & 3u) : (int)((u << (2 - e)) & 3u);
    const int c = 1 + 4 * e + frac;
    return c < kSizeClasses ? c : kSizeClasses - 1;
}

// Dispatch order of the clusters: a counting sort by decreasing size class, so
// the longest workgroups start first (longest-processing-time-first).  The
// order inside a class depends on atomics; it only affects scheduling.
// Each thread takes clusters tid, tid + 256, ... in groups of kPlanUnroll, whose
// offsets are all loaded before any of their LDS atomics; the exclusive scan
// over the classes (largest first) is one wave's prefix sum, two classes per
// lane.  This workgroup runs beside the staging workgroups and sets the prep
// kernel's length when it is the slower one.
constexpr int kPlanUnroll = 16;
static_assert(kSizeClasses == 2 * kWave, "the class scan takes two classes per lane");

// Exclusive prefix sum of x over the lanes of one full wave.
__device__ __forceinline__ uint32_t wave_exclusive_sum(uint32_t x, int lane) {
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += y;
    }
    return incl - x;
}

// Start of each size class in the dispatch order (largest class first) and the
// number of clusters refit by a whole workgroup; the first wave of the block.
__device__ __forceinline__ void plan_scan(const uint32_t *count, uint32_t *start,
                                          int64_t *__restrict__ n_big) {
    if (threadIdx.x < kWave) {
        // Position q = 0, 1, ... in the dispatch order is class kSizeClasses - 1 - q.
        const int lane = threadIdx.x;
        const int c_hi = kSizeClasses - 1 - 2 * lane, c_lo = c_hi - 1;
        const uint32_t a = count[c_hi], b = count[c_lo];
        const uint32_t excl = wave_exclusive_sum(a + b, lane);
        start[c_hi] = excl;
        start[c_lo] = excl + a;
        // Clusters refit by a whole workgroup: classes kRefitBigClass and up.
        if (c_hi == kRefitBigClass) *n_big = excl + a;
        if (c_lo == kRefitBigClass) *n_big = excl + a + b;
    }
}

__device__ void plan_order(const int32_t *__restrict__ off, int64_t point_base, int64_t n_clusters,
                           int64_t n_points, int32_t *__restrict__ order,
                           int64_t *__restrict__ n_big) {
    __shared__ uint32_t count[kSizeClasses];
    __shared__ uint32_t start[kSizeClasses];
    for (int c = threadIdx.x; c < kSizeClasses; c += kPrepBlock) count[c] = 0;
    __syncthreads();
    const int64_t group = (int64_t)kPlanUnroll * kPrepBlock;
    if (n_clusters <= group) {
        // One group: every thread's classes stay in registers from the count
        // to the placement, so the offsets are read once (their loads queue
        // behind the staging traffic of the other workgroups).
        int cls[kPlanUnroll];
#pragma unroll
        for (int u = 0; u < kPlanUnroll; ++u) {
            const int64_t k = threadIdx.x + (int64_t)u * kPrepBlock;
            cls[u] = k < n_clusters ? size_class(cluster_span(off, k, n_points, point_base).n) : -1;
        }
#pragma unroll
        for (int u = 0; u < kPlanUnroll; ++u)
            if (cls[u] >= 0) atomicAdd(&count[cls[u]], 1u);
        __syncthreads();
        plan_scan(count, start, n_big);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPlanUnroll; ++u) {
            if (cls[u] >= 0) {
                const uint32_t pos = atomicAdd(&start[cls[u]], 1u);
                order[pos] = (int32_t)(threadIdx.x + u * kPrepBlock);
            }
        }
        return;
    }
    for (int64_t k0 = threadIdx.x; k0 < n_clusters; k0 += group) {
        int cls[kPlanUnroll];
#pragma unroll
        for (int u = 0; u < kPlanUnroll; ++u) {
            const int64_t k = k0 + (int64_t)u * kPrepBlock;
            cls[u] = k < n_clusters ? size_class(cluster_span(off, k, n_points, point_base).n) : -1;
        }
#pragma unroll
        for (int u = 0; u < kPlanUnroll; ++u)
            if (cls[u] >= 0) atomicAdd(&count[cls[u]], 1u);
    }
    __syncthreads();
    plan_scan(count, start, n_big);
    __syncthreads();
    for (int64_t k0 = threadIdx.x; k0 < n_clusters; k0 += group) {
        int cls[kPlanUnroll];
#pragma unroll
        for (int u = 0; u < kPlanUnroll; ++u) {
            const int64_t k = k0 + (int64_t)u * kPrepBlock;
            cls[u] = k < n_clusters ? size_class(cluster_span(off, k, n_points, point_base).n) : -1;
        }
#pragma unroll
        for (int u = 0; u < kPlanUnroll; ++u) {
            if (cls[u] >= 0) {
                const uint32_t pos = atomicAdd(&start[cls[u]], 1u);
                order[pos] = (int32_t)(k0 + (int64_t)u * kPrepBlock);
            }
        }
    }
}

// Stages point p: FP64 sincos of its azimuth, float32 (cos, sin) and v_d for
// scoring, and the float32 low parts of the FP64 (cos, sin) (c - (double)(float)c,
// rounded) for the solves and the refit.  A non-finite point is staged as
// (0, 0, +inf) with zero low parts: its float32 residual is inf or NaN, never
// below tau, and +inf marks it for the solves and the refit.
__device__ __forceinline__ void stage_point(const float *__restrict__ theta,
                                            const float *__restrict__ vd, int64_t p,
                                            float2 *__restrict__ cs32, float *__restrict__ v32,
                                            float2 *__restrict__ cslo) {
    const float t = theta[p], v = vd[p];
    double s, c;
    sincos((double)t, &s, &c);
    const bool ok = isfinite(t) && isfinite(v);
    const float ch = ok ? (float)c : 0.0f, sh = ok ? (float)s : 0.0f;
    cs32[p] = make_float2(ch, sh);
    v32[p] = ok ? v : __builtin_inff();
    cslo[p] = make_float2(ok ? (float)(c - (double)ch) : 0.0f, ok ? (float)(s - (double)sh) : 0.0f);
}

// Block 0 plans the order (when `order` is non-null); it is dispatched first,
// so the planning overlaps the staging.  Blocks [1, gridDim.x) stage the
// points and clear the per-cluster best keys.
__global__ __launch_bounds__(kPrepBlock) void prep_kernel(
    const float *__restrict__ theta, const float *__restrict__ vd, int64_t n_points,
    float2 *__restrict__ cs32, float *__restrict__ v32, float2 *__restrict__ cslo,
    uint32_t *__restrict__ bits,
    int64_t n_words, const int32_t *__restrict__ off, int64_t point_base, int64_t n_clusters,
    int32_t *__restrict__ order, int64_t *__restrict__ n_big,
    unsigned long long *__restrict__ best_key) {
    if (blockIdx.x == 0) {
        if (order != nullptr) plan_order(off, point_base, n_clusters, n_points, order, n_big);
        return;
    }
    const int64_t p = (int64_t)(blockIdx.x - 1) * kPrepBlock + threadIdx.x;
    if (p < n_clusters) best_key[p] = 0;
    if (p < n_points) stage_point(theta, vd, p, cs32, v32, cslo);
    if (bits != nullptr && p < n_words) bits[p] = 0u;
}

// R rows of 64 points per lane (registers) against ng groups of kHypGroup
// hypotheses read from LDS (broadcast reads: every lane gets the same (vx, vy));
// returns the count of hypothesis q of the wave in lane q.  kScalarLoop: the
// group count is read as a wave-uniform value, which keeps the loop counter on
// the scalar unit (measured 1 % faster in the persistent batched kernel, 0.5 %
// slower in the single-frame kernel, whose schedule it changes).
template <int R, bool kScalarLoop = false>
__device__ __forceinline__ uint32_t score_rows(const float2 *__restrict__ cs_chunk,
                                               const float *__restrict__ v_chunk, int npts,
                                               int lane, const float4 *hp, int ng, float tau) {
    float c[R], s[R], v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        // Uniform row base and row length, one lane offset: no per-row address
        // registers.
        const int len = npts - r * kWave;
        c[r] = 0.0f;
        s[r] = 0.0f;
        v[r] = __builtin_inff();
        if (lane < len) {
            const float2 q = cs_chunk[r * kWave + lane];
            c[r] = q.x;
            s[r] = q.y;
            v[r] = v_chunk[r * kWave + lane];
        }
    }
    uint32_t counts = 0;
    const int n_groups = kScalarLoop ? __builtin_amdgcn_readfirstlane(ng) : ng;
    for (int g = 0; g < n_groups; ++g) {
        const float4 h0 = hp[2 * g], h1 = hp[2 * g + 1];
        const float hx[kHypGroup] = {h0.x, h0.z, h1.x, h1.z};
        const float hy[kHypGroup] = {h0.y, h0.w, h1.y, h1.w};
#pragma unroll
        for (int u = 0; u < kHypGroup; ++u) {
            uint32_t n = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float t = __builtin_fmaf(-hx[u], c[r], v[r]);
                const float e = __builtin_fmaf(-hy[u], s[r], t);
                n += (uint32_t)__builtin_popcountll(
                    __builtin_amdgcn_ballot_w64(__builtin_fabsf(e) < tau));
            }
            counts = (uint32_t)amdgcn_writelane((int)n, g * kHypGroup + u, (int)counts);
            // One hypothesis at a time: interleaving several keeps R ballot masks
            // per hypothesis live and spills scalar registers.
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    return counts;
}

// Inlier counts of the wave's nh hypotheses (LDS at hp) over all points of the
// cluster, rows_max (<= kMaxRows) register rows of points per pass; lane q
// returns the count of hypothesis q.
template <int kMaxRows = kRowsMax, bool kScalarLoop = false>
__device__ __forceinline__ uint32_t score_cluster(const Points &pts, Span sp, int lane,
                                                  const float4 *hp, int nh, float tau,
                                                  int rows_max) {
    const int ng = (nh + kHypGroup - 1) / kHypGroup;
    const int64_t end = sp.lo + sp.n;
    const int64_t pass = (int64_t)rows_max * kWave;
    uint32_t total = 0;
    for (int64_t base = sp.lo; base < end; base += pass) {
        const int64_t left = end - base;
        const int npts = (int)(left < pass ? left : pass);
        const int rows = (npts + kWave - 1) / kWave;
        const float2 *cs_chunk = pts.cs32 + base;
        const float *v_chunk = pts.v32 + base;
        switch (rows) {
#define RV_ROWS(R)                                                                   \
    case R:                                                                          \
        if constexpr (R <= kMaxRows)                                                 \
            total += score_rows<R, kScalarLoop>(cs_chunk, v_chunk, npts, lane, hp, ng, tau); \
        break;
            RV_ROWS(1) RV_ROWS(2) RV_ROWS(3) RV_ROWS(4) RV_ROWS(5) RV_ROWS(6) RV_ROWS(7)
            RV_ROWS(8) RV_ROWS(9) RV_ROWS(10) RV_ROWS(11) RV_ROWS(12) RV_ROWS(13)
            RV_ROWS(14) RV_ROWS(15) RV_ROWS(16)
#undef RV_ROWS
            default: break;
        }
    }
    return total;
}

// The last t = n mod 64 points of a cluster, when t < kTailLanesMax, are
// scored with lanes = hypotheses instead of as one partly idle row: a row
// costs two FMAs and a compare for 64 lanes whatever t is, while each tail
// point costs every lane two FMAs, a compare and an add (about 12 SIMD-cycles
// per point against about 10 per row and hypothesis), so below about 50 points
// the tail is cheaper this way (thresholds of 32, 48 and 63 measured alike:
// about 5 % off the small frame, 1 % off the batched step, no change on the
// dense frame).  Thread tid holds hypothesis tid of the block
// in both forms, so the two partial counts add up in the same thread; the
// residual and the test are the rows form's, so every count is the same bit
// for bit.
constexpr int kTailLanesMax = 32;

struct TailShared {
    float4 c[kWave / 4], s[kWave / 4], v[kWave / 4];  // padded with (0, 0, +inf)
};

__device__ __forceinline__ int lanes_tail(int64_t n) {
    const int t = (int)(n % kWave);
    return t < kTailLanesMax ? t : 0;
}

// One staged point held by a thread between its loads and its LDS store, so
// that the loads can be issued before other long-latency work (a hypothesis's
// seed loads) and stored after it.
struct PointLoad {
    float2 cs;
    float v;
};

// Thread tid's point among the `count` points from `first` (a valid point of
// the span for the other threads: every load is in bounds, none is used).
__device__ __forceinline__ PointLoad load_point(const Points &pts, int64_t first, int count) {
    const int tid = threadIdx.x;
    const int64_t p = first + (tid < count ? tid : 0);
    PointLoad L;
    L.cs = pts.cs32[p];
    L.v = pts.v32[p];
    return L;
}

// Stores the points of load_point into LDS as float4 quads, padded to a
// multiple of four with (0, 0, +inf), a point that never counts; the caller's
// next block barrier publishes them.
__device__ __forceinline__ void store_points(const PointLoad &L, int count, float4 *c, float4 *s,
                                             float4 *v) {
    const int tid = threadIdx.x;
    if (tid < ((count + 3) & ~3)) {
        const bool real = tid < count;
        reinterpret_cast<float *>(c)[tid] = real ? L.cs.x : 0.0f;
        reinterpret_cast<float *>(s)[tid] = real ? L.cs.y : 0.0f;
        reinterpret_cast<float *>(v)[tid] = real ? L.v : __builtin_inff();
    }
}

// Inliers of hypothesis (hx, hy) among the staged tail points (LDS broadcasts).
__device__ __forceinline__ uint32_t tail_count(const TailShared &sh, int tail, float hx, float hy,
                                               float tau) {
    uint32_t cnt = 0;
    for (int q = 0; q < (tail + 3) / 4; ++q) {
        const float4 c = sh.c[q], sn = sh.s[q], v = sh.v[q];
        const float cc[4] = {c.x, c.y, c.z, c.w}, ss[4] = {sn.x, sn.y, sn.z, sn.w};
        const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float e = __builtin_fmaf(-hy, ss[u], __builtin_fmaf(-hx, cc[u], vv[u]));
            cnt += __builtin_fabsf(e) < tau ? 1u : 0u;
        }
    }
    return cnt;
}

// A cluster's hypotheses: Philox key and the cluster index of the counter
// (the cluster's index within its own frame), and the index of its outputs.
struct ClusterId {
    int64_t out;       // index into the per-cluster outputs
    uint32_t local;    // counter word 1 of its hypotheses
    uint32_t key0, key1;
};

// One scoring block: hypotheses [b * 256, b * 256 + 256) of one cluster.  Each
// thread draws and solves one hypothesis into LDS; each wave then scores 64 of
// them against every point of the cluster.  The block's best (count, lowest
// index) key over its valid hypotheses is merged into best_key with a 64-bit
// atomic maximum, whose result does not depend on the order of the blocks.
// Called by all threads of the block; contains block barriers.
// kUniformTail: the block's key is merged under a wave-uniform guard (needed
// where score_block runs inside a loop with barriers, see batch_score_kernel);
// otherwise under threadIdx.x == 0, which leaves the single-pass kernel's
// register allocation free of spills.
template <bool kUniformTail>
__device__ __forceinline__ void score_block(Span sp, ClusterId id, int b, int32_t n_hyp,
                                            const Points &pts, float tau, int rows_max,
                                            float4 *s_hyp, unsigned long long *s_key,
                                            TailShared &s_tail,
                                            unsigned long long *__restrict__ best_key,
                                            int32_t *__restrict__ hyp_counts) {
    const int tid = threadIdx.x;
    const int64_t h = (int64_t)b * kScoreBlock + tid;
    if (!sp.ok || sp.n < 2) {
        if (hyp_counts != nullptr && h < n_hyp) hyp_counts[id.out * n_hyp + h] = 0;
        return;
    }
    const int tail = lanes_tail(sp.n);  // the same for the whole block
    {
        // The tail points' loads go out before the hypothesis's seed loads and
        // are stored after its solve, so the two latencies overlap.
        PointLoad tl;
        if (tail > 0) tl = load_point(pts, sp.lo + sp.n - tail, tail);
        float hx = __builtin_nanf(""), hy = __builtin_nanf("");
        if (h < n_hyp) {
            const Hypothesis hyp = make_hypothesis(pts, sp, (uint32_t)h, id.local, id.key0, id.key1);
            hx = (float)hyp.vx;  // NaN exactly when the pair is degenerate
            hy = (float)hyp.vy;
        }
        reinterpret_cast<float2 *>(s_hyp)[tid] = make_float2(hx, hy);
        if (tail > 0) store_points(tl, tail, s_tail.c, s_tail.s, s_tail.v);
    }
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int lane = tid % kWave;
    const int64_t h0 = (int64_t)b * kScoreBlock + wave * kWave;
    unsigned long long key = 0;
    if (h0 < n_hyp) {
        const int nh = (int64_t)n_hyp - h0 < kWave ? (int)((int64_t)n_hyp - h0) : kWave;
        Span rows = sp;
        rows.n -= tail;
        uint32_t cnt = score_cluster<kRowsMax, kUniformTail>(
            pts, rows, lane, s_hyp + wave * (kWave / 2), nh, tau, rows_max);
        // The lane's own hypothesis is re-read from LDS rather than kept in
        // registers through the scoring loop.
        const float2 own = reinterpret_cast<const float2 *>(s_hyp)[tid];
        if (tail > 0) cnt += tail_count(s_tail, tail, own.x, own.y, tau);
        const int64_t hl = h0 + lane;
        if (lane < nh) {
            if (hyp_counts != nullptr) hyp_counts[id.out * n_hyp + hl] = (int32_t)cnt;
            if (!__builtin_isnan(own.x))
                key = ((unsigned long long)cnt << 32) | (0xFFFFFFFFull - (uint32_t)hl);
        }
    }
    key = wave_max_u64(key);
    if (lane == 0) s_key[wave] = key;
    __syncthreads();
    if (kUniformTail) {
        if (wave == 0) {  // wave-uniform guard; one lane merges the block's key
            for (int w = 1; w < kScoreBlock / kWave; ++w) key = s_key[w] > key ? s_key[w] : key;
            if (lane == 0 && key != 0) atomicMax(&best_key[id.out], key);
        }
    } else if (tid == 0) {
        for (int w = 1; w < kScoreBlock / kWave; ++w) key = s_key[w] > key ? s_key[w] : key;
        if (key != 0) atomicMax(&best_key[id.out], key);
    }
}

// ---------------------------------------------------------------------------
// FP16 residual form of the scoring (batched form, clusters of at least
// Tuning::fp16_min points).  It selects exactly the hypothesis the float32
// form selects; only the work differs.
//
// Per workgroup (cluster, block of 256 hypotheses):
//   1. reference velocity r = (rx, ry): the block's hypothesis with the most
//      float32 inliers among the cluster's first kFp16Sample points;
//   2. every point of a pass holds half2 (cos, sin) (rounded toward zero) and
//      the float32 residual w = fma(-ry, sin, fma(-rx, cos, v_d)); hypothesis
//      h = (hx, hy) arrives as half2 -(hx - rx, hy - ry), and one
//      v_dot2_f32_f16 adds the two FP16 products to w in float32;
//   3. the FP16 count hi_h uses the widened threshold tau + B_h, where B_h
//      bounds |FP16 residual - float32 residual| at every point whose float32
//      residual is below tau, so hi_h >= the float32 count n_h;
//   4. the hypothesis with the largest (hi_h, lowest index) is counted exactly
//      in float32 (T = its n_h); every other hypothesis with hi_h >= T is
//      counted exactly too.  A hypothesis left out has n_h <= hi_h < T, so the
//      block's best exact key, merged with the same 64-bit atomic maximum, is
//      the float32 form's.
//
// Error bound (A = |hx - rx| + |hy - ry|, M = |hx| + |hy| + |rx| + |ry|, both
// in float32; u = 2^-24): for a point with |float32 residual| < tau, the
// terms are the rounding of w (about u (2|R| + 2A + M)), of -(h - r) to FP16
// (2^-11 A) and of (cos, sin) toward zero (2^-10 A, plus 2^-24 A for FP16
// subnormals), and the sums inside the dot product (at most 8u (2A + |R|));
// together below 2^-9 A + 2^-20 (tau + M + 1).  B_h takes twice that,
// 2^-8 A + 2^-18 (tau + M + 1), which also covers the float32 rounding of
// tau + B_h.  A hypothesis with A >= 2^14 (or not finite) is not converted:
// its FP16 row counts every finite point (threshold +inf), a valid upper bound.
// (cos, sin) below 2^-14 in magnitude may lose their value in the dot product
// if it flushes FP16 subnormals; that error, at most 2^-14 A, is inside 2^-8 A.
// ---------------------------------------------------------------------------

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

constexpr int kFp16Sample = 4 * kWave;  // points of the reference-velocity sample
constexpr float kFp16MaxOffset = 16384.0f;

// (bits of half2 -(h - r), widened threshold) of one hypothesis; an invalid
// one (NaN) gets threshold 0, which no residual passes.
__device__ __forceinline__ float2 fp16_hypothesis(float hx, float hy, float rx, float ry,
                                                  float tau) {
    if (__builtin_isnan(hx) || __builtin_isnan(hy)) return make_float2(0.0f, 0.0f);
    float dx = hx - rx, dy = hy - ry;
    const float a = __builtin_fabsf(dx) + __builtin_fabsf(dy);
    if (!(a < kFp16MaxOffset)) return make_float2(0.0f, __builtin_inff());
    const float m = __builtin_fabsf(hx) + __builtin_fabsf(hy) + __builtin_fabsf(rx) +
                    __builtin_fabsf(ry);
    // An offset component below the smallest normal FP16 value is sent as 0 and
    // its magnitude (at most 2^-14 per point, |cos|, |sin| <= 1) joins the band,
    // so the bound holds whether or not the dot product keeps FP16 subnormals.
    float tiny = 0.0f;
    if (__builtin_fabsf(dx) < 0x1p-14f) {
        tiny += __builtin_fabsf(dx);
        dx = 0.0f;
    }
    if (__builtin_fabsf(dy) < 0x1p-14f) {
        tiny += __builtin_fabsf(dy);
        dy = 0.0f;
    }
    const float band = a * 0x1p-8f + (tau + m + 1.0f) * 0x1p-18f + 2.0f * tiny;
    const half2_t nd = half2_t{(_Float16)(-dx), (_Float16)(-dy)};
    return make_float2(__builtin_bit_cast(float, nd), tau + band);
}

// One hypothesis (nd = half2 -(h - r), threshold t) against four rows of
// points in the FP16 form: e = v_dot2_f32_f16(cs, nd) + w, each product in
// FP16 and the sum in float32, then |e| < t as four 64-lane masks; returns the
// number of set bits.  The VOP3P v_dot2_f32_f16 writes its own destination:
// the compiler's choice, the accumulating v_dot2c_f32_f16, overwrites w and so
// needs a copy of w for every row and hypothesis (three vector instructions
// per row instead of two).  One asm block, so that each compare issues three
// instructions after the dot product whose result it reads: gfx950 needs three
// wait states between a DOT instruction's write and another VALU instruction's
// read of that register.  Every lane must be active (the masks are ballots).
__device__ __forceinline__ uint32_t fp16_count4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                float w0, float w1, float w2, float w3,
                                                uint32_t nd, float t) {
    float e0, e1, e2, e3;
    uint64_t m0, m1, m2, m3;
    asm("v_dot2_f32_f16 %0, %8, %12, %14\n\t"
        "v_dot2_f32_f16 %1, %9, %12, %15\n\t"
        "v_dot2_f32_f16 %2, %10, %12, %16\n\t"
        "v_dot2_f32_f16 %3, %11, %12, %17\n\t"
        "v_cmp_lt_f32_e64 %4, |%0|, %13\n\t"
        "v_cmp_lt_f32_e64 %5, |%1|, %13\n\t"
        "v_cmp_lt_f32_e64 %6, |%2|, %13\n\t"
        "v_cmp_lt_f32_e64 %7, |%3|, %13"
        : "=&v"(e0), "=&v"(e1), "=&v"(e2), "=&v"(e3), "=s"(m0), "=s"(m1), "=s"(m2), "=s"(m3)
        : "v"(c0), "v"(c1), "v"(c2), "v"(c3), "v"(nd), "v"(t), "v"(w0), "v"(w1), "v"(w2),
          "v"(w3));
    return (uint32_t)(__builtin_popcountll(m0) + __builtin_popcountll(m1) +
                      __builtin_popcountll(m2) + __builtin_popcountll(m3));
}

// score_rows in the FP16 form: returns hi of hypothesis q of the wave in lane q.
// R is a multiple of four; rows past the points are padding (w = +inf).
template <int R>
__device__ __forceinline__ uint32_t score_rows_fp16(const float2 *__restrict__ cs_chunk,
                                                    const float *__restrict__ v_chunk, int npts,
                                                    int lane, const float4 *hp, int ng, float rx,
                                                    float ry) {
    static_assert(R % 4 == 0, "rows come in blocks of four");
    uint32_t cs[R];
    float w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int len = npts - r * kWave;
        cs[r] = 0u;
        w[r] = __builtin_inff();
        if (lane < len) {
            const float2 q = cs_chunk[r * kWave + lane];
            const float v = v_chunk[r * kWave + lane];
            cs[r] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(q.x, q.y));
            w[r] = __builtin_fmaf(-ry, q.y, __builtin_fmaf(-rx, q.x, v));
        }
    }
    uint32_t counts = 0;
    for (int g = 0; g < ng; ++g) {
        const float4 h0 = hp[2 * g], h1 = hp[2 * g + 1];
        const float hd[kHypGroup] = {h0.x, h0.z, h1.x, h1.z};
        const float ht[kHypGroup] = {h0.y, h0.w, h1.y, h1.w};
#pragma unroll
        for (int u = 0; u < kHypGroup; ++u) {
            const uint32_t nd = __builtin_bit_cast(uint32_t, hd[u]);
            uint32_t n = 0;
#pragma unroll
            for (int r = 0; r < R; r += 4)
                n += fp16_count4(cs[r], cs[r + 1], cs[r + 2], cs[r + 3], w[r], w[r + 1], w[r + 2],
                                 w[r + 3], nd, ht[u]);
            counts = (uint32_t)amdgcn_writelane((int)n, g * kHypGroup + u, (int)counts);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    return counts;
}

// score_cluster in the FP16 form (a pass's rows rounded up to a multiple of
// four).
__device__ __forceinline__ uint32_t score_cluster_fp16(const Points &pts, Span sp, int lane,
                                                       const float4 *hp, int nh, int rows_max,
                                                       float rx, float ry) {
    const int ng = (nh + kHypGroup - 1) / kHypGroup;
    const int64_t end = sp.lo + sp.n;
    const int64_t pass = (int64_t)rows_max * kWave;
    uint32_t total = 0;
    for (int64_t base = sp.lo; base < end; base += pass) {
        const int64_t left = end - base;
        const int npts = (int)(left < pass ? left : pass);
        const int blocks = (npts + 4 * kWave - 1) / (4 * kWave);
        const float2 *cs_chunk = pts.cs32 + base;
        const float *v_chunk = pts.v32 + base;
        switch (blocks) {
#define RV_ROWS16(B)                                                                       \
    case B:                                                                                \
        total += score_rows_fp16<4 * B>(cs_chunk, v_chunk, npts, lane, hp, ng, rx, ry);    \
        break;
            RV_ROWS16(1) RV_ROWS16(2) RV_ROWS16(3) RV_ROWS16(4)
#undef RV_ROWS16
            default: break;
        }
    }
    return total;
}

// Workgroup LDS of the FP16 form.
struct Fp16Shared {
    float4 h32[kScoreBlock / 2];               // float32 (vx, vy) of the block's hypotheses
    float4 h16[kScoreBlock / 2];               // fp16_hypothesis() of each
    float4 list[kWave / 2];                    // hypotheses counted exactly, float32
    uint32_t part[kScoreBlock / kWave][kWave]; // per-wave partial exact counts
    uint32_t idx[kScoreBlock];                 // candidates: positions in the block
    unsigned long long key[kScoreBlock / kWave];
    uint32_t n_cand[kScoreBlock / kWave];
};

constexpr int kExactRows = 8;  // register rows per pass of the exact counts

__device__ __forceinline__ unsigned long long hyp_key(uint32_t count, int64_t h) {
    return ((unsigned long long)count << 32) | (0xFFFFFFFFull - (uint32_t)h);
}

// ---------------------------------------------------------------------------
// Small clusters with lanes = hypotheses (batched form, clusters of at most
// Tuning::lanes_max points, at most kLaneTile).  With lanes = points a cluster
// of n < 64 points leaves 64 - n lanes of every compare idle; here each thread
// keeps the hypothesis it solved in registers, the cluster's points are staged
// in LDS and read by every lane at the same address (a broadcast), and each
// lane counts its own inliers with one compare and one add per point: four
// vector instructions per point and 64 hypotheses, none on the scalar unit.
// The residual and the test are the float32 loop's, fma(-hy, s, fma(-hx, c,
// v_d)) and |.| < tau, so every count, and the block's key, is the same bit for
// bit.
// ---------------------------------------------------------------------------

constexpr int kLaneTile = 256;        // points staged in LDS: the largest cluster of this form
constexpr int kDefaultLanesMax = 64;  // default Tuning::lanes_max
// Single-frame calls (score_kernel, small_frame_kernel): clusters of at most
// this many points score with lanes = hypotheses.
constexpr int kSingleLanesMax = 64;

struct LaneShared {
    float4 c[kLaneTile / 4], s[kLaneTile / 4], v[kLaneTile / 4];  // padded with (0, 0, +inf)
    unsigned long long key[kScoreBlock / kWave];
};

// One scoring block of a cluster with 2 <= n <= kLaneTile points, lanes =
// hypotheses.  Called by all threads of the block from the persistent loop
// (every branch around a barrier is on a wave-uniform value).
__device__ __forceinline__ void score_block_lanes(Span sp, ClusterId id, int b, int32_t n_hyp,
                                                  const Points &pts, float tau, LaneShared &sh,
                                                  unsigned long long *__restrict__ best_key,
                                                  int32_t *__restrict__ hyp_counts) {
    const int tid = threadIdx.x;
    const int n = (int)sp.n;
    const int n4 = (n + 3) / 4;
    // The point loads go out before the hypothesis's seed loads and are stored
    // after its solve, so the two latencies overlap.
    const PointLoad pl = load_point(pts, sp.lo, n);
    const int64_t h = (int64_t)b * kScoreBlock + tid;
    float hx = __builtin_nanf(""), hy = __builtin_nanf("");
    if (h < n_hyp) {
        const Hypothesis hyp = make_hypothesis(pts, sp, (uint32_t)h, id.local, id.key0, id.key1);
        hx = (float)hyp.vx;  // NaN exactly when the pair is degenerate: counts 0
        hy = (float)hyp.vy;
    }
    store_points(pl, n, sh.c, sh.s, sh.v);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int lane = tid % kWave;
    uint32_t cnt = 0;
    for (int q = 0; q < n4; ++q) {
        const float4 c = sh.c[q], sn = sh.s[q], v = sh.v[q];
        const float cc[4] = {c.x, c.y, c.z, c.w}, ss[4] = {sn.x, sn.y, sn.z, sn.w};
        const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float e = __builtin_fmaf(-hy, ss[u], __builtin_fmaf(-hx, cc[u], vv[u]));
            cnt += __builtin_fabsf(e) < tau ? 1u : 0u;
        }
    }
    unsigned long long key = 0;
    if (h < n_hyp) {
        if (hyp_counts != nullptr) hyp_counts[id.out * n_hyp + h] = (int32_t)cnt;
        if (!__builtin_isnan(hx)) key = hyp_key(cnt, h);
    }
    key = wave_max_u64(key);
    if (lane == 0) sh.key[wave] = key;
    __syncthreads();
    if (wave == 0) {  // wave-uniform guard; one lane merges the block's key
        for (int w = 1; w < kScoreBlock / kWave; ++w) key = sh.key[w] > key ? sh.key[w] : key;
        if (lane == 0 && key != 0) atomicMax(&best_key[id.out], key);
    }
    // The next item restages the tile only after the work-queue fetch's two
    // block barriers, which every wave reaches after its last read of it.
}

// Exact float32 counts of the nl (<= 64) hypotheses in sh.list over the whole
// cluster; wave w scores rows [w rows/4, (w+1) rows/4) of the cluster.  Lane q
// of every wave returns the count of list entry q.  Contains barriers.
__device__ __forceinline__ uint32_t exact_counts(Span sp, const Points &pts, float tau, int nl,
                                                 Fp16Shared &sh, int wave, int lane) {
    const int64_t rows = (sp.n + kWave - 1) / kWave;
    const int64_t r0 = rows * wave / (kScoreBlock / kWave);
    const int64_t r1 = rows * (wave + 1) / (kScoreBlock / kWave);
    const int64_t p1 = r1 * kWave < sp.n ? r1 * kWave : sp.n;
    Span part;
    part.lo = sp.lo + r0 * kWave;
    part.n = p1 - r0 * kWave;
    part.ok = true;
    sh.part[wave][lane] = score_cluster<kExactRows>(pts, part, lane, sh.list, nl, tau, kExactRows);
    __syncthreads();
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < kScoreBlock / kWave; ++w) total += sh.part[w][lane];
    __syncthreads();
    return total;
}

// One scoring block in the FP16 form (sp.ok and sp.n >= 2; called from the
// persistent loop: every branch around a barrier is on a wave-uniform value).
// hyp_counts, when requested, receives hi_h.
__device__ __forceinline__ void score_block_fp16(Span sp, ClusterId id, int b, int32_t n_hyp,
                                                 const Points &pts, float tau, int rows_max,
                                                 Fp16Shared &sh,
                                                 unsigned long long *__restrict__ best_key,
                                                 int32_t *__restrict__ hyp_counts) {
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)b * kScoreBlock;
    const int64_t h = base + tid;
    float hx = __builtin_nanf(""), hy = __builtin_nanf("");
    if (h < n_hyp) {
        const Hypothesis hyp = make_hypothesis(pts, sp, (uint32_t)h, id.local, id.key0, id.key1);
        hx = (float)hyp.vx;
        hy = (float)hyp.vy;
    }
    float2 *h32 = reinterpret_cast<float2 *>(sh.h32);
    h32[tid] = make_float2(hx, hy);
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int lane = tid % kWave;
    const int64_t w0 = base + wave * kWave;
    const int nh = w0 < n_hyp ? ((int64_t)n_hyp - w0 < kWave ? (int)((int64_t)n_hyp - w0) : kWave)
                              : 0;

    // 1. Reference velocity from the sample.
    Span sample = sp;
    sample.n = sp.n < kFp16Sample ? sp.n : kFp16Sample;
    unsigned long long key = 0;
    if (nh > 0) {
        const uint32_t cnt = score_cluster<kFp16Sample / kWave>(
            pts, sample, lane, sh.h32 + wave * (kWave / 2), nh, tau, kFp16Sample / kWave);
        if (lane < nh && !__builtin_isnan(h32[tid].x)) key = hyp_key(cnt, base + tid);
    }
    key = wave_max_u64(key);
    if (lane == 0) sh.key[wave] = key;
    __syncthreads();
    unsigned long long ref = 0;
#pragma unroll
    for (int w = 0; w < kScoreBlock / kWave; ++w) ref = sh.key[w] > ref ? sh.key[w] : ref;
    ref = uniform_u64(ref);
    float rx = 0.0f, ry = 0.0f;
    if (ref != 0) {
        const float2 r = h32[(0xFFFFFFFFu - (uint32_t)ref) - (uint32_t)base];
        if (__builtin_fabsf(r.x) + __builtin_fabsf(r.y) < kFp16MaxOffset) {
            rx = r.x;
            ry = r.y;
        }
    }
    // The same value in every lane: kept in scalar registers.
    rx = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, rx)));
    ry = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, ry)));
    reinterpret_cast<float2 *>(sh.h16)[tid] = fp16_hypothesis(hx, hy, rx, ry, tau);
    __syncthreads();

    // 2-3. FP16 upper-bound counts (the lane's own hypothesis is re-read from
    // LDS afterwards rather than kept in registers through the loop).
    uint32_t hi = 0;
    if (nh > 0) hi = score_cluster_fp16(pts, sp, lane, sh.h16 + wave * (kWave / 2), nh, rows_max, rx, ry);
    const bool valid = lane < nh && !__builtin_isnan(h32[tid].x);
    // A hypothesis without a finite widened threshold (offset beyond the FP16
    // range) counted every finite point: its hi says nothing about its count.
    const bool wide = valid && !(reinterpret_cast<const float2 *>(sh.h16)[tid].y < __builtin_inff());
    if (hyp_counts != nullptr && lane < nh) hyp_counts[id.out * n_hyp + base + tid] = (int32_t)hi;
    key = valid && !wide ? hyp_key(hi, base + tid) : 0ull;
    key = wave_max_u64(key);
    const uint64_t wide_mask = __builtin_amdgcn_ballot_w64(wide);
    if (lane == 0) {
        sh.key[wave] = key;
        sh.n_cand[wave] = (uint32_t)__builtin_popcountll(wide_mask);
    }
    __syncthreads();
    unsigned long long top = 0;
    uint32_t wide_before = 0, n_wide = 0;
#pragma unroll
    for (int w = 0; w < kScoreBlock / kWave; ++w) {
        top = sh.key[w] > top ? sh.key[w] : top;
        const uint32_t c = sh.n_cand[w];
        wide_before += w < wave ? c : 0u;
        n_wide += c;
    }
    top = uniform_u64(top);
    n_wide = __builtin_amdgcn_readfirstlane(n_wide);
    if (top == 0 && n_wide == 0) return;  // no valid hypothesis in this block

    // 4. Exact float32 counts.  First pass: the hypothesis with the largest
    // (hi, lowest index) among those with a finite threshold (T = its exact
    // count) together with the hypotheses without one, up to 64 in all.  Then
    // every other valid hypothesis with hi >= T, 64 per pass.  A hypothesis
    // left out has n_h <= hi_h < T, so the best exact key is the float32 form's.
    const uint32_t has_top = top != 0 ? 1u : 0u;
    const uint32_t h_top = 0xFFFFFFFFu - (uint32_t)top;
    const uint32_t wide_rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(wide_mask >> 32),
                                  __builtin_amdgcn_mbcnt_lo((uint32_t)wide_mask, 0u));
    const uint32_t slot = has_top + wide_before + wide_rank;
    const bool first = wide && slot < (uint32_t)kWave;  // counted in the first pass
    if (first) {
        reinterpret_cast<float2 *>(sh.list)[slot] = h32[tid];
        sh.idx[slot] = (uint32_t)tid;
    }
    if (tid == 0 && has_top) {
        reinterpret_cast<float2 *>(sh.list)[0] = h32[h_top - (uint32_t)base];
        sh.idx[0] = h_top - (uint32_t)base;
    }
    __syncthreads();
    const uint32_t n1 = has_top + n_wide < (uint32_t)kWave ? has_top + n_wide : (uint32_t)kWave;
    const uint32_t c1 = exact_counts(sp, pts, tau, (int)n1, sh, wave, lane);
    const uint32_t t_exact = has_top ? __builtin_amdgcn_readfirstlane(c1) : 0u;
    unsigned long long best = lane < (int)n1 ? hyp_key(c1, base + sh.idx[lane]) : 0ull;
    best = wave_max_u64(best);
    const bool cand = valid && !first && (!has_top || (uint32_t)(base + tid) != h_top) &&
                      hi >= t_exact;
    const uint64_t m = __builtin_amdgcn_ballot_w64(cand);
    if (lane == 0) sh.n_cand[wave] = (uint32_t)__builtin_popcountll(m);
    __syncthreads();
    uint32_t before = 0, n_cand = 0;
#pragma unroll
    for (int w = 0; w < kScoreBlock / kWave; ++w) {
        const uint32_t c = sh.n_cand[w];
        before += w < wave ? c : 0u;
        n_cand += c;
    }
    n_cand = __builtin_amdgcn_readfirstlane(n_cand);
    if (cand) {
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        sh.idx[before + rank] = (uint32_t)tid;
    }
    __syncthreads();
    for (uint32_t c0 = 0; c0 < n_cand; c0 += kWave) {
        const int nl = n_cand - c0 < (uint32_t)kWave ? (int)(n_cand - c0) : kWave;
        if (tid < nl) reinterpret_cast<float2 *>(sh.list)[tid] = h32[sh.idx[c0 + tid]];
        __syncthreads();
        const uint32_t cnt = exact_counts(sp, pts, tau, nl, sh, wave, lane);
        unsigned long long k2 = 0;
        if (lane < nl) k2 = hyp_key(cnt, base + sh.idx[c0 + lane]);
        k2 = wave_max_u64(k2);
        best = k2 > best ? k2 : best;
    }
    if (wave == 0) {
        if (lane == 0) atomicMax(&best_key[id.out], best);
    }
}

struct Outputs {
    float *vx, *vy, *heading;
    int32_t *n_inliers;
    uint8_t *status;
    int32_t *n_near, *best, *hyp_counts;
    uint32_t *bits;
};

__device__ __forceinline__ void write_failed(const Outputs &o, int64_t k, uint8_t st) {
    const float qnan = __builtin_nanf("");
    o.vx[k] = qnan;
    o.vy[k] = qnan;
    o.heading[k] = qnan;
    o.n_inliers[k] = 0;
    o.status[k] = st;
    if (o.n_near) o.n_near[k] = 0;
    if (o.best) o.best[k] = -1;
}

// FP64 sums of a refit, per lane.
struct RefitSums {
    double scc = 0.0, scs = 0.0, sss = 0.0, scv = 0.0, ssv = 0.0;
    int n_in = 0, n_near = 0;
};

// Re-classification of one 64-aligned block of points [p0, p0 + 64) under h*
// (one wave, wave-uniform call): lane point p = p0 + lane counts when it lies
// in [lo, end) and its v_d is finite (+inf marks a non-finite point); the
// block's ballot fills two words of the frame-wide mask.  v and cs are loaded
// by the caller, so that the loads of several blocks are in flight together.
__device__ __forceinline__ void refit_points(int64_t p0, bool in_range, float v, double2 cs,
                                             const Hypothesis &hy, double dtau, RefitSums &a,
                                             const Outputs &o, int lane) {
    bool inlier = false;
    if (in_range && isfinite(v)) {
        const double c = cs.x, s = cs.y, dv = v;
        const double res = fabs(dv - hy.vx * c - hy.vy * s);
        a.n_near += fabs(res - dtau) <= RV_NEAR_TAU_WINDOW ? 1 : 0;
        if (res < dtau) {
            inlier = true;
            a.n_in += 1;
            a.scc += c * c;
            a.scs += c * s;
            a.sss += s * s;
            a.scv += c * dv;
            a.ssv += s * dv;
        }
    }
    if (o.bits != nullptr) {
        const uint64_t m = __builtin_amdgcn_ballot_w64(inlier);
        if (lane == 0) {
            const uint32_t w0 = (uint32_t)m, w1 = (uint32_t)(m >> 32);
            if (w0) atomicOr(&o.bits[p0 >> 5], w0);
            if (w1) atomicOr(&o.bits[(p0 >> 5) + 1], w1);
        }
    }
}

// All points of a cluster under h*, 64-aligned blocks from first_block in
// steps of `stride`, kRefitUnroll blocks per iteration: the loads of all of
// them are issued (from a clamped, always valid index) before any block is
// used.  Each lane visits its points in the same order as one block per
// iteration, so the sums are the same.  The first iteration's loads do not
// depend on h*: the callers issue them (refit_load) before solving h*, so
// their latency overlaps the hypothesis's.
constexpr int kRefitUnroll = 4;

struct RefitLoads {
    float v[kRefitUnroll];
    float2 hi[kRefitUnroll], lo[kRefitUnroll];
    bool in[kRefitUnroll];
};

__device__ __forceinline__ RefitLoads refit_load(Span sp, int64_t p0, int64_t stride,
                                                 const Points &pts, int lane) {
    RefitLoads L;
    const int64_t end = sp.lo + sp.n;
#pragma unroll
    for (int u = 0; u < kRefitUnroll; ++u) {
        const int64_t p = p0 + u * stride + lane;
        L.in[u] = p >= sp.lo && p < end;
        const int64_t q = L.in[u] ? p : sp.lo;
        L.v[u] = pts.v32[q];
        L.hi[u] = pts.cs32[q];
        L.lo[u] = pts.cslo[q];
    }
    return L;
}

__device__ __forceinline__ void refit_group(const RefitLoads &L, int64_t p0, int64_t stride,
                                            int64_t end, const Hypothesis &hy, double dtau,
                                            RefitSums &a, const Outputs &o, int lane) {
#pragma unroll
    for (int u = 0; u < kRefitUnroll; ++u)
        if (p0 + u * stride < end)
            refit_points(p0 + u * stride, L.in[u], L.v[u], cs64(L.hi[u], L.lo[u]), hy, dtau, a, o,
                         lane);
}

// The first group's loads come from the caller (issued before the hypothesis
// solve); the first group is taken apart from the loop so that no copy of a
// whole group of loads is selected at run time (such a select puts the group
// in scratch memory).
__device__ __forceinline__ RefitSums refit_sweep(Span sp, int64_t first_block, int64_t stride,
                                                 const RefitLoads &first, const Points &pts,
                                                 const Hypothesis &hy, double dtau,
                                                 const Outputs &o, int lane) {
    RefitSums a;
    const int64_t end = sp.lo + sp.n;
    refit_group(first, first_block, stride, end, hy, dtau, a, o, lane);
    for (int64_t p0 = first_block + kRefitUnroll * stride; p0 < end; p0 += kRefitUnroll * stride)
        refit_group(refit_load(sp, p0, stride, pts, lane), p0, stride, end, hy, dtau, a, o, lane);
    return a;
}

// Refit of one cluster by one workgroup of kRefitBlock threads: the kept
// hypothesis (from its best key), FP64 re-classification of every point under
// it, least-squares refit on its inliers (Sec. 3.2, Eq. 7, Alg. 2: normal
// equations A^T A v = A^T v_d, summed per thread and reduced in a fixed tree)
// and heading atan2(vy, vx) (Eq. 8).
__device__ __forceinline__ void refit_block(Span sp, ClusterId id, unsigned long long best,
                                            const Points &pts, float tau, const Outputs &o,
                                            double (*s_sum)[5], int (*s_cnt)[2]) {
    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    const int64_t k = id.out;
    if (!sp.ok || sp.n < 2) {
        if (tid == 0) write_failed(o, k, sp.ok ? RV_CLUSTER_TOO_FEW_POINTS : RV_CLUSTER_BAD_OFFSETS);
        return;
    }
    if (best == 0) {
        if (tid == 0) write_failed(o, k, RV_CLUSTER_ALL_DEGENERATE);
        return;
    }
    // Waves walk 64-aligned global blocks so one wave ballot maps onto two
    // words of the frame-wide bitmask.
    const int64_t first_block = (sp.lo & ~(int64_t)(kWave - 1)) + (int64_t)wave * kWave;
    const RefitLoads first = refit_load(sp, first_block, kRefitBlock, pts, lane);
    const uint32_t hbest = 0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull);
    const Hypothesis hy = make_hypothesis(pts, sp, hbest, id.local, id.key0, id.key1);
    const double dtau = tau;
    const RefitSums a = refit_sweep(sp, first_block, kRefitBlock, first, pts, hy, dtau, o, lane);
    double scc = a.scc, scs = a.scs, sss = a.sss, scv = a.scv, ssv = a.ssv;
    int n_in = a.n_in, n_near = a.n_near;
    scc = wave_sum(scc);
    scs = wave_sum(scs);
    sss = wave_sum(sss);
    scv = wave_sum(scv);
    ssv = wave_sum(ssv);
    n_in = wave_sum_i(n_in);
    n_near = wave_sum_i(n_near);
    if (lane == 0) {
        s_sum[wave][0] = scc;
        s_sum[wave][1] = scs;
        s_sum[wave][2] = sss;
        s_sum[wave][3] = scv;
        s_sum[wave][4] = ssv;
        s_cnt[wave][0] = n_in;
        s_cnt[wave][1] = n_near;
    }
    __syncthreads();
    if (tid != 0) return;
    scc = s_sum[0][0];
    scs = s_sum[0][1];
    sss = s_sum[0][2];
    scv = s_sum[0][3];
    ssv = s_sum[0][4];
    n_in = s_cnt[0][0];
    n_near = s_cnt[0][1];
    for (int w = 1; w < kRefitBlock / kWave; ++w) {
        scc += s_sum[w][0];
        scs += s_sum[w][1];
        sss += s_sum[w][2];
        scv += s_sum[w][3];
        ssv += s_sum[w][4];
        n_in += s_cnt[w][0];
        n_near += s_cnt[w][1];
    }
    o.n_inliers[k] = n_in;
    if (o.n_near) o.n_near[k] = n_near;
    if (o.best) o.best[k] = (int32_t)hbest;
    const double det = scc * sss - scs * scs;
    if (n_in < 2 || !(det > 0.0)) {
        const float qnan = __builtin_nanf("");
        o.vx[k] = qnan;
        o.vy[k] = qnan;
        o.heading[k] = qnan;
        o.status[k] = RV_CLUSTER_SINGULAR_REFIT;
        return;
    }
    const double fvx = (sss * scv - scs * ssv) / det;
    const double fvy = (scc * ssv - scs * scv) / det;
    o.vx[k] = (float)fvx;
    o.vy[k] = (float)fvy;
    o.heading[k] = (float)atan2(fvy, fvx);
    o.status[k] = RV_CLUSTER_OK;
}

// Refit of one cluster by one wave: the kept hypothesis (from its best key),
// FP64 re-classification of every point under it, least-squares refit on its
// inliers (Sec. 3.2, Eq. 7, Alg. 2: normal equations A^T A v = A^T v_d, summed
// per lane over the cluster's 64-point blocks and reduced across the wave in a
// fixed tree) and heading atan2(vy, vx) (Eq. 8).  One wave per cluster keeps
// small clusters from idling a whole workgroup and needs no barrier.
__device__ __forceinline__ void refit_wave(Span sp, ClusterId id, unsigned long long best,
                                           const Points &pts, float tau, const Outputs &o) {
    const int lane = threadIdx.x % kWave;
    const int64_t k = id.out;
    if (!sp.ok || sp.n < 2) {
        if (lane == 0) write_failed(o, k, sp.ok ? RV_CLUSTER_TOO_FEW_POINTS : RV_CLUSTER_BAD_OFFSETS);
        return;
    }
    if (best == 0) {
        if (lane == 0) write_failed(o, k, RV_CLUSTER_ALL_DEGENERATE);
        return;
    }
    // 64-aligned global blocks of points, so one ballot maps onto two words of
    // the frame-wide bitmask.
    const int64_t first_block = sp.lo & ~(int64_t)(kWave - 1);
    const RefitLoads first = refit_load(sp, first_block, kWave, pts, lane);
    const uint32_t hbest = 0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull);
    const Hypothesis hy = make_hypothesis(pts, sp, hbest, id.local, id.key0, id.key1);
    const double dtau = tau;
    const RefitSums a = refit_sweep(sp, first_block, kWave, first, pts, hy, dtau, o, lane);
    double scc = a.scc, scs = a.scs, sss = a.sss, scv = a.scv, ssv = a.ssv;
    int n_in = a.n_in, n_near = a.n_near;
    scc = wave_sum(scc);
    scs = wave_sum(scs);
    sss = wave_sum(sss);
    scv = wave_sum(scv);
    ssv = wave_sum(ssv);
    n_in = wave_sum_i(n_in);
    n_near = wave_sum_i(n_near);
    if (lane != 0) return;
    o.n_inliers[k] = n_in;
    if (o.n_near) o.n_near[k] = n_near;
    if (o.best) o.best[k] = (int32_t)hbest;
    const double det = scc * sss - scs * scs;
    if (n_in < 2 || !(det > 0.0)) {
        const float qnan = __builtin_nanf("");
        o.vx[k] = qnan;
        o.vy[k] = qnan;
        o.heading[k] = qnan;
        o.status[k] = RV_CLUSTER_SINGULAR_REFIT;
        return;
    }
    const double fvx = (sss * scv - scs * ssv) / det;
    const double fvy = (scc * ssv - scs * scv) / det;
    o.vx[k] = (float)fvx;
    o.vy[k] = (float)fvy;
    o.heading[k] = (float)atan2(fvy, fvx);
    o.status[k] = RV_CLUSTER_OK;
}

// ---- single frame ---------------------------------------------------------

// Work item = (cluster, block of 256 hypotheses).  Block i takes the item that
// keeps clusters in the planned order while all items of one cluster run on the
// same XCD (blocks are dealt to the 8 XCDs round-robin), sharing that XCD's L2
// copy of the cluster's points.  Eight waves per SIMD: the scoring loop fits in
// 64 VGPRs.
__global__ __launch_bounds__(kScoreBlock) __attribute__((amdgpu_waves_per_eu(8))) void score_kernel(
    const int32_t *__restrict__ off, const int32_t *__restrict__ order, int64_t n_clusters,
    int64_t n_points, int32_t n_hyp, int32_t blocks_per_cluster, uint32_t key0, uint32_t key1,
    uint32_t cluster_base, int64_t point_base, Points pts, float tau,
    unsigned long long *__restrict__ best_key, int32_t *__restrict__ hyp_counts) {
    __shared__ float4 s_hyp[kScoreBlock / 2];  // (vx, vy) pairs, two per float4
    __shared__ unsigned long long s_key[kScoreBlock / kWave];
    __shared__ LaneShared s_lanes;
    __shared__ TailShared s_tail;
    const uint32_t xcd = blockIdx.x % kXcds;
    const uint32_t r = blockIdx.x / kXcds;
    const int64_t j = xcd + (int64_t)kXcds * (r / (uint32_t)blocks_per_cluster);
    if (j >= n_clusters) return;
    const int b = (int)(r % (uint32_t)blocks_per_cluster);
    const int64_t k = order != nullptr ? order[j] : j;
    ClusterId id;
    id.out = k;
    id.local = cluster_base + (uint32_t)k;
    id.key0 = key0;
    id.key1 = key1;
    const Span sp = cluster_span(off, k, n_points, point_base);
    if (sp.ok && sp.n >= 2 && sp.n <= kSingleLanesMax) {  // the same for the whole block
        score_block_lanes(sp, id, b, n_hyp, pts, tau, s_lanes, best_key, hyp_counts);
        return;
    }
    score_block<false>(sp, id, b, n_hyp, pts, tau, kRowsMax, s_hyp, s_key, s_tail, best_key,
                       hyp_counts);
}

// Refit of a frame's or batch's clusters over their planned (largest-first)
// positions, in one launch: workgroups [0, n_big) take the first n_big
// clusters (size class >= kRefitBigClass, i.e. >= 1024 points), one each with
// all four waves (refit_block); the following workgroups take the other
// clusters four at a time, one per wave (refit_wave).  n_big is counted on the
// device by the ordering pass; without an order (n_big == nullptr) every
// cluster gets a workgroup.  The grid is an upper bound (one workgroup per
// cluster); surplus workgroups exit at once.
template <typename ClusterAt>
__device__ __forceinline__ void refit_planned(int64_t n_clusters, const int64_t *n_big,
                                              const ClusterAt &at, const Points &pts, float tau,
                                              const Outputs &o, double (*s_sum)[5],
                                              int (*s_cnt)[2]) {
    const int64_t b = blockIdx.x;
    const int64_t big = n_big != nullptr ? *n_big : n_clusters;
    if (b < big) {
        refit_block(at.span(b), at.id(b), at.best(b), pts, tau, o, s_sum, s_cnt);
        return;
    }
    const int64_t j = big + (b - big) * kRefitWaves + threadIdx.x / kWave;
    if (j >= n_clusters) return;
    refit_wave(at.span(j), at.id(j), at.best(j), pts, tau, o);
}

// Cluster at planned position j of a single frame.
struct FrameClusterAt {
    const int32_t *off, *order;
    int64_t n_points;
    uint32_t key0, key1, cluster_base;
    int64_t point_base;
    const unsigned long long *best_key;
    __device__ int64_t index(int64_t j) const { return order != nullptr ? order[j] : j; }
    __device__ Span span(int64_t j) const {
        return cluster_span(off, index(j), n_points, point_base);
    }
    __device__ unsigned long long best(int64_t j) const { return best_key[index(j)]; }
    __device__ ClusterId id(int64_t j) const {
        ClusterId c;
        c.out = index(j);
        c.local = cluster_base + (uint32_t)c.out;
        c.key0 = key0;
        c.key1 = key1;
        return c;
    }
};

__global__ __launch_bounds__(kRefitBlock) void refit_kernel(
    const int32_t *__restrict__ off, const int32_t *__restrict__ order, int64_t n_clusters,
    const int64_t *__restrict__ n_big, int64_t n_points, uint32_t key0, uint32_t key1,
    uint32_t cluster_base, int64_t point_base, Points pts,
    const unsigned long long *__restrict__ best_key, float tau, Outputs o) {
    __shared__ double s_sum[kRefitBlock / kWave][5];
    __shared__ int s_cnt[kRefitBlock / kWave][2];
    const FrameClusterAt at = {off, order, n_points, key0, key1, cluster_base, point_base,
                               best_key};
    refit_planned(n_clusters, n_big, at, pts, tau, o, s_sum, s_cnt);
}

// ---- many frames in one launch sequence ----------------------------------
//
// The frames share one CSR: frame f owns clusters [frame_off[f], frame_off[f+1]).
// A cluster draws its hypotheses with its frame's seed and its index within
// the frame, so its result is bitwise the one a single-frame call gives.  The
// scoring kernel is persistent: a fixed grid drains device work queues of
// (cluster, 256-hypothesis block) items, clusters largest first.  There is one
// queue per XCD (its own 256-byte line): cluster j of the dispatch order
// belongs to queue j % 8, and workgroup b serves queue b % 8 first (workgroups
// are dispatched to the XCDs round-robin), so a cluster's blocks share one L2
// and no counter is hammered by the whole chip; a workgroup whose queue is
// empty takes items from the others.

// Small frames (see use_small_frame_path): one workgroup per cluster stages the
// cluster's own points, scores its hypotheses (at most 256: one block), keeps
// the best and refits, in a single launch.  The arithmetic is the three-kernel
// path's, so every output is bitwise the same; these frames are bound by
// launch latency, and one launch replaces three.  A workgroup reads back only
// points it staged itself, after a workgroup barrier (its waves share the
// compute unit's L1, which its own stores keep current).
__global__ __launch_bounds__(kScoreBlock) __attribute__((amdgpu_waves_per_eu(8))) void small_frame_kernel(
    const float *__restrict__ theta, const float *__restrict__ vd, const int32_t *__restrict__ off,
    int64_t n_points, int32_t n_hyp, uint32_t key0, uint32_t key1, uint32_t cluster_base,
    int64_t point_base, Points pts, float tau,
    float2 *__restrict__ cs32, float *__restrict__ v32, float2 *__restrict__ cslo,
    unsigned long long *__restrict__ best_key, Outputs o) {
    __shared__ float4 s_hyp[kScoreBlock / 2];
    __shared__ unsigned long long s_key[kScoreBlock / kWave];
    __shared__ double s_sum[kRefitBlock / kWave][5];
    __shared__ int s_cnt[kRefitBlock / kWave][2];
    __shared__ LaneShared s_lanes;
    __shared__ TailShared s_tail;
    const int64_t k = blockIdx.x;
    const Span sp = cluster_span(off, k, n_points, point_base);
    for (int64_t p = sp.lo + threadIdx.x; p < sp.lo + sp.n; p += kScoreBlock)
        stage_point(theta, vd, p, cs32, v32, cslo);
    if (threadIdx.x == 0) best_key[k] = 0;
    __syncthreads();
    ClusterId id;
    id.out = k;
    id.local = cluster_base + (uint32_t)k;
    id.key0 = key0;
    id.key1 = key1;
    // The workgroup's own block key is the cluster's best (one block per
    // cluster); the per-wave keys are still in LDS after the scoring's barrier.
    const bool lanes = sp.ok && sp.n >= 2 && sp.n <= kSingleLanesMax;  // block-uniform
    if (lanes)
        score_block_lanes(sp, id, 0, n_hyp, pts, tau, s_lanes, best_key, o.hyp_counts);
    else
        score_block<false>(sp, id, 0, n_hyp, pts, tau, kRowsMax, s_hyp, s_key, s_tail,
                           best_key, o.hyp_counts);
    const unsigned long long *keys = lanes ? s_lanes.key : s_key;
    unsigned long long best = 0;
#pragma unroll
    for (int w = 0; w < kScoreBlock / kWave; ++w) best = keys[w] > best ? keys[w] : best;
    refit_block(sp, id, uniform_u64(best), pts, tau, o, s_sum, s_cnt);
}

struct Batch {
    const int32_t *frame_off;  // [n_frames + 1]
    const uint64_t *seeds;     // [n_frames], device
    int64_t n_frames;
};

// Register rows per pass for each cluster-size bucket: bucket 0 holds n < 64,
// bucket b holds n in [32 * 2^b, 64 * 2^b), the last bucket everything larger.
struct Tuning {
    int32_t rows[RV_TUNE_BUCKETS];
    int32_t fp16_min;   // clusters of at least this many points use the FP16 form; 0: none
    int32_t lanes_max;  // clusters of at most this many points score with lanes = hypotheses
};

// Scoring form of a cluster (ItemDesc::form).
enum : int16_t { kFormRows = 0, kFormFp16 = 1, kFormLanes = 2 };

// Everything the scoring and refit workgroups need about one cluster, at its
// position in the dispatch order: one 32-byte load instead of a chain of
// dependent loads (order, offsets, frame, seed).
struct alignas(32) ItemDesc {
    int32_t lo, n;         // point span; n = 0 when the offsets are bad
    int32_t out;           // output index (the cluster's index in the batch)
    uint32_t local;        // counter word 1: index within its frame
    uint32_t key0, key1;   // Philox key: its frame's seed
    int32_t ok;            // offsets valid
    int16_t rows;          // register rows per pass for its size
    int16_t form;          // kFormRows, kFormFp16 or kFormLanes
};

constexpr int kQueueStride = 32;  // 64-bit counters: 256 bytes between queues

__device__ __forceinline__ int size_bucket(int64_t n) {
    int b = 0;
    while (b < RV_TUNE_BUCKETS - 1 && n >= ((int64_t)64 << b)) ++b;
    return b;
}

// Frame of cluster k: the last f with frame_off[f] <= k (binary search; stays
// inside [0, n_frames) whatever the offsets hold).
__device__ __forceinline__ int64_t frame_of_cluster(const int32_t *__restrict__ fo,
                                                    int64_t n_frames, int64_t k) {
    int64_t lo = 0, hi = n_frames;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (fo[mid] <= k)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ Span desc_span(const ItemDesc &d) {
    Span sp;
    sp.lo = d.lo;
    sp.n = d.n;
    sp.ok = d.ok != 0;
    return sp;
}

__device__ __forceinline__ ClusterId desc_id(const ItemDesc &d) {
    ClusterId id;
    id.out = d.out;
    id.local = d.local;
    id.key0 = d.key0;
    id.key1 = d.key1;
    return id;
}

// Clears the size-class histogram and the work queues.
__global__ __launch_bounds__(kSizeClasses) void batch_init_kernel(
    uint32_t *__restrict__ hist, unsigned long long *__restrict__ queues) {
    hist[threadIdx.x] = 0;
    if (threadIdx.x < kXcds) queues[threadIdx.x * kQueueStride] = 0;
}

// One thread per point: staging as in prep_kernel.  One thread per cluster:
// clear its best key and count it in its size class (per-block LDS histogram,
// one global atomic per class and block).
__global__ __launch_bounds__(kPrepBlock) void batch_prep_kernel(
    const float *__restrict__ theta, const float *__restrict__ vd, int64_t n_points,
    float2 *__restrict__ cs32, float *__restrict__ v32, float2 *__restrict__ cslo,
    uint32_t *__restrict__ bits, int64_t n_words, const int32_t *__restrict__ off,
    int64_t n_clusters, unsigned long long *__restrict__ best_key, uint32_t *__restrict__ hist) {
    __shared__ uint32_t local[kSizeClasses];
    for (int c = threadIdx.x; c < kSizeClasses; c += kPrepBlock) local[c] = 0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * kPrepBlock + threadIdx.x;
    if (p < n_points) stage_point(theta, vd, p, cs32, v32, cslo);
    if (bits != nullptr && p < n_words) bits[p] = 0u;
    if (p < n_clusters) {
        best_key[p] = 0;
        atomicAdd(&local[size_class(cluster_span(off, p, n_points).n)], 1u);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kSizeClasses; c += kPrepBlock)
        if (local[c] != 0) atomicAdd(&hist[c], local[c]);
}

// Start of each size class in the dispatch order (largest class first).
__global__ __launch_bounds__(kWave) void batch_scan_kernel(uint32_t *__restrict__ hist,
                                                           int64_t *__restrict__ n_big) {
    // One wave, two classes per lane (position q in the dispatch order is class
    // kSizeClasses - 1 - q); each lane reads and rewrites only its own two.
    const int lane = threadIdx.x;
    const int c_hi = kSizeClasses - 1 - 2 * lane, c_lo = c_hi - 1;
    const uint32_t a = hist[c_hi], b = hist[c_lo];
    const uint32_t excl = wave_exclusive_sum(a + b, lane);
    hist[c_hi] = excl;
    hist[c_lo] = excl + a;
    // Clusters refit by a whole workgroup: classes kRefitBigClass and up.
    if (c_hi == kRefitBigClass) *n_big = excl + a;
    if (c_lo == kRefitBigClass) *n_big = excl + a + b;
}

// Places every cluster in the dispatch order (one global atomic per class and
// block reserves a range, LDS atomics rank the block's clusters inside it) and
// writes its descriptor there.
__global__ __launch_bounds__(kPrepBlock) void batch_scatter_kernel(
    const int32_t *__restrict__ off, int64_t n_clusters, int64_t n_points, Batch bt, Tuning tune,
    uint32_t *__restrict__ start, ItemDesc *__restrict__ desc) {
    __shared__ uint32_t count[kSizeClasses];
    __shared__ uint32_t base[kSizeClasses];
    for (int c = threadIdx.x; c < kSizeClasses; c += kPrepBlock) count[c] = 0;
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * kPrepBlock + threadIdx.x;
    int cls = -1;
    uint32_t rank = 0;
    Span sp;
    if (k < n_clusters) {
        sp = cluster_span(off, k, n_points);
        cls = size_class(sp.n);
        rank = atomicAdd(&count[cls], 1u);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kSizeClasses; c += kPrepBlock)
        base[c] = count[c] != 0 ? atomicAdd(&start[c], count[c]) : 0u;
    __syncthreads();
    if (cls < 0) return;
    const int64_t f = frame_of_cluster(bt.frame_off, bt.n_frames, k);
    const uint64_t seed = bt.seeds[f];
    ItemDesc d;
    d.lo = (int32_t)sp.lo;
    d.n = (int32_t)sp.n;
    d.out = (int32_t)k;
    d.local = (uint32_t)(k - bt.frame_off[f]);
    d.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
    d.key1 = (uint32_t)(seed >> 32);
    d.ok = sp.ok ? 1 : 0;
    d.rows = (int16_t)tune.rows[size_bucket(sp.n)];
    d.form = kFormRows;
    if (sp.ok && sp.n >= 2 && sp.n <= tune.lanes_max)
        d.form = kFormLanes;
    else if (tune.fp16_min > 0 && sp.ok && sp.n >= 2 && sp.n >= tune.fp16_min)
        d.form = kFormFp16;
    desc[base[cls] + rank] = d;
}

// Persistent scoring over the per-XCD queues (see above).  Every branch that
// leads to or around a barrier in the item loop is taken on a wave-uniform
// value (wave index, item read back with readfirstlane): with a per-lane guard
// such as threadIdx.x == 0 the compiler may thread that guard across the
// loop's back edge into a lane-masked inner loop that lane 0 leaves to fetch
// the next item while lanes 1..63 wait on the old one.  The float32-only
// instantiation runs eight waves per SIMD (a few reloads of loop state per pass
// of rows, measured 1-2 % faster than seven waves without them); kFp16: the
// instantiation that also runs FP16-form items (launched only when the tuning
// enables that form, so that the float32-only kernel keeps its own register
// allocation), at seven waves per SIMD.
template <bool kFp16>
__global__ __launch_bounds__(kScoreBlock) __attribute__((amdgpu_waves_per_eu(kFp16 ? 7 : 8))) void batch_score_kernel(
    const ItemDesc *__restrict__ desc, int64_t n_clusters, int32_t n_hyp,
    int32_t blocks_per_cluster, Points pts, float tau, unsigned long long *__restrict__ queues,
    unsigned long long *__restrict__ best_key, int32_t *__restrict__ hyp_counts) {
    __shared__ float4 s_hyp[kScoreBlock / 2];
    __shared__ unsigned long long s_key[kScoreBlock / kWave];
    __shared__ unsigned long long s_item;
    __shared__ Fp16Shared s_fp16;  // unreferenced, so not allocated, when !kFp16
    __shared__ LaneShared s_lanes;
    __shared__ TailShared s_tail;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const uint32_t home = blockIdx.x % kXcds;
    const uint64_t bpc = (uint64_t)blocks_per_cluster;
    for (uint32_t step = 0; step < kXcds; ++step) {
        const uint32_t q = (home + step) % kXcds;
        const int64_t clusters_q = n_clusters > (int64_t)q ? (n_clusters - q + kXcds - 1) / kXcds : 0;
        const unsigned long long total = (unsigned long long)clusters_q * bpc;
        for (;;) {
            if (wave == 0) {
                unsigned long long got = 0;
                if (lane == 0) got = atomicAdd(&queues[q * kQueueStride], 1ull);
                s_item = uniform_u64(got);  // the same value from every lane of wave 0
            }
            __syncthreads();
            const unsigned long long item = uniform_u64(s_item);
            __syncthreads();
            if (item >= total) break;
            const int64_t j = (int64_t)q + (int64_t)kXcds * (int64_t)(item / bpc);
            const int b = (int)(item % bpc);
            const ItemDesc d = desc[j];
            if (d.form == kFormLanes) {
                score_block_lanes(desc_span(d), desc_id(d), b, n_hyp, pts, tau, s_lanes, best_key,
                                  hyp_counts);
                continue;
            }
            if constexpr (kFp16) {
                if (d.form == kFormFp16) {
                    score_block_fp16(desc_span(d), desc_id(d), b, n_hyp, pts, tau, d.rows, s_fp16,
                                     best_key, hyp_counts);
                    continue;
                }
            }
            score_block<true>(desc_span(d), desc_id(d), b, n_hyp, pts, tau, d.rows, s_hyp, s_key,
                              s_tail, best_key, hyp_counts);
        }
    }
}

// Cluster at dispatch position j of a batch (its descriptor).
struct BatchClusterAt {
    const ItemDesc *desc;
    const unsigned long long *best_key;
    __device__ Span span(int64_t j) const { return desc_span(desc[j]); }
    __device__ ClusterId id(int64_t j) const { return desc_id(desc[j]); }
    __device__ unsigned long long best(int64_t j) const { return best_key[desc[j].out]; }
};

__global__ __launch_bounds__(kRefitBlock) void batch_refit_kernel(
    const ItemDesc *__restrict__ desc, int64_t n_clusters, const int64_t *__restrict__ n_big,
    Points pts, const unsigned long long *__restrict__ best_key, float tau, Outputs o) {
    __shared__ double s_sum[kRefitBlock / kWave][5];
    __shared__ int s_cnt[kRefitBlock / kWave][2];
    const BatchClusterAt at = {desc, best_key};
    refit_planned(n_clusters, n_big, at, pts, tau, o, s_sum, s_cnt);
}

__global__ __launch_bounds__(kPrepBlock) void philox_kernel(const uint32_t *__restrict__ ctr,
                                                        const uint32_t *__restrict__ key,
                                                        uint32_t *__restrict__ out,
                                                        int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * kPrepBlock + threadIdx.x;
    if (t >= n) return;
    const uint4 r = philox4x32_10(
        make_uint4(ctr[4 * t], ctr[4 * t + 1], ctr[4 * t + 2], ctr[4 * t + 3]), key[2 * t],
        key[2 * t + 1]);
    out[4 * t] = r.x;
    out[4 * t + 1] = r.y;
    out[4 * t + 2] = r.z;
    out[4 * t + 3] = r.w;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

using rv_internal::fail;
using rv_internal::g_error;
using rv_internal::g_free;
using rv_internal::g_pending;
using rv_internal::g_timing;
using rv_internal::g_timing_mutex;
using rv_internal::keep_timed_call;
using rv_internal::kStages;
using rv_internal::take_timed_call;
using rv_internal::TimedCall;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t cs32, v32, cslo, order, best_key, n_big, total;
};

Layout make_layout(int64_t n_clusters, int64_t n_points) {
    Layout L;
    const size_t np = (size_t)n_points;
    size_t at = 0;
    L.cs32 = at; at = align_up(at + np * sizeof(float2));
    L.v32 = at; at = align_up(at + np * sizeof(float));
    L.cslo = at; at = align_up(at + np * sizeof(float2));
    L.order = at; at = align_up(at + (size_t)n_clusters * sizeof(int32_t));
    L.best_key = at; at = align_up(at + (size_t)n_clusters * sizeof(unsigned long long));
    L.n_big = at; at = align_up(at + sizeof(int64_t));
    L.total = at;
    return L;
}

// Stage timing: events recorded around each kernel of each call.


struct BatchLayout {
    size_t cs32, v32, cslo, desc, best_key, hist, queues, n_big, total;
};

BatchLayout make_batch_layout(int64_t n_clusters, int64_t n_points) {
    BatchLayout L;
    const size_t np = (size_t)n_points, nc = (size_t)n_clusters;
    size_t at = 0;
    L.cs32 = at; at = align_up(at + np * sizeof(float2));
    L.v32 = at; at = align_up(at + np * sizeof(float));
    L.cslo = at; at = align_up(at + np * sizeof(float2));
    L.desc = at; at = align_up(at + nc * sizeof(ItemDesc));
    L.best_key = at; at = align_up(at + nc * sizeof(unsigned long long));
    L.hist = at; at = align_up(at + kSizeClasses * sizeof(uint32_t));
    L.queues = at; at = align_up(at + kXcds * kQueueStride * sizeof(unsigned long long));
    L.n_big = at; at = align_up(at + sizeof(int64_t));
    L.total = at;
    return L;
}

struct BatchArgs {
    const float *theta, *vd;
    const int32_t *off, *frame_off;
    const uint64_t *seeds;
    int64_t n_frames, n_clusters, n_points;
    int32_t n_hyp;
    float tau;
    Outputs o;
    rv_tuning_t tuning;
    void *workspace;
    size_t workspace_bytes;
};

int check_batch(const BatchArgs &a) {
    if (a.n_frames < 1 || a.n_frames > (int64_t)INT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "n_frames must be in [1, 2^31 - 1]");
    if (a.n_clusters < 0 || a.n_clusters > (int64_t)INT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "n_clusters must be in [0, 2^31 - 1]");
    if (a.n_points < 0 || a.n_points > INT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "n_points must be in [0, 2^31 - 1]");
    if (a.n_hyp < 1 || a.n_hyp > RV_MAX_HYP)
        return fail(RV_ERR_INVALID_ARG, "n_hyp must be in [1, %d]", RV_MAX_HYP);
    if (!(a.tau > 0.0f) || !isfinite(a.tau))
        return fail(RV_ERR_INVALID_ARG, "tau must be finite and > 0");
    if (a.off == nullptr || a.frame_off == nullptr || a.seeds == nullptr)
        return fail(RV_ERR_INVALID_ARG, "cluster_offsets, frame_offsets or seeds is NULL");
    if (a.n_points > 0 && (a.theta == nullptr || a.vd == nullptr))
        return fail(RV_ERR_INVALID_ARG, "theta or vd is NULL");
    if (a.n_clusters > 0 && (a.o.vx == nullptr || a.o.vy == nullptr || a.o.heading == nullptr ||
                             a.o.n_inliers == nullptr || a.o.status == nullptr))
        return fail(RV_ERR_INVALID_ARG, "a required output is NULL");
    for (int b = 0; b < RV_TUNE_BUCKETS; ++b)
        if (a.tuning.rows_max[b] < 1 || a.tuning.rows_max[b] > kRowsMax)
            return fail(RV_ERR_INVALID_ARG, "tuning.rows_max must be in [1, %d]", kRowsMax);
    if (a.tuning.blocks_per_cu < 0 || a.tuning.blocks_per_cu > 64)
        return fail(RV_ERR_INVALID_ARG, "tuning.blocks_per_cu must be in [0, 64]");
    if (a.tuning.fp16_min_points < 0)
        return fail(RV_ERR_INVALID_ARG, "tuning.fp16_min_points must be >= 0");
    if (a.tuning.lanes_max_points < 0 || a.tuning.lanes_max_points > kLaneTile)
        return fail(RV_ERR_INVALID_ARG, "tuning.lanes_max_points must be in [0, %d]", kLaneTile);
    const BatchLayout L = make_batch_layout(a.n_clusters, a.n_points);
    if (a.workspace == nullptr || a.workspace_bytes < L.total)
        return fail(RV_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                    a.workspace == nullptr ? (size_t)0 : a.workspace_bytes);
    if (((uintptr_t)a.workspace % kAlign) != 0)
        return fail(RV_ERR_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    return RV_OK;
}

int64_t batch_blocks_per_cluster(const BatchArgs &a) {
    return ((int64_t)a.n_hyp + kScoreBlock - 1) / kScoreBlock;
}

// Compute units of the current device, queried once per device (a launch that
// is being captured into a graph only reads the cache, filled by the caller's
// earlier call).
int device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int cus = cache[dev].load(std::memory_order_relaxed);
    if (cus > 0) return cus;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cache[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

// The refit kernel over planned positions; n_big (device, nullable) is the
// ordering pass's count of big clusters.
void launch_refit(bool batch, const int32_t *off, const int32_t *order, const ItemDesc *desc,
                  int64_t n_clusters, const int64_t *n_big, int64_t n_points, uint32_t key0,
                  uint32_t key1, uint32_t cluster_base, int64_t point_base, const Points &pts,
                  const unsigned long long *best_key, float tau, const Outputs &o,
                  hipStream_t st) {
    if (batch)
        hipLaunchKernelGGL(batch_refit_kernel, dim3((unsigned)n_clusters), dim3(kRefitBlock), 0, st,
                           desc, n_clusters, n_big, pts, best_key, tau, o);
    else
        hipLaunchKernelGGL(refit_kernel, dim3((unsigned)n_clusters), dim3(kRefitBlock), 0, st, off,
                           order, n_clusters, n_big, n_points, key0, key1, cluster_base,
                           point_base, pts, best_key, tau, o);
}

// Persistent grid of the batched scoring kernel on the current device.
int persistent_blocks(int blocks_per_cu, bool fp16, int64_t items, unsigned *grid) {
    int fit = 0;
    const int cus = device_cus();
    const hipError_t e =
        fp16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, batch_score_kernel<true>, kScoreBlock, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, batch_score_kernel<false>, kScoreBlock, 0);
    if (cus <= 0 || e != hipSuccess)
        return fail(RV_ERR_HIP, "device query failed");
    int per_cu = blocks_per_cu > 0 && blocks_per_cu < fit ? blocks_per_cu : fit;
    if (per_cu < 1) per_cu = 1;
    int64_t g = (int64_t)cus * per_cu;
    if (g > items) g = items;
    *grid = (unsigned)(g > 0 ? g : 1);
    return RV_OK;
}

// The launch sequence of the batched form (argument checks and the persistent
// grid size done by the caller, so that no device query falls inside a capture).
int launch_batch(const BatchArgs &a, unsigned grid, hipStream_t st, bool allow_timing) {
    if (a.n_clusters == 0) return RV_OK;
    const BatchLayout L = make_batch_layout(a.n_clusters, a.n_points);
    char *ws = (char *)a.workspace;
    float2 *cs32 = (float2 *)(ws + L.cs32);
    float *v32 = (float *)(ws + L.v32);
    float2 *cslo = (float2 *)(ws + L.cslo);
    ItemDesc *desc = (ItemDesc *)(ws + L.desc);
    unsigned long long *best_key = (unsigned long long *)(ws + L.best_key);
    uint32_t *hist = (uint32_t *)(ws + L.hist);
    unsigned long long *queues = (unsigned long long *)(ws + L.queues);
    int64_t *n_big = (int64_t *)(ws + L.n_big);
    Points pts;
    pts.cs32 = cs32;
    pts.v32 = v32;
    pts.cslo = cslo;
    pts.theta = a.theta;
    Batch bt;
    bt.frame_off = a.frame_off;
    bt.seeds = a.seeds;
    bt.n_frames = a.n_frames;
    Tuning tune;
    for (int b = 0; b < RV_TUNE_BUCKETS; ++b) tune.rows[b] = a.tuning.rows_max[b];
    tune.fp16_min = a.tuning.fp16_min_points;
    tune.lanes_max = a.tuning.lanes_max_points;
    const int64_t bpc = batch_blocks_per_cluster(a);
    const int64_t n_words = a.o.bits != nullptr ? (a.n_points + 31) / 32 : 0;
    int64_t prep_items = a.n_points > n_words ? a.n_points : n_words;
    prep_items = prep_items > a.n_clusters ? prep_items : a.n_clusters;

    TimedCall tc;
    const bool timed = allow_timing && take_timed_call(tc);
    if (timed) (void)hipEventRecord(tc.ev[0], st);
    hipLaunchKernelGGL(batch_init_kernel, dim3(1), dim3(kSizeClasses), 0, st, hist, queues);
    hipLaunchKernelGGL(batch_prep_kernel, dim3((unsigned)((prep_items + kPrepBlock - 1) / kPrepBlock)),
                       dim3(kPrepBlock), 0, st, a.theta, a.vd, a.n_points, cs32, v32, cslo,
                       a.o.bits, n_words, a.off, a.n_clusters, best_key, hist);
    hipLaunchKernelGGL(batch_scan_kernel, dim3(1), dim3(64), 0, st, hist, n_big);
    hipLaunchKernelGGL(batch_scatter_kernel,
                       dim3((unsigned)((a.n_clusters + kPrepBlock - 1) / kPrepBlock)),
                       dim3(kPrepBlock), 0, st, a.off, a.n_clusters, a.n_points, bt, tune, hist, desc);
    if (timed) (void)hipEventRecord(tc.ev[1], st);
    if (a.tuning.fp16_min_points > 0)
        hipLaunchKernelGGL(batch_score_kernel<true>, dim3(grid), dim3(kScoreBlock), 0, st,
                           (const ItemDesc *)desc, a.n_clusters, a.n_hyp, (int32_t)bpc, pts, a.tau,
                           queues, best_key, a.o.hyp_counts);
    else
        hipLaunchKernelGGL(batch_score_kernel<false>, dim3(grid), dim3(kScoreBlock), 0, st,
                           (const ItemDesc *)desc, a.n_clusters, a.n_hyp, (int32_t)bpc, pts, a.tau,
                           queues, best_key, a.o.hyp_counts);
    if (timed) (void)hipEventRecord(tc.ev[2], st);
    launch_refit(true, nullptr, nullptr, (const ItemDesc *)desc, a.n_clusters, n_big, a.n_points,
                 0, 0, 0, 0, pts, best_key, a.tau, a.o, st);
    if (timed) {
        (void)hipEventRecord(tc.ev[3], st);
        keep_timed_call(tc);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return RV_OK;
}

// Frames small enough that launch latency dominates take the one-launch path
// (small_frame_kernel): at most 256 hypotheses (one scoring block per cluster,
// as on the three-kernel path), at most 65,536 points (each workgroup stages
// its own cluster) and no frame-wide inlier mask (its words are shared by
// neighbouring clusters and are cleared by the staging kernel).
constexpr int64_t kSmallFrameMaxPoints = 1 << 16;
constexpr int64_t kSmallFrameMaxClusters = 1 << 16;

bool use_small_frame_path(int64_t n_clusters, int64_t n_points, int32_t n_hyp,
                          const uint32_t *inlier_bits) {
    return inlier_bits == nullptr && n_hyp <= kScoreBlock && n_points <= kSmallFrameMaxPoints &&
           n_clusters <= kSmallFrameMaxClusters;
}

BatchArgs make_batch_args(const float *theta, const float *vd, const int32_t *cluster_offsets,
                          const int32_t *frame_offsets, const uint64_t *seeds, int64_t n_frames,
                          int64_t n_clusters, int64_t n_points, int32_t n_hyp, float tau,
                          float *vx, float *vy, float *heading, int32_t *n_inliers,
                          uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                          int32_t *hyp_counts, int32_t *best_hyp, const rv_tuning_t *tuning,
                          void *workspace, size_t workspace_bytes) {
    BatchArgs a;
    a.theta = theta;
    a.vd = vd;
    a.off = cluster_offsets;
    a.frame_off = frame_offsets;
    a.seeds = seeds;
    a.n_frames = n_frames;
    a.n_clusters = n_clusters;
    a.n_points = n_points;
    a.n_hyp = n_hyp;
    a.tau = tau;
    a.o.vx = vx;
    a.o.vy = vy;
    a.o.heading = heading;
    a.o.n_inliers = n_inliers;
    a.o.status = status;
    a.o.n_near = n_near_tau;
    a.o.best = best_hyp;
    a.o.hyp_counts = hyp_counts;
    a.o.bits = inlier_bits;
    if (tuning != nullptr)
        a.tuning = *tuning;
    else
        rv_tuning_default(&a.tuning);
    a.workspace = workspace;
    a.workspace_bytes = workspace_bytes;
    return a;
}

// rv_estimate_velocity's checks and launches; allow_timing: record stage events
// when rv_stage_timing is on (the allocation-free entry point never does, since
// a first event set is created on demand).
int estimate_frame(const float *theta, const float *vd, const int32_t *cluster_offsets,
                   int64_t n_clusters, int64_t n_points, int32_t n_hyp, float tau, uint64_t seed,
                   float *vx, float *vy, float *heading, int32_t *n_inliers, uint8_t *status,
                   int32_t *n_near_tau, uint32_t *inlier_bits, int32_t *hyp_counts,
                   int32_t *best_hyp, void *workspace, size_t workspace_bytes, void *stream,
                   uint32_t first_cluster, int64_t first_point, bool allow_timing) {
    if (n_clusters < 0) return fail(RV_ERR_INVALID_ARG, "n_clusters < 0");
    if ((uint64_t)first_cluster + (uint64_t)n_clusters > ((uint64_t)1 << 32))
        return fail(RV_ERR_INVALID_ARG, "first_cluster + n_clusters exceeds 2^32");
    if (n_points < 0 || n_points > INT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "n_points must be in [0, 2^31 - 1]");
    if (n_hyp < 1 || n_hyp > RV_MAX_HYP)
        return fail(RV_ERR_INVALID_ARG, "n_hyp must be in [1, %d]", RV_MAX_HYP);
    if (!(tau > 0.0f) || !isfinite(tau))
        return fail(RV_ERR_INVALID_ARG, "tau must be finite and > 0");
    if (cluster_offsets == nullptr) return fail(RV_ERR_INVALID_ARG, "cluster_offsets is NULL");
    if (n_points > 0 && (theta == nullptr || vd == nullptr))
        return fail(RV_ERR_INVALID_ARG, "theta or vd is NULL");
    if (n_clusters > 0 &&
        (vx == nullptr || vy == nullptr || heading == nullptr || n_inliers == nullptr ||
         status == nullptr))
        return fail(RV_ERR_INVALID_ARG, "a required output is NULL");
    const int64_t blocks_per_cluster = ((int64_t)n_hyp + kScoreBlock - 1) / kScoreBlock;
    const int64_t clusters_xcd = (n_clusters + kXcds - 1) / kXcds * kXcds;
    if (clusters_xcd > (int64_t)INT32_MAX / blocks_per_cluster)
        return fail(RV_ERR_INVALID_ARG, "n_clusters * ceil(n_hyp / 256) exceeds 2^31 - 1");
    const Layout L = make_layout(n_clusters, n_points);
    if (workspace == nullptr || workspace_bytes < L.total)
        return fail(RV_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                    workspace == nullptr ? (size_t)0 : workspace_bytes);
    if (((uintptr_t)workspace % kAlign) != 0)
        return fail(RV_ERR_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    if (n_clusters == 0) return RV_OK;

    char *ws = (char *)workspace;
    float2 *cs32 = (float2 *)(ws + L.cs32);
    float *v32 = (float *)(ws + L.v32);
    float2 *cslo = (float2 *)(ws + L.cslo);
    Points pts;
    pts.cs32 = cs32;
    pts.v32 = v32;
    pts.cslo = cslo;
    pts.theta = theta;
    int32_t *order = n_clusters <= kPlanMaxClusters ? (int32_t *)(ws + L.order) : nullptr;
    int64_t *n_big = (int64_t *)(ws + L.n_big);
    unsigned long long *best_key = (unsigned long long *)(ws + L.best_key);
    const uint32_t key0 = (uint32_t)(seed & 0xFFFFFFFFu), key1 = (uint32_t)(seed >> 32);
    const int64_t n_words = inlier_bits != nullptr ? (n_points + 31) / 32 : 0;
    hipStream_t st = (hipStream_t)stream;

    Outputs o;
    o.vx = vx;
    o.vy = vy;
    o.heading = heading;
    o.n_inliers = n_inliers;
    o.status = status;
    o.n_near = n_near_tau;
    o.best = best_hyp;
    o.hyp_counts = hyp_counts;
    o.bits = inlier_bits;

    TimedCall tc;
    const bool timed = allow_timing && take_timed_call(tc);
    if (timed) (void)hipEventRecord(tc.ev[0], st);
    if (use_small_frame_path(n_clusters, n_points, n_hyp, inlier_bits)) {
        // One launch; its time counts as the scoring stage.
        if (timed) (void)hipEventRecord(tc.ev[1], st);
        hipLaunchKernelGGL(small_frame_kernel, dim3((unsigned)n_clusters), dim3(kScoreBlock), 0, st,
                           theta, vd, cluster_offsets, n_points, n_hyp, key0, key1, first_cluster,
                           first_point, pts, tau, cs32, v32, cslo, best_key, o);
        if (timed) {
            (void)hipEventRecord(tc.ev[2], st);
            (void)hipEventRecord(tc.ev[3], st);
            keep_timed_call(tc);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(RV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
        return RV_OK;
    }
    int64_t prep_items = n_points > n_words ? n_points : n_words;
    prep_items = prep_items > n_clusters ? prep_items : n_clusters;
    const int64_t prep_blocks = (prep_items + kPrepBlock - 1) / kPrepBlock + 1;  // + planner
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)prep_blocks), dim3(kPrepBlock), 0, st, theta,
                       vd, n_points, cs32, v32, cslo, inlier_bits, n_words, cluster_offsets,
                       first_point, n_clusters, order, n_big, best_key);
    if (timed) (void)hipEventRecord(tc.ev[1], st);
    hipLaunchKernelGGL(score_kernel, dim3((unsigned)(clusters_xcd * blocks_per_cluster)),
                       dim3(kScoreBlock), 0, st, cluster_offsets, (const int32_t *)order,
                       n_clusters, n_points, n_hyp, (int32_t)blocks_per_cluster, key0, key1,
                       first_cluster, first_point, pts, tau, best_key, hyp_counts);
    if (timed) (void)hipEventRecord(tc.ev[2], st);
    launch_refit(false, cluster_offsets, order, nullptr, n_clusters,
                 order != nullptr ? (const int64_t *)n_big : nullptr, n_points, key0, key1,
                 first_cluster, first_point, pts, best_key, tau, o, st);
    if (timed) {
        (void)hipEventRecord(tc.ev[3], st);
        keep_timed_call(tc);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return RV_OK;
}

// ---- Allocation-free single-frame entry point ------------------------------
//
// rv_estimate_velocity_noalloc keeps its workspace in `scratch`, a device array
// of RV_NOALLOC_SCRATCH_BYTES that each GPU holds from the load of this code
// object on it until the process ends.  In host code the array's name denotes a host-side
// stand-in, not device memory: host code only passes on the address that
// hipGetSymbolAddress returns for the current device, looked up once per device
// and kept in g_scratch.  Every kernel writes the parts of the workspace it
// reads before reading them (staged points, dispatch order, best keys), so the
// contents a previous call left need no clearing.
static __device__ __align__(256) unsigned char scratch[RV_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch[kMaxDevices];

// Device address of `scratch` on the device of `stream` (which must be the
// current device: the symbol is looked up with that device current).
int device_scratch(hipStream_t stream, void **ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(RV_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (stream != nullptr) {
        int sdev = -1;
        e = hipStreamGetDevice(stream, &sdev);
        if (e != hipSuccess)
            return fail(RV_ERR_HIP, "hipStreamGetDevice failed: %s", hipGetErrorString(e));
        if (sdev != dev)
            return fail(RV_ERR_INVALID_ARG,
                        "stream belongs to device %d, the current device is %d", sdev, dev);
    }
    if (dev < 0 || dev >= kMaxDevices)
        return fail(RV_ERR_HIP, "device index %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(RV_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    return RV_OK;
}

// ---- A frame sent and estimated in parts ---------------------------------------
// Events that order a part's estimate after its copy, kept per device and
// reused: a wait enqueued on a stream holds on to the record that precedes it,
// so an event may go back to the pool as soon as its wait is enqueued.
std::mutex g_event_mutex;
std::vector<hipEvent_t> g_events[kMaxDevices];

int take_events(int dev, int n, hipEvent_t *ev) {
    std::lock_guard<std::mutex> lock(g_event_mutex);
    std::vector<hipEvent_t> &pool = g_events[dev];
    for (int i = 0; i < n; ++i) {
        if (pool.empty()) {
            const hipError_t e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
            if (e != hipSuccess) {
                for (int j = 0; j < i; ++j) pool.push_back(ev[j]);
                return fail(RV_ERR_HIP, "hipEventCreateWithFlags failed: %s",
                            hipGetErrorString(e));
            }
        } else {
            ev[i] = pool.back();
            pool.pop_back();
        }
    }
    return RV_OK;
}

void give_events(int dev, int n, const hipEvent_t *ev) {
    std::lock_guard<std::mutex> lock(g_event_mutex);
    for (int i = 0; i < n; ++i) g_events[dev].push_back(ev[i]);
}

// Clusters [cut[j], cut[j+1]) form part j.  Part j gets a share of the points
// proportional to n_parts - j (shares P, P - 1, ..., 1 out of P (P + 1) / 2):
// only the last part's estimate is not hidden behind a later copy, so the
// parts shrink toward the end.  The first cluster that starts at or after part
// j's first point starts it (parts without clusters are dropped).  Returns the
// number of parts.
int cut_parts(const int32_t *off, int64_t n_clusters, int64_t n_points, int n_parts,
              int64_t *cut) {
    int m = 0;
    cut[m++] = 0;
    int64_t k = 0;
    const int64_t total = (int64_t)n_parts * (n_parts + 1);
    for (int j = 1; j < n_parts; ++j) {
        const int64_t target = n_points * ((int64_t)j * (2 * n_parts - j + 1)) / total;
        while (k < n_clusters && off[k] < target) ++k;
        if (k > cut[m - 1] && k < n_clusters) cut[m++] = k;
    }
    cut[m++] = n_clusters;  // n_clusters > 0: every cut above is below it
    return m - 1;
}

int estimate_pipelined(const float *theta_host, const float *vd_host,
                       const int32_t *offsets_host, int64_t n_clusters, int64_t n_points,
                       int32_t n_parts, int32_t n_hyp, float tau, uint64_t seed, float *theta_dev,
                       float *vd_dev, int32_t *offsets_dev, float *vx, float *vy, float *heading,
                       int32_t *n_inliers, uint8_t *status, int32_t *n_near_tau,
                       int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                       size_t workspace_bytes, hipStream_t st, hipStream_t copy_st) {
    if (n_clusters < 0 || n_points < 0 || n_points > INT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "sizes out of range");
    if (n_parts < 1 || n_parts > RV_MAX_PARTS)
        return fail(RV_ERR_INVALID_ARG, "n_parts must be in [1, %d]", RV_MAX_PARTS);
    if (offsets_host == nullptr || offsets_dev == nullptr)
        return fail(RV_ERR_INVALID_ARG, "offsets pointers are NULL");
    if (n_points > 0 && (theta_host == nullptr || vd_host == nullptr || theta_dev == nullptr ||
                         vd_dev == nullptr))
        return fail(RV_ERR_INVALID_ARG, "theta or vd pointers are NULL");
    // The host reads the offsets to cut the frame and to size the copies, so
    // they must describe the frame exactly.
    if (offsets_host[0] != 0 || offsets_host[n_clusters] != n_points)
        return fail(RV_ERR_INVALID_ARG, "offsets must start at 0 and end at n_points");
    for (int64_t k = 0; k < n_clusters; ++k)
        if (offsets_host[k + 1] < offsets_host[k])
            return fail(RV_ERR_INVALID_ARG, "offsets decrease at cluster %lld", (long long)k);
    if (n_clusters == 0) return RV_OK;
    if (workspace_bytes < rv_workspace_bytes(n_clusters, n_points, n_hyp))
        return fail(RV_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", workspace_bytes,
                    rv_workspace_bytes(n_clusters, n_points, n_hyp));
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(RV_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(RV_ERR_HIP, "device index %d outside [0, %d)", dev, kMaxDevices);
    int64_t cut[RV_MAX_PARTS + 1];
    const int m = cut_parts(offsets_host, n_clusters, n_points, n_parts, cut);
    hipEvent_t ev[RV_MAX_PARTS + 1];
    int rc = take_events(dev, m + 1, ev);
    if (rc != RV_OK) return rc;
    // The copies wait for the work already queued on `stream` (a previous
    // call's estimates may still read the same device buffers); then every
    // copy is enqueued first, so that the copy engine never waits for the
    // host, and each part's estimate behind its copy.
    e = hipEventRecord(ev[m], st);
    if (e == hipSuccess) e = hipStreamWaitEvent(copy_st, ev[m], 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(offsets_dev, offsets_host, (size_t)(n_clusters + 1) * sizeof(int32_t),
                           hipMemcpyHostToDevice, copy_st);
    for (int j = 0; j < m && e == hipSuccess; ++j) {
        const int64_t p0 = offsets_host[cut[j]], p1 = offsets_host[cut[j + 1]];
        if (p1 > p0) {
            e = hipMemcpyAsync(theta_dev + p0, theta_host + p0, (size_t)(p1 - p0) * sizeof(float),
                               hipMemcpyHostToDevice, copy_st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(vd_dev + p0, vd_host + p0, (size_t)(p1 - p0) * sizeof(float),
                                   hipMemcpyHostToDevice, copy_st);
        }
        if (e == hipSuccess) e = hipEventRecord(ev[j], copy_st);
    }
    for (int j = 0; j < m && e == hipSuccess && rc == RV_OK; ++j) {
        e = hipStreamWaitEvent(st, ev[j], 0);
        if (e != hipSuccess) break;
        const int64_t c0 = cut[j], c1 = cut[j + 1];
        const int64_t p0 = offsets_host[c0], p1 = offsets_host[c1];
        rc = estimate_frame(theta_dev + p0, vd_dev + p0, offsets_dev + c0, c1 - c0, p1 - p0, n_hyp,
                            tau, seed, vx + c0, vy + c0, heading + c0, n_inliers + c0,
                            status + c0, n_near_tau != nullptr ? n_near_tau + c0 : nullptr,
                            nullptr, hyp_counts != nullptr ? hyp_counts + c0 * n_hyp : nullptr,
                            best_hyp != nullptr ? best_hyp + c0 : nullptr, workspace,
                            workspace_bytes, (void *)st, (uint32_t)c0, p0, false);
    }
    give_events(dev, m + 1, ev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RV_ERR_HIP, "pipelined copy or wait failed: %s", hipGetErrorString(e));
    }
    return rc;
}

}  // namespace

extern "C" {

size_t rv_workspace_bytes(int64_t n_clusters, int64_t n_points, int32_t n_hyp) {
    if (n_clusters < 0 || n_points < 0 || n_hyp < 0) return 0;
    return make_layout(n_clusters, n_points).total;
}

const char *rv_last_error(void) { return g_error; }

int rv_estimate_velocity(const float *theta, const float *vd, const int32_t *cluster_offsets,
                         int64_t n_clusters, int64_t n_points, int32_t n_hyp, float tau,
                         uint64_t seed, float *vx, float *vy, float *heading, int32_t *n_inliers,
                         uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                         int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                         size_t workspace_bytes, void *stream) {
    g_error[0] = '\0';
    return estimate_frame(theta, vd, cluster_offsets, n_clusters, n_points, n_hyp, tau, seed, vx,
                          vy, heading, n_inliers, status, n_near_tau, inlier_bits, hyp_counts,
                          best_hyp, workspace, workspace_bytes, stream, 0u, 0, true);
}

int rv_estimate_velocity_part(const float *theta, const float *vd, const int32_t *cluster_offsets,
                              int64_t n_clusters, int64_t n_points, int64_t first_cluster,
                              int64_t first_point, int32_t n_hyp, float tau, uint64_t seed,
                              float *vx, float *vy, float *heading, int32_t *n_inliers,
                              uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                              int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                              size_t workspace_bytes, void *stream) {
    g_error[0] = '\0';
    if (first_cluster < 0 || first_cluster > (int64_t)UINT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "first_cluster must be in [0, 2^32 - 1]");
    if (first_point < 0 || first_point > INT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "first_point must be in [0, 2^31 - 1]");
    return estimate_frame(theta, vd, cluster_offsets, n_clusters, n_points, n_hyp, tau, seed, vx,
                          vy, heading, n_inliers, status, n_near_tau, inlier_bits, hyp_counts,
                          best_hyp, workspace, workspace_bytes, stream, (uint32_t)first_cluster,
                          first_point, true);
}

int rv_estimate_velocity_pipelined(const float *theta_host, const float *vd_host,
                                   const int32_t *offsets_host, int64_t n_clusters,
                                   int64_t n_points, int32_t n_parts, int32_t n_hyp, float tau,
                                   uint64_t seed, float *theta_dev, float *vd_dev,
                                   int32_t *offsets_dev, float *vx, float *vy, float *heading,
                                   int32_t *n_inliers, uint8_t *status, int32_t *n_near_tau,
                                   int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                                   size_t workspace_bytes, void *stream, void *copy_stream) {
    g_error[0] = '\0';
    return estimate_pipelined(theta_host, vd_host, offsets_host, n_clusters, n_points, n_parts,
                              n_hyp, tau, seed, theta_dev, vd_dev, offsets_dev, vx, vy, heading,
                              n_inliers, status, n_near_tau, hyp_counts, best_hyp, workspace,
                              workspace_bytes, (hipStream_t)stream, (hipStream_t)copy_stream);
}

int rv_estimate_velocity_noalloc(const float *theta, const float *vd,
                                 const int32_t *cluster_offsets, int64_t n_clusters,
                                 int64_t n_points, int32_t n_hyp, float tau, uint64_t seed,
                                 float *vx, float *vy, float *heading, int32_t *n_inliers,
                                 uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                                 int32_t *hyp_counts, int32_t *best_hyp, void *stream) {
    g_error[0] = '\0';
    const size_t need = rv_workspace_bytes(n_clusters, n_points, n_hyp);
    if (need > RV_NOALLOC_SCRATCH_BYTES)
        return fail(RV_ERR_WORKSPACE,
                    "frame of %lld clusters and %lld points needs %zu bytes of workspace; the "
                    "allocation-free entry point holds %zu",
                    (long long)n_clusters, (long long)n_points, need,
                    (size_t)RV_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    if (int rc = device_scratch((hipStream_t)stream, &ws)) return rc;
    return estimate_frame(theta, vd, cluster_offsets, n_clusters, n_points, n_hyp, tau, seed, vx,
                          vy, heading, n_inliers, status, n_near_tau, inlier_bits, hyp_counts,
                          best_hyp, ws, RV_NOALLOC_SCRATCH_BYTES, stream, 0u, 0, false);
}

int rv_stage_timing(int enable) {
    std::lock_guard<std::mutex> lock(g_timing_mutex);
    g_timing = enable != 0;
    return RV_OK;
}

int rv_stage_times(double *ms, int64_t *n_calls) {
    std::vector<TimedCall> calls;
    {
        std::lock_guard<std::mutex> lock(g_timing_mutex);
        calls.swap(g_pending);
    }
    double sum[kStages] = {0.0, 0.0, 0.0};
    int rc = RV_OK;
    for (const TimedCall &tc : calls) {
        if (hipEventSynchronize(tc.ev[kStages]) != hipSuccess) {
            rc = fail(RV_ERR_HIP, "hipEventSynchronize failed");
            continue;
        }
        for (int s = 0; s < kStages; ++s) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, tc.ev[s], tc.ev[s + 1]) != hipSuccess) {
                rc = fail(RV_ERR_HIP, "hipEventElapsedTime failed");
                continue;
            }
            sum[s] += t;
        }
    }
    {
        std::lock_guard<std::mutex> lock(g_timing_mutex);
        g_free.insert(g_free.end(), calls.begin(), calls.end());
    }
    if (ms)
        for (int s = 0; s < kStages; ++s) ms[s] = sum[s];
    if (n_calls) *n_calls = (int64_t)calls.size();
    return rc;
}

int rv_host_device_pointer(const void *host_ptr, void **device_ptr) {
    g_error[0] = '\0';
    if (device_ptr == nullptr) return fail(RV_ERR_INVALID_ARG, "device_ptr is NULL");
    *device_ptr = nullptr;
    if (host_ptr == nullptr) return fail(RV_ERR_INVALID_ARG, "host_ptr is NULL");
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, host_ptr);
    if (e != hipSuccess || attr.type != hipMemoryTypeHost) {
        (void)hipGetLastError();  // a failed query leaves its error behind
        return fail(RV_ERR_INVALID_ARG, "%p is not pinned host memory (hipHostMalloc)", host_ptr);
    }
    void *d = nullptr;
    e = hipHostGetDevicePointer(&d, const_cast<void *>(host_ptr), 0);
    if (e != hipSuccess || d == nullptr) {
        (void)hipGetLastError();
        return fail(RV_ERR_INVALID_ARG, "no device mapping of %p: %s", host_ptr,
                    hipGetErrorString(e));
    }
    *device_ptr = d;
    return RV_OK;
}

int rv_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n,
                     void *stream) {
    g_error[0] = '\0';
    if (n < 0) return fail(RV_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return RV_OK;
    if (ctr == nullptr || key == nullptr || out == nullptr)
        return fail(RV_ERR_INVALID_ARG, "a pointer is NULL");
    const int64_t grid = (n + kPrepBlock - 1) / kPrepBlock;
    if (grid > INT32_MAX) return fail(RV_ERR_INVALID_ARG, "n too large");
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)grid), dim3(kPrepBlock), 0,
                       (hipStream_t)stream, ctr, key, out, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return RV_OK;
}


void rv_tuning_default(rv_tuning_t *t) {
    if (t == nullptr) return;
    for (int b = 0; b < RV_TUNE_BUCKETS; ++b) t->rows_max[b] = kRowsMax;
    t->blocks_per_cu = 0;
    t->fp16_min_points = 0;
    t->lanes_max_points = kDefaultLanesMax;
}

size_t rv_batch_workspace_bytes(int64_t n_frames, int64_t n_clusters, int64_t n_points,
                                int32_t n_hyp) {
    if (n_frames < 1 || n_clusters < 0 || n_points < 0 || n_hyp < 0) return 0;
    return make_batch_layout(n_clusters, n_points).total;
}

int rv_estimate_velocity_batch(const float *theta, const float *vd, const int32_t *cluster_offsets,
                               const int32_t *frame_offsets, const uint64_t *seeds,
                               int64_t n_frames, int64_t n_clusters, int64_t n_points,
                               int32_t n_hyp, float tau, float *vx, float *vy, float *heading,
                               int32_t *n_inliers, uint8_t *status, int32_t *n_near_tau,
                               uint32_t *inlier_bits, int32_t *hyp_counts, int32_t *best_hyp,
                               const rv_tuning_t *tuning, void *workspace,
                               size_t workspace_bytes, void *stream) {
    g_error[0] = '\0';
    const BatchArgs a = make_batch_args(theta, vd, cluster_offsets, frame_offsets, seeds,
                                        n_frames, n_clusters, n_points, n_hyp, tau, vx, vy,
                                        heading, n_inliers, status, n_near_tau, inlier_bits,
                                        hyp_counts, best_hyp, tuning, workspace, workspace_bytes);
    if (int rc = check_batch(a)) return rc;
    unsigned grid = 1;
    if (a.n_clusters > 0)
        if (int rc = persistent_blocks(a.tuning.blocks_per_cu, a.tuning.fp16_min_points > 0,
                                     a.n_clusters * batch_blocks_per_cluster(a), &grid))
            return rc;
    return launch_batch(a, grid, (hipStream_t)stream, true);
}

struct rv_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

int rv_graph_capture_batch(const float *theta, const float *vd, const int32_t *cluster_offsets,
                           const int32_t *frame_offsets, const uint64_t *seeds, int64_t n_frames,
                           int64_t n_clusters, int64_t n_points, int32_t n_hyp, float tau,
                           float *vx, float *vy, float *heading, int32_t *n_inliers,
                           uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                           int32_t *hyp_counts, int32_t *best_hyp, const rv_tuning_t *tuning,
                           void *workspace, size_t workspace_bytes, rv_graph_t **graph) {
    g_error[0] = '\0';
    if (graph == nullptr) return fail(RV_ERR_INVALID_ARG, "graph is NULL");
    *graph = nullptr;
    const BatchArgs a = make_batch_args(theta, vd, cluster_offsets, frame_offsets, seeds,
                                        n_frames, n_clusters, n_points, n_hyp, tau, vx, vy,
                                        heading, n_inliers, status, n_near_tau, inlier_bits,
                                        hyp_counts, best_hyp, tuning, workspace, workspace_bytes);
    if (int rc = check_batch(a)) return rc;
    unsigned grid = 1;
    if (a.n_clusters > 0)
        if (int rc = persistent_blocks(a.tuning.blocks_per_cu, a.tuning.fp16_min_points > 0,
                                     a.n_clusters * batch_blocks_per_cluster(a), &grid))
            return rc;
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        return fail(RV_ERR_HIP, "hipStreamCreate failed");
    rv_graph_t *g = new rv_graph_t;
    g->graph = nullptr;
    g->exec = nullptr;
    int rc = RV_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = fail(RV_ERR_HIP, "hipStreamBeginCapture failed");
    } else {
        rc = launch_batch(a, grid, cap, false);
        const hipError_t e = hipStreamEndCapture(cap, &g->graph);
        if (rc == RV_OK && e != hipSuccess)
            rc = fail(RV_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        if (rc == RV_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
            rc = fail(RV_ERR_HIP, "hipGraphInstantiate failed");
    }
    (void)hipStreamDestroy(cap);
    if (rc != RV_OK) {
        rv_graph_destroy(g);
        return rc;
    }
    *graph = g;
    return RV_OK;
}

int rv_graph_launch(rv_graph_t *graph, void *stream) {
    g_error[0] = '\0';
    if (graph == nullptr || graph->exec == nullptr) return fail(RV_ERR_INVALID_ARG, "graph is NULL");
    const hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(RV_ERR_HIP, "hipGraphLaunch failed: %s", hipGetErrorString(e));
    return RV_OK;
}

void rv_graph_destroy(rv_graph_t *graph) {
    if (graph == nullptr) return;
    if (graph->exec != nullptr) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph != nullptr) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

}  // extern "C"
