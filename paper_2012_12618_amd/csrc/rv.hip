// rv.hip -- gfx950 kernels and host entry points of the per-cluster RANSAC
// velocity and heading estimator declared in include/rv.h.
//
// One call enqueues four kernels on the caller's stream:
//   prep    one thread per point: FP64 sincos of the azimuth; stages float32
//           (cos, sin, v_d) for scoring and FP64 (cos, sin) for the solves;
//           clears the optional frame-wide inlier bitmask.
//   hyp     one thread per (cluster, hypothesis): Philox4x32-10 seed pair,
//           validity, FP64 2x2 solve (Sec. 3.2, Eq. 6 for two seeds), stored
//           rounded to float32 (Sec. 3.1, Alg. 1: slope/intercept step).
//   score   the hot loop (Sec. 3.1, Alg. 1: the per-point distance test).
//           Workgroup = (cluster, block of 256 hypotheses); each wave owns 64
//           hypotheses.  Lanes hold points in registers (rows of 64 points);
//           the hypothesis (vx, vy) is wave-uniform and read through scalar
//           loads.  Per point: two float32 FMAs and one compare whose 64-lane
//           ballot is popcounted by the scalar unit.  Counts go to global memory.
//   refit   one workgroup per cluster: arg-max over the counts (lowest index
//           on ties), FP64 re-classification under the kept hypothesis, FP64
//           normal-equation sums in a fixed reduction tree, 2x2 solve (Sec. 3.2,
//           Eq. 7, Alg. 2) and atan2 heading (Eq. 8).
//
// No floating-point atomics and fixed reduction orders: results are bitwise
// reproducible run to run and independent of the other clusters in the frame.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "rv.h"

// v_writelane_b32: write a wave-uniform value into one lane of a VGPR (the
// LLVM intrinsic; clang exposes no builtin for it).
__device__ int amdgcn_writelane(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace {

constexpr int kBlock = 256;             // threads per workgroup (4 x wave64)
constexpr int kWave = 64;
constexpr int kHypPerWave = 64;         // one count slot per lane
constexpr int kHypPerBlock = 256;       // 4 waves x 64 hypotheses
constexpr int kRowsMax = 16;            // rows of 64 points held in registers per pass
constexpr int kHypGroup = 8;            // hypotheses per scalar load in the scoring loop
constexpr int kXcds = 8;                // MI355X: 8 XCDs, workgroups dealt round-robin
constexpr int kSizeClasses = 128;       // quarter-octave size classes for the dispatch order
constexpr int kPlanBlock = 1024;
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// mixed into the counter words, key advanced by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint32_t hi0 = __umulhi(kPhiloxM0, x.x);
        const uint32_t lo0 = kPhiloxM0 * x.x;
        const uint32_t hi1 = __umulhi(kPhiloxM1, x.z);
        const uint32_t lo1 = kPhiloxM1 * x.z;
        x = make_uint4(hi1 ^ x.y ^ k0, lo1, hi0 ^ x.w ^ k1, lo0);
    }
    return x;
}

// Two distinct indices in [0, n) from two uniform words (multiply-shift map;
// the second index skips the first).  Requires 2 <= n < 2^31.
__device__ __forceinline__ void seed_pair(uint32_t u0, uint32_t u1, uint32_t n, uint32_t &i,
                                          uint32_t &j) {
    i = __umulhi(u0, n);
    const uint32_t b = __umulhi(u1, n - 1u);
    j = b + (b >= i ? 1u : 0u);
}

struct Span {
    int64_t lo;
    int64_t n;
    bool ok;
};

__device__ __forceinline__ Span cluster_span(const int32_t *__restrict__ off, int64_t k,
                                             int64_t n_points) {
    const int64_t a = off[k];
    const int64_t b = off[k + 1];
    Span s;
    s.ok = a >= 0 && b >= a && b <= n_points;
    s.lo = s.ok ? a : 0;
    s.n = s.ok ? b - a : 0;
    return s;
}

struct Hypothesis {
    double vx, vy;
    bool valid;
};

// Hypothesis h of cluster k: seed pair, validity and the FP64 2x2 solve of
// v_d = vx cos + vy sin at the two seeds (Cramer's rule).
__device__ __forceinline__ Hypothesis make_hypothesis(
    const float *__restrict__ theta, const float *__restrict__ vd,
    const double *__restrict__ c64, const double *__restrict__ s64, Span sp, uint32_t h,
    uint32_t k, uint32_t key0, uint32_t key1) {
    const uint4 u = philox4x32_10(make_uint4(h, k, 0u, 0u), key0, key1);
    uint32_t i, j;
    seed_pair(u.x, u.y, (uint32_t)sp.n, i, j);
    const int64_t pi = sp.lo + i, pj = sp.lo + j;
    const float ti = theta[pi], tj = theta[pj], vi = vd[pi], vj = vd[pj];
    Hypothesis hy;
    hy.valid = isfinite(ti) && isfinite(tj) && isfinite(vi) && isfinite(vj) &&
               fabs((double)tj - (double)ti) >= RV_MIN_SEED_SEPARATION;
    if (!hy.valid) {
        hy.vx = hy.vy = __builtin_nan("");
        return hy;
    }
    const double ci = c64[pi], si = s64[pi], cj = c64[pj], sj = s64[pj];
    const double dvi = vi, dvj = vj;
    const double det = ci * sj - si * cj;
    hy.vx = (dvi * sj - dvj * si) / det;
    hy.vy = (ci * dvj - cj * dvi) / det;
    return hy;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void prep_kernel(
    const float *__restrict__ theta, const float *__restrict__ vd, int64_t n_points,
    float *__restrict__ c32, float *__restrict__ s32, float *__restrict__ v32,
    double *__restrict__ c64, double *__restrict__ s64, uint32_t *__restrict__ bits,
    int64_t n_words) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < n_points) {
        const float t = theta[p], v = vd[p];
        double s, c;
        sincos((double)t, &s, &c);
        const bool ok = isfinite(t) && isfinite(v);
        c64[p] = c;
        s64[p] = s;
        // A non-finite point scores as (0, 0, +inf): its residual is inf or NaN,
        // never below tau.
        c32[p] = ok ? (float)c : 0.0f;
        s32[p] = ok ? (float)s : 0.0f;
        v32[p] = ok ? v : __builtin_inff();
    }
    if (bits != nullptr && p < n_words) bits[p] = 0u;
}

// Hypotheses are stored in rows of n_hyp_pad = n_hyp rounded up to kHypGroup
// (the padding holds NaN and never counts), so the scoring loop can fetch a
// full group of kHypGroup (vx, vy) pairs with one scalar load.
__global__ __launch_bounds__(kBlock) void hyp_kernel(
    const float *__restrict__ theta, const float *__restrict__ vd,
    const int32_t *__restrict__ off, int64_t n_points, int32_t n_hyp, int32_t n_hyp_pad,
    int32_t blocks_per_cluster, uint32_t key0, uint32_t key1, const double *__restrict__ c64,
    const double *__restrict__ s64, float2 *__restrict__ hyp, uint8_t *__restrict__ valid) {
    const int64_t k = blockIdx.x / blocks_per_cluster;
    const int64_t h = (int64_t)(blockIdx.x % blocks_per_cluster) * kBlock + threadIdx.x;
    if (h >= n_hyp_pad) return;
    const float qnan = __builtin_nanf("");
    const Span sp = cluster_span(off, k, n_points);
    if (h >= n_hyp || !sp.ok || sp.n < 2) {
        hyp[k * n_hyp_pad + h] = make_float2(qnan, qnan);
        if (h < n_hyp) valid[k * n_hyp + h] = 0;
        return;
    }
    const Hypothesis hy =
        make_hypothesis(theta, vd, c64, s64, sp, (uint32_t)h, (uint32_t)k, key0, key1);
    hyp[k * n_hyp_pad + h] = make_float2((float)hy.vx, (float)hy.vy);
    valid[k * n_hyp + h] = hy.valid ? 1 : 0;
}

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
// the longest work items start first (longest-processing-time-first).  The
// order inside a class depends on atomics; it only affects scheduling.
__global__ __launch_bounds__(kPlanBlock) void plan_kernel(const int32_t *__restrict__ off,
                                                          int64_t n_clusters, int64_t n_points,
                                                          int32_t *__restrict__ order) {
    __shared__ uint32_t count[kSizeClasses];
    __shared__ uint32_t start[kSizeClasses];
    for (int c = threadIdx.x; c < kSizeClasses; c += kPlanBlock) count[c] = 0;
    __syncthreads();
    for (int64_t k = threadIdx.x; k < n_clusters; k += kPlanBlock)
        atomicAdd(&count[size_class(cluster_span(off, k, n_points).n)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t at = 0;
        for (int c = kSizeClasses - 1; c >= 0; --c) {
            start[c] = at;
            at += count[c];
        }
    }
    __syncthreads();
    for (int64_t k = threadIdx.x; k < n_clusters; k += kPlanBlock) {
        const uint32_t pos = atomicAdd(&start[size_class(cluster_span(off, k, n_points).n)], 1u);
        order[pos] = (int32_t)k;
    }
}

// R rows of 64 points per lane (registers) against ng groups of kHypGroup
// wave-uniform hypotheses (scalar loads, one group fetched ahead); returns the
// count of hypothesis q of the wave in lane q.
template <int R>
__device__ __forceinline__ uint32_t score_rows(const float *__restrict__ c32,
                                               const float *__restrict__ s32,
                                               const float *__restrict__ v32, int64_t base,
                                               int64_t end, int lane,
                                               const float4 *__restrict__ hp, int ng,
                                               float tau) {
    float c[R], s[R], v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t p = base + r * kWave + lane;
        c[r] = 0.0f;
        s[r] = 0.0f;
        v[r] = __builtin_inff();
        if (p < end) {
            c[r] = c32[p];
            s[r] = s32[p];
            v[r] = v32[p];
        }
    }
    uint32_t counts = 0;
    float4 h0 = hp[0], h1 = hp[1], h2 = hp[2], h3 = hp[3];
    for (int g = 0; g < ng; ++g) {
        const int gn = g + 1 < ng ? g + 1 : g;
        const float4 n0 = hp[4 * gn], n1 = hp[4 * gn + 1], n2 = hp[4 * gn + 2],
                     n3 = hp[4 * gn + 3];
        const float hx[kHypGroup] = {h0.x, h0.z, h1.x, h1.z, h2.x, h2.z, h3.x, h3.z};
        const float hy[kHypGroup] = {h0.y, h0.w, h1.y, h1.w, h2.y, h2.w, h3.y, h3.w};
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
        }
        h0 = n0;
        h1 = n1;
        h2 = n2;
        h3 = n3;
    }
    return counts;
}

// Work item = (cluster, block of 256 hypotheses); the item of block i is chosen
// so that clusters are taken in the planned order and all items of one cluster
// run on the same XCD (blocks are dealt to the 8 XCDs round-robin), sharing
// that XCD's L2 copy of the cluster's points.
__global__ __launch_bounds__(kBlock) void score_kernel(
    const int32_t *__restrict__ off, const int32_t *__restrict__ order, int64_t n_clusters,
    int64_t n_points, int32_t n_hyp, int32_t n_hyp_pad, int32_t blocks_per_cluster,
    const float *__restrict__ c32, const float *__restrict__ s32, const float *__restrict__ v32,
    const float2 *__restrict__ hyp, float tau, int32_t *__restrict__ counts) {
    const uint32_t xcd = blockIdx.x % kXcds;
    const uint32_t r = blockIdx.x / kXcds;
    const int64_t j = xcd + (int64_t)kXcds * (r / (uint32_t)blocks_per_cluster);
    if (j >= n_clusters) return;
    const int b = (int)(r % (uint32_t)blocks_per_cluster);
    const int64_t k = order[j];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t h0 = (int64_t)b * kHypPerBlock + wave * kHypPerWave;
    if (h0 >= n_hyp) return;
    const int nh = (int64_t)n_hyp - h0 < kHypPerWave ? (int)((int64_t)n_hyp - h0) : kHypPerWave;
    const Span sp = cluster_span(off, k, n_points);
    if (!sp.ok || sp.n < 2) {
        if (lane < nh) counts[k * n_hyp + h0 + lane] = 0;
        return;
    }
    const int ng = (nh + kHypGroup - 1) / kHypGroup;
    const float4 *hp = reinterpret_cast<const float4 *>(hyp + k * n_hyp_pad + h0);
    const int64_t end = sp.lo + sp.n;
    uint32_t total = 0;
    for (int64_t base = sp.lo; base < end; base += (int64_t)kRowsMax * kWave) {
        const int64_t left = (end - base + kWave - 1) / kWave;
        const int rows = (int)(left < kRowsMax ? left : kRowsMax);
        switch (rows) {
#define RV_ROWS(R) \
    case R: total += score_rows<R>(c32, s32, v32, base, end, lane, hp, ng, tau); break;
            RV_ROWS(1) RV_ROWS(2) RV_ROWS(3) RV_ROWS(4) RV_ROWS(5) RV_ROWS(6) RV_ROWS(7)
            RV_ROWS(8) RV_ROWS(9) RV_ROWS(10) RV_ROWS(11) RV_ROWS(12) RV_ROWS(13)
            RV_ROWS(14) RV_ROWS(15) RV_ROWS(16)
#undef RV_ROWS
            default: break;
        }
    }
    if (lane < nh) counts[k * n_hyp + h0 + lane] = (int32_t)total;
}

__global__ __launch_bounds__(kBlock) void refit_kernel(
    const int32_t *__restrict__ off, int64_t n_points, int32_t n_hyp, uint32_t key0,
    uint32_t key1, const float *__restrict__ theta, const float *__restrict__ vd,
    const double *__restrict__ c64, const double *__restrict__ s64,
    const int32_t *__restrict__ counts, const uint8_t *__restrict__ valid, double tau,
    float *__restrict__ out_vx, float *__restrict__ out_vy, float *__restrict__ out_heading,
    int32_t *__restrict__ out_n_inliers, uint8_t *__restrict__ out_status,
    int32_t *__restrict__ out_n_near, uint32_t *__restrict__ bits,
    int32_t *__restrict__ out_best) {
    __shared__ uint64_t red_key[kBlock / kWave];
    __shared__ double red_sum[kBlock / kWave][5];
    __shared__ int red_cnt[kBlock / kWave][2];

    const int64_t k = blockIdx.x;
    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    const Span sp = cluster_span(off, k, n_points);
    const float qnan = __builtin_nanf("");

    uint8_t st = RV_CLUSTER_OK;
    if (!sp.ok)
        st = RV_CLUSTER_BAD_OFFSETS;
    else if (sp.n < 2)
        st = RV_CLUSTER_TOO_FEW_POINTS;
    if (st != RV_CLUSTER_OK) {
        if (tid == 0) {
            out_vx[k] = qnan;
            out_vy[k] = qnan;
            out_heading[k] = qnan;
            out_n_inliers[k] = 0;
            out_status[k] = st;
            if (out_n_near) out_n_near[k] = 0;
            if (out_best) out_best[k] = -1;
        }
        return;
    }

    // Keep the valid hypothesis with the most inliers; lowest index on ties.
    uint64_t key = 0;
    for (int64_t h = tid; h < n_hyp; h += kBlock) {
        const int64_t q = k * n_hyp + h;
        if (valid[q]) {
            const uint64_t kk = ((uint64_t)(uint32_t)counts[q] << 32) |
                                (uint64_t)(0xFFFFFFFFu - (uint32_t)h);
            key = kk > key ? kk : key;
        }
    }
    key = wave_max_u64(key);
    if (lane == 0) red_key[wave] = key;
    __syncthreads();
    key = red_key[0];
    for (int w = 1; w < kBlock / kWave; ++w) key = red_key[w] > key ? red_key[w] : key;
    if (key == 0) {
        if (tid == 0) {
            out_vx[k] = qnan;
            out_vy[k] = qnan;
            out_heading[k] = qnan;
            out_n_inliers[k] = 0;
            out_status[k] = RV_CLUSTER_ALL_DEGENERATE;
            if (out_n_near) out_n_near[k] = 0;
            if (out_best) out_best[k] = -1;
        }
        return;
    }
    const uint32_t hbest = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFu);
    const Hypothesis hy =
        make_hypothesis(theta, vd, c64, s64, sp, hbest, (uint32_t)k, key0, key1);

    // Re-classify under the kept hypothesis in FP64 and accumulate the normal
    // equations (A^T A) v = A^T v_d over its inliers.  Waves walk 64-aligned
    // global blocks so one ballot maps onto two words of the bitmask.
    const int64_t end = sp.lo + sp.n;
    double scc = 0.0, scs = 0.0, sss = 0.0, scv = 0.0, ssv = 0.0;
    int n_in = 0, n_near = 0;
    for (int64_t p0 = (sp.lo & ~(int64_t)(kWave - 1)) + wave * kWave; p0 < end; p0 += kBlock) {
        const int64_t p = p0 + lane;
        bool inlier = false;
        if (p >= sp.lo && p < end) {
            const float t = theta[p], v = vd[p];
            if (isfinite(t) && isfinite(v)) {
                const double c = c64[p], s = s64[p], dv = v;
                const double res = fabs(dv - hy.vx * c - hy.vy * s);
                n_near += fabs(res - tau) <= RV_NEAR_TAU_WINDOW ? 1 : 0;
                if (res < tau) {
                    inlier = true;
                    n_in += 1;
                    scc += c * c;
                    scs += c * s;
                    sss += s * s;
                    scv += c * dv;
                    ssv += s * dv;
                }
            }
        }
        if (bits != nullptr) {
            const uint64_t m = __builtin_amdgcn_ballot_w64(inlier);
            if (lane == 0) {
                const uint32_t w0 = (uint32_t)m, w1 = (uint32_t)(m >> 32);
                if (w0) atomicOr(&bits[p0 >> 5], w0);
                if (w1) atomicOr(&bits[(p0 >> 5) + 1], w1);
            }
        }
    }
    scc = wave_sum(scc);
    scs = wave_sum(scs);
    sss = wave_sum(sss);
    scv = wave_sum(scv);
    ssv = wave_sum(ssv);
    n_in = wave_sum_i(n_in);
    n_near = wave_sum_i(n_near);
    if (lane == 0) {
        red_sum[wave][0] = scc;
        red_sum[wave][1] = scs;
        red_sum[wave][2] = sss;
        red_sum[wave][3] = scv;
        red_sum[wave][4] = ssv;
        red_cnt[wave][0] = n_in;
        red_cnt[wave][1] = n_near;
    }
    __syncthreads();
    if (tid != 0) return;
    scc = red_sum[0][0];
    scs = red_sum[0][1];
    sss = red_sum[0][2];
    scv = red_sum[0][3];
    ssv = red_sum[0][4];
    n_in = red_cnt[0][0];
    n_near = red_cnt[0][1];
    for (int w = 1; w < kBlock / kWave; ++w) {
        scc += red_sum[w][0];
        scs += red_sum[w][1];
        sss += red_sum[w][2];
        scv += red_sum[w][3];
        ssv += red_sum[w][4];
        n_in += red_cnt[w][0];
        n_near += red_cnt[w][1];
    }
    out_n_inliers[k] = n_in;
    if (out_n_near) out_n_near[k] = n_near;
    if (out_best) out_best[k] = (int32_t)hbest;
    const double det = scc * sss - scs * scs;
    if (n_in < 2 || !(det > 0.0)) {
        out_vx[k] = qnan;
        out_vy[k] = qnan;
        out_heading[k] = qnan;
        out_status[k] = RV_CLUSTER_SINGULAR_REFIT;
        return;
    }
    const double fvx = (sss * scv - scs * ssv) / det;
    const double fvy = (scc * ssv - scs * scv) / det;
    out_vx[k] = (float)fvx;
    out_vy[k] = (float)fvy;
    out_heading[k] = (float)atan2(fvy, fvx);
    out_status[k] = RV_CLUSTER_OK;
}

__global__ __launch_bounds__(kBlock) void philox_kernel(const uint32_t *__restrict__ ctr,
                                                        const uint32_t *__restrict__ key,
                                                        uint32_t *__restrict__ out,
                                                        int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
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

thread_local char g_error[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
    return code;
}

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t c32, s32, v32, c64, s64, hyp, valid, counts, order, total;
};

int64_t padded_hyp(int32_t n_hyp) { return ((int64_t)n_hyp + kHypGroup - 1) / kHypGroup * kHypGroup; }

Layout make_layout(int64_t n_clusters, int64_t n_points, int32_t n_hyp) {
    Layout L;
    const size_t np = (size_t)n_points;
    const size_t nq = (size_t)n_clusters * (size_t)n_hyp;
    size_t at = 0;
    L.c32 = at; at = align_up(at + np * sizeof(float));
    L.s32 = at; at = align_up(at + np * sizeof(float));
    L.v32 = at; at = align_up(at + np * sizeof(float));
    L.c64 = at; at = align_up(at + np * sizeof(double));
    L.s64 = at; at = align_up(at + np * sizeof(double));
    const size_t nq_pad = (size_t)n_clusters * (size_t)padded_hyp(n_hyp);
    L.hyp = at; at = align_up(at + nq_pad * sizeof(float2));
    L.valid = at; at = align_up(at + nq * sizeof(uint8_t));
    L.counts = at; at = align_up(at + nq * sizeof(int32_t));
    L.order = at; at = align_up(at + (size_t)n_clusters * sizeof(int32_t));
    L.total = at;
    return L;
}

// Stage timing: events recorded around each kernel of each call.
constexpr int kStages = 4;
struct TimedCall {
    hipEvent_t ev[kStages + 1];
};
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

}  // namespace

extern "C" {

size_t rv_workspace_bytes(int64_t n_clusters, int64_t n_points, int32_t n_hyp) {
    if (n_clusters < 0 || n_points < 0 || n_hyp < 0) return 0;
    return make_layout(n_clusters, n_points, n_hyp).total;
}

const char *rv_last_error(void) { return g_error; }

int rv_estimate_velocity(const float *theta, const float *vd, const int32_t *cluster_offsets,
                         int64_t n_clusters, int64_t n_points, int32_t n_hyp, float tau,
                         uint64_t seed, float *vx, float *vy, float *heading, int32_t *n_inliers,
                         uint8_t *status, int32_t *n_near_tau, uint32_t *inlier_bits,
                         int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                         size_t workspace_bytes, void *stream) {
    g_error[0] = '\0';
    if (n_clusters < 0) return fail(RV_ERR_INVALID_ARG, "n_clusters < 0");
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
    const int64_t n_hyp_pad = padded_hyp(n_hyp);
    const int64_t score_bpc = ((int64_t)n_hyp + kHypPerBlock - 1) / kHypPerBlock;
    const int64_t hyp_bpc = (n_hyp_pad + kBlock - 1) / kBlock;
    const int64_t clusters_xcd = (n_clusters + kXcds - 1) / kXcds * kXcds;
    if (clusters_xcd > (int64_t)INT32_MAX / hyp_bpc)
        return fail(RV_ERR_INVALID_ARG, "n_clusters * ceil(n_hyp / 256) exceeds 2^31 - 1");
    const Layout L = make_layout(n_clusters, n_points, n_hyp);
    if (workspace == nullptr || workspace_bytes < L.total)
        return fail(RV_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                    workspace == nullptr ? (size_t)0 : workspace_bytes);
    if (((uintptr_t)workspace % kAlign) != 0)
        return fail(RV_ERR_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    if (n_clusters == 0) return RV_OK;

    char *ws = (char *)workspace;
    float *c32 = (float *)(ws + L.c32);
    float *s32 = (float *)(ws + L.s32);
    float *v32 = (float *)(ws + L.v32);
    double *c64 = (double *)(ws + L.c64);
    double *s64 = (double *)(ws + L.s64);
    float2 *hyp = (float2 *)(ws + L.hyp);
    uint8_t *valid = (uint8_t *)(ws + L.valid);
    int32_t *counts = hyp_counts != nullptr ? hyp_counts : (int32_t *)(ws + L.counts);
    int32_t *order = (int32_t *)(ws + L.order);
    const uint32_t key0 = (uint32_t)(seed & 0xFFFFFFFFu), key1 = (uint32_t)(seed >> 32);
    const int64_t n_words = inlier_bits != nullptr ? (n_points + 31) / 32 : 0;
    hipStream_t st = (hipStream_t)stream;

    TimedCall tc;
    const bool timed = take_timed_call(tc);
    if (timed) (void)hipEventRecord(tc.ev[0], st);

    const int64_t prep_items = n_points > n_words ? n_points : n_words;
    if (prep_items > 0)
        hipLaunchKernelGGL(prep_kernel, dim3((unsigned)((prep_items + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, theta, vd, n_points, c32, s32, v32, c64, s64,
                           inlier_bits, n_words);
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanBlock), 0, st, cluster_offsets,
                       n_clusters, n_points, order);
    if (timed) (void)hipEventRecord(tc.ev[1], st);
    hipLaunchKernelGGL(hyp_kernel, dim3((unsigned)(n_clusters * hyp_bpc)), dim3(kBlock), 0, st,
                       theta, vd, cluster_offsets, n_points, n_hyp, (int32_t)n_hyp_pad,
                       (int32_t)hyp_bpc, key0, key1, c64, s64, hyp, valid);
    if (timed) (void)hipEventRecord(tc.ev[2], st);
    hipLaunchKernelGGL(score_kernel, dim3((unsigned)(clusters_xcd * score_bpc)), dim3(kBlock), 0,
                       st, cluster_offsets, (const int32_t *)order, n_clusters, n_points, n_hyp,
                       (int32_t)n_hyp_pad, (int32_t)score_bpc, c32, s32, v32,
                       (const float2 *)hyp, tau, counts);
    if (timed) (void)hipEventRecord(tc.ev[3], st);
    hipLaunchKernelGGL(refit_kernel, dim3((unsigned)n_clusters), dim3(kBlock), 0, st,
                       cluster_offsets, n_points, n_hyp, key0, key1, theta, vd, c64, s64,
                       (const int32_t *)counts, (const uint8_t *)valid, (double)tau, vx, vy,
                       heading, n_inliers, status, n_near_tau, inlier_bits, best_hyp);
    if (timed) {
        (void)hipEventRecord(tc.ev[4], st);
        keep_timed_call(tc);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return RV_OK;
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
    double sum[kStages] = {0.0, 0.0, 0.0, 0.0};
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

int rv_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n,
                     void *stream) {
    g_error[0] = '\0';
    if (n < 0) return fail(RV_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return RV_OK;
    if (ctr == nullptr || key == nullptr || out == nullptr)
        return fail(RV_ERR_INVALID_ARG, "a pointer is NULL");
    const int64_t grid = (n + kBlock - 1) / kBlock;
    if (grid > INT32_MAX) return fail(RV_ERR_INVALID_ARG, "n too large");
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)grid), dim3(kBlock), 0,
                       (hipStream_t)stream, ctr, key, out, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return RV_OK;
}

}  // extern "C"
