// rv_paper.hip -- gfx950 kernels and host entry point of the paper-literal
// variant of the inlier kernel (Sec. 3.1, Alg. 1 with Eq. 5's threshold),
// followed by the least-squares kernel (Sec. 3.2, Eq. 7, Alg. 2, Eq. 8).
//
// Per cluster:
//   stats   one workgroup: per-cluster min-max normalisation of azimuth and
//           Doppler onto [0, 1] (Alg. 1's normalize(); a zero span maps to 0),
//           then the median absolute deviation of the normalised Doppler
//           values (Eq. 5, read as the statistic the text names): two medians
//           in LDS, by ranks for up to 256 points, else by bitonic sorts of
//           up to 4096 doubles.
//   score   one thread per (trial, cluster), the mapping of Alg. 1: the trial
//           draws its seed pair from Philox4x32-10 exactly as the
//           velocity-profile kernels do, fits the line through the two
//           normalised seeds, and counts the points whose perpendicular
//           distance (aa x + bb y + cc over sqrt(aa^2 + bb^2)) is at most the
//           threshold (for each line, as one comparison of the numerator
//           against the largest value that passes, found once per trial); the
//           block's best (count, lowest index) key is merged per cluster with a
//           64-bit atomic maximum.
//   refit   one workgroup: re-classifies every point under the kept line,
//           writes the inlier mask, and solves the normal equations of the
//           velocity profile on the inliers; heading = atan2(vy, vx).
// Each step is a device function.  Calls that ask for the frame-wide inlier
// mask, or have more than 256 trials per cluster, or frames above 65,536
// points or clusters, run them as three kernels; all others run them in one
// kernel, a workgroup per cluster, with the same results bit for bit.
//
// Everything is FP64 and evaluated exactly as written (no contraction), so
// counts, masks and thresholds are the same bits as a plain FP64 evaluation of
// the same expressions.

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "rv.h"
#include "rv_device.h"
#include "rv_internal.h"

#pragma clang fp contract(off)

using rv_internal::fail;
using rv_internal::g_error;
using rv_internal::keep_timed_call;
using rv_internal::take_timed_call;
using rv_internal::TimedCall;

namespace {

constexpr int kPaperBlock = 256;
constexpr int kPaperWaves = kPaperBlock / kWave;
constexpr double kPaperMinSeparation = RV_MIN_SEED_SEPARATION;

// Normalised coordinate of one value: (a - lo) / span, 0 for a zero span.
__device__ __forceinline__ double unit_coord(float a, double lo, double span) {
    return span > 0.0 ? ((double)a - lo) / span : 0.0;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Ascending bitonic sort of s[0, P) (P a power of two, <= RV_PAPER_MAX_POINTS)
// by the whole workgroup; every loop bound is uniform.
__device__ void bitonic_sort(double *s, int P) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += kPaperBlock) {
                const int lo = (i / stride) * 2 * stride + (i % stride);
                const int hi = lo + stride;
                const bool ascending = (lo & size) == 0;
                const double a = s[lo], b = s[hi];
                if ((a > b) == ascending) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Median of the m smallest entries of a sorted array (mean of the two middle
// values for an even m); m >= 1.
__device__ __forceinline__ double sorted_median(const double *s, int m) {
    return (m & 1) ? s[m / 2] : (s[m / 2 - 1] + s[m / 2]) / 2.0;
}

// The same median for n <= kPaperBlock entries without sorting (entries past
// n are the +inf padding, never below a finite entry, so they are left out):
// thread i ranks entry s[i] against all n (how many are below it, how many not
// above it); the entry whose rank range holds a middle position is that order
// statistic (equal entries write the same value), and the two middle values
// are combined as sorted_median combines them.  Called by the whole workgroup;
// the barrier orders the writes of mid[] before its reads.
__device__ double rank_median(const double *s, int n, int m, double *mid) {
    const int q1 = m / 2, q0 = (m & 1) ? q1 : q1 - 1;
    const int i = threadIdx.x;
    if (i < n) {
        const double a = s[i];
        int below = 0, upto = 0;
        for (int j = 0; j < n; ++j) {
            const double b = s[j];
            below += b < a ? 1 : 0;
            upto += b <= a ? 1 : 0;
        }
        if (below <= q0 && q0 < upto) mid[0] = a;
        if (below <= q1 && q1 < upto) mid[1] = a;
    }
    __syncthreads();
    return (m & 1) ? mid[1] : (mid[0] + mid[1]) / 2.0;
}

// Spans of a cluster with 2 <= n <= RV_PAPER_MAX_POINTS points, the only ones
// the score and refit kernels work on.
__device__ __forceinline__ bool paper_cluster(const Span &sp) {
    return sp.ok && sp.n >= 2 && sp.n <= RV_PAPER_MAX_POINTS;
}

// Workgroup LDS of the threshold step.
struct StatsShared {
    double sort[RV_PAPER_MAX_POINTS];
    double red[4][kPaperWaves];
    int cnt[kPaperWaves];
    double mid[2][2];
};

// Threshold step of cluster k (whole workgroup; uniform early returns): the
// normalised (x, y) of its points into xy (and into s_xy, when given, for
// clusters of at most kPaperBlock points), and its threshold into thresh[k],
// NaN when the cluster takes no part or has no usable point.  Returns the
// threshold in every thread.
__device__ double paper_stats(const float *__restrict__ theta, const float *__restrict__ vd,
                              Span sp, int64_t k, double2 *__restrict__ xy,
                              double *__restrict__ thresh, StatsShared &sh, double2 *s_xy) {
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    if (tid == 0) thresh[k] = __builtin_nan("");
    if (!paper_cluster(sp)) return __builtin_nan("");
    const int n = (int)sp.n;
    const float *t = theta + sp.lo, *v = vd + sp.lo;
    // With at most one point per thread, each thread keeps its point and its
    // normalised Doppler value in registers across the steps (every loop
    // below then runs once, at p = tid).
    const bool one = n <= kPaperBlock;
    float t_own = 0.0f, v_own = 0.0f;
    double y_own = 0.0;
    if (one && tid < n) {
        t_own = t[tid];
        v_own = v[tid];
    }

    double tmin = __builtin_inf(), tmax = -__builtin_inf();
    double vmin = __builtin_inf(), vmax = -__builtin_inf();
    int m_ok = 0;
    for (int p = tid; p < n; p += kPaperBlock) {
        const float tp = one ? t_own : t[p], vp = one ? v_own : v[p];
        if (!(isfinite(tp) && isfinite(vp))) continue;
        tmin = fmin(tmin, (double)tp);
        tmax = fmax(tmax, (double)tp);
        vmin = fmin(vmin, (double)vp);
        vmax = fmax(vmax, (double)vp);
        m_ok += 1;
    }
    tmin = wave_min(tmin);
    tmax = wave_max(tmax);
    vmin = wave_min(vmin);
    vmax = wave_max(vmax);
    m_ok = wave_sum_i(m_ok);
    if (lane == 0) {
        sh.red[0][wave] = tmin;
        sh.red[1][wave] = tmax;
        sh.red[2][wave] = vmin;
        sh.red[3][wave] = vmax;
        sh.cnt[wave] = m_ok;
    }
    __syncthreads();
    tmin = sh.red[0][0];
    tmax = sh.red[1][0];
    vmin = sh.red[2][0];
    vmax = sh.red[3][0];
    m_ok = sh.cnt[0];
    for (int w = 1; w < kPaperWaves; ++w) {
        tmin = fmin(tmin, sh.red[0][w]);
        tmax = fmax(tmax, sh.red[1][w]);
        vmin = fmin(vmin, sh.red[2][w]);
        vmax = fmax(vmax, sh.red[3][w]);
        m_ok += sh.cnt[w];
    }
    const double tspan = tmax - tmin, vspan = vmax - vmin;

    // Normalised coordinates (x = NaN marks a point that takes no part), and
    // the finite y values, padded with +inf to a power of two, for the median.
    int P = 2;
    while (P < n) P <<= 1;
    for (int p = tid; p < P; p += kPaperBlock) {
        double y = __builtin_inf();
        if (p < n) {
            const float tp = one ? t_own : t[p], vp = one ? v_own : v[p];
            const bool ok = isfinite(tp) && isfinite(vp);
            const double x = ok ? unit_coord(tp, tmin, tspan) : __builtin_nan("");
            y = ok ? unit_coord(vp, vmin, vspan) : __builtin_inf();
            const double2 q = make_double2(x, ok ? y : __builtin_nan(""));
            xy[sp.lo + p] = q;
            if (one && s_xy != nullptr) s_xy[p] = q;
        }
        if (one) y_own = y;
        sh.sort[p] = y;
    }
    __syncthreads();
    if (m_ok == 0) return __builtin_nan("");
    // Up to one entry per thread: ranks; above that: a bitonic sort.
    const bool ranks = P <= kPaperBlock;
    double med;
    if (ranks) {
        med = rank_median(sh.sort, n, m_ok, sh.mid[0]);
    } else {
        bitonic_sort(sh.sort, P);
        med = sorted_median(sh.sort, m_ok);
    }
    __syncthreads();
    for (int p = tid; p < P; p += kPaperBlock) {
        double d = __builtin_inf();
        if (one) {
            // y_own is +inf exactly for a point that takes no part.
            if (p < n && y_own < __builtin_inf()) d = fabs(y_own - med);
        } else if (p < n && isfinite(t[p]) && isfinite(v[p])) {
            d = fabs(unit_coord(v[p], vmin, vspan) - med);
        }
        sh.sort[p] = d;
    }
    __syncthreads();
    double mad;
    if (ranks) {
        mad = rank_median(sh.sort, n, m_ok, sh.mid[1]);
    } else {
        bitonic_sort(sh.sort, P);
        mad = sorted_median(sh.sort, m_ok);
    }
    if (tid == 0) thresh[k] = mad;
    return mad;
}

__global__ __launch_bounds__(kPaperBlock) void paper_stats_kernel(
    const float *__restrict__ theta, const float *__restrict__ vd,
    const int32_t *__restrict__ off, int64_t n_points, double2 *__restrict__ xy,
    double *__restrict__ thresh, unsigned long long *__restrict__ best_key) {
    __shared__ StatsShared sh;
    const int64_t k = blockIdx.x;
    if (threadIdx.x == 0) best_key[k] = 0;
    (void)paper_stats(theta, vd, cluster_span(off, k, n_points), k, xy, thresh, sh, nullptr);
}

// Line of a trial through its normalised seeds (Alg. 1: slope and intercept)
// and the denominator of its distance.
struct Line {
    double m, c, distd;
    bool valid;
};

__device__ __forceinline__ Line trial_line(const float *__restrict__ t, const double2 *__restrict__ xy,
                                           int n, uint32_t h, uint32_t k, uint32_t key0,
                                           uint32_t key1) {
    const uint4 u = philox4x32_10(make_uint4(h, k, 0u, 0u), key0, key1);
    uint32_t i, j;
    seed_pair(u.x, u.y, (uint32_t)n, i, j);
    const double2 a = xy[i], b = xy[j];
    Line L;
    L.valid = !__builtin_isnan(a.x) && !__builtin_isnan(b.x) &&
              fabs((double)t[j] - (double)t[i]) >= kPaperMinSeparation;
    L.m = L.c = L.distd = 0.0;
    if (!L.valid) return L;
    L.m = (b.y - a.y) / (b.x - a.x);
    L.c = a.y - L.m * a.x;
    const double aa = -L.m, bb = 1.0;
    L.distd = sqrt(aa * aa + bb * bb);
    return L;
}

// Numerator of Alg. 1's distance, aa x + bb y + cc with aa = -m, bb = 1 and
// cc = -c, evaluated as written.
__device__ __forceinline__ double dist_num(const Line &L, double2 p) {
    const double aa = -L.m, bb = 1.0, cc = -L.c;
    return (aa * p.x + bb * p.y) + cc;
}

// Alg. 1's inlier test of one point against a valid line.
__device__ __forceinline__ bool within(const Line &L, double2 p, double th) {
    return fabs(dist_num(L, p) / L.distd) <= th;
}

// The same test without a division per point.  For one line, the rounded
// quotient |num| / distd is at most th exactly when |num| <= bound, the
// largest double x >= 0 whose quotient x / distd rounds to at most th: a
// correctly rounded quotient never decreases as x grows.  bound lies within a
// few units in the last place of th * distd; it is found by bisection over the
// bit patterns of the eight doubles around that product (non-negative doubles
// order like their bit patterns), each step one division of the same kind as
// the literal test's.  Returns false where that bracket does not hold (th = 0,
// extreme magnitudes); the trial then runs the literal test.
__device__ __forceinline__ bool pass_bound(double distd, double th, double &bound) {
    if (!(distd >= 1.0) || !(distd < __builtin_inf()) || !(th > 0.0) || !(th < __builtin_inf()))
        return false;
    const double x0 = th * distd;
    if (!(x0 > 0x1p-1000) || !(x0 < 0x1p1000)) return false;
    long long lo = __builtin_bit_cast(long long, x0) - 4;
    long long hi = lo + 8;
    if (!(__builtin_bit_cast(double, lo) / distd <= th) ||
        __builtin_bit_cast(double, hi) / distd <= th)
        return false;
    while (hi - lo > 1) {
        const long long mid = lo + (hi - lo) / 2;
        if (__builtin_bit_cast(double, mid) / distd <= th)
            lo = mid;
        else
            hi = mid;
    }
    bound = __builtin_bit_cast(double, lo);
    return true;
}

// Trial h of cluster k in this thread (Alg. 1's thread) and the best (count,
// lowest index) key over the workgroup's trials, returned in every thread
// (0 when none is valid).  Whole workgroup; uniform early return.
__device__ unsigned long long paper_score(const float *__restrict__ theta, Span sp, int64_t k,
                                          int64_t h, int32_t n_hyp, uint32_t key0, uint32_t key1,
                                          const double2 *__restrict__ pts, double th,
                                          int32_t *__restrict__ hyp_counts,
                                          unsigned long long *s_key) {
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    if (!paper_cluster(sp)) {
        if (hyp_counts != nullptr && h < n_hyp) hyp_counts[k * n_hyp + h] = 0;
        return 0;
    }
    const int n = (int)sp.n;
    unsigned long long key = 0;
    if (h < n_hyp) {
        const Line L = trial_line(theta + sp.lo, pts, n, (uint32_t)h, (uint32_t)k, key0, key1);
        int count = 0;
        if (L.valid) {
            // A point that takes no part is stored as (NaN, NaN); its distance
            // is NaN and never passes.  Points are independent: the loops are
            // unrolled and have no branch.
            double bound;
            if (pass_bound(L.distd, th, bound)) {
#pragma unroll 8
                for (int p = 0; p < n; ++p) count += fabs(dist_num(L, pts[p])) <= bound ? 1 : 0;
            } else {
#pragma unroll 8
                for (int p = 0; p < n; ++p) count += within(L, pts[p], th) ? 1 : 0;
            }
            key = ((unsigned long long)count << 32) | (0xFFFFFFFFull - (uint32_t)h);
        }
        if (hyp_counts != nullptr) hyp_counts[k * n_hyp + h] = count;
    }
    key = wave_max_u64(key);
    if (lane == 0) s_key[wave] = key;
    __syncthreads();
    key = s_key[0];
    for (int w = 1; w < kPaperWaves; ++w) key = s_key[w] > key ? s_key[w] : key;
    return key;
}

// Block = (cluster, 256 trials); blocks of one cluster merge their keys with a
// 64-bit atomic maximum, whose result does not depend on their order.
__global__ __launch_bounds__(kPaperBlock) void paper_score_kernel(
    const float *__restrict__ theta, const int32_t *__restrict__ off, int64_t n_points,
    int32_t n_hyp, int32_t blocks_per_cluster, uint32_t key0, uint32_t key1,
    const double2 *__restrict__ xy, const double *__restrict__ thresh,
    unsigned long long *__restrict__ best_key, int32_t *__restrict__ hyp_counts) {
    __shared__ unsigned long long s_key[kPaperWaves];
    const int64_t k = blockIdx.x / blocks_per_cluster;
    const int b = (int)(blockIdx.x % blocks_per_cluster);
    const int64_t h = (int64_t)b * kPaperBlock + threadIdx.x;
    const Span sp = cluster_span(off, k, n_points);
    const double2 *pts = paper_cluster(sp) ? xy + sp.lo : xy;
    const unsigned long long key =
        paper_score(theta, sp, k, h, n_hyp, key0, key1, pts, thresh[k], hyp_counts, s_key);
    if (threadIdx.x == 0 && key != 0) atomicMax(&best_key[k], key);
}

struct PaperOutputs {
    float *vx, *vy, *heading;
    int32_t *n_inliers;
    uint8_t *status;
    int32_t *best;
    uint32_t *bits;
};

__device__ __forceinline__ void paper_failed(const PaperOutputs &o, int64_t k, uint8_t st) {
    const float qnan = __builtin_nanf("");
    o.vx[k] = qnan;
    o.vy[k] = qnan;
    o.heading[k] = qnan;
    o.n_inliers[k] = 0;
    o.status[k] = st;
    if (o.best) o.best[k] = -1;
}

// Refit of cluster k under its kept trial `best` (0: none valid) with
// threshold th (whole workgroup; uniform early returns).
__device__ void paper_refit(const float *__restrict__ theta, const float *__restrict__ vd, Span sp,
                            int64_t k, uint32_t key0, uint32_t key1, const double2 *__restrict__ xy,
                            double th, unsigned long long best, const PaperOutputs &o,
                            double (*s_sum)[5], int *s_cnt) {
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    if (!sp.ok || sp.n < 2 || sp.n > RV_PAPER_MAX_POINTS) {
        if (tid == 0)
            paper_failed(o, k, !sp.ok ? RV_CLUSTER_BAD_OFFSETS
                                      : (sp.n < 2 ? RV_CLUSTER_TOO_FEW_POINTS : RV_CLUSTER_TOO_LARGE));
        return;
    }
    if (best == 0) {
        if (tid == 0) paper_failed(o, k, RV_CLUSTER_ALL_DEGENERATE);
        return;
    }
    const int n = (int)sp.n;
    const uint32_t hbest = 0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFull);
    const double2 *pts = xy + sp.lo;
    const Line L = trial_line(theta + sp.lo, pts, n, hbest, (uint32_t)k, key0, key1);
    const int64_t end = sp.lo + sp.n;
    double scc = 0.0, scs = 0.0, sss = 0.0, scv = 0.0, ssv = 0.0;
    int n_in = 0;
    // 64-aligned global blocks of points, so one wave ballot covers two mask words.
    for (int64_t p0 = (sp.lo & ~(int64_t)(kWave - 1)) + (int64_t)wave * kWave; p0 < end;
         p0 += kPaperBlock) {
        const int64_t p = p0 + lane;
        bool inlier = false;
        if (p >= sp.lo && p < end) {
            const double2 q = xy[p];
            if (!__builtin_isnan(q.x) && within(L, q, th)) {
                inlier = true;
                n_in += 1;
                double s, c;
                sincos((double)theta[p], &s, &c);
                const double dv = vd[p];
                scc += c * c;
                scs += c * s;
                sss += s * s;
                scv += c * dv;
                ssv += s * dv;
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
    scc = wave_sum(scc);
    scs = wave_sum(scs);
    sss = wave_sum(sss);
    scv = wave_sum(scv);
    ssv = wave_sum(ssv);
    n_in = wave_sum_i(n_in);
    if (lane == 0) {
        s_sum[wave][0] = scc;
        s_sum[wave][1] = scs;
        s_sum[wave][2] = sss;
        s_sum[wave][3] = scv;
        s_sum[wave][4] = ssv;
        s_cnt[wave] = n_in;
    }
    __syncthreads();
    if (tid != 0) return;
    scc = s_sum[0][0];
    scs = s_sum[0][1];
    sss = s_sum[0][2];
    scv = s_sum[0][3];
    ssv = s_sum[0][4];
    n_in = s_cnt[0];
    for (int w = 1; w < kPaperWaves; ++w) {
        scc += s_sum[w][0];
        scs += s_sum[w][1];
        sss += s_sum[w][2];
        scv += s_sum[w][3];
        ssv += s_sum[w][4];
        n_in += s_cnt[w];
    }
    o.n_inliers[k] = n_in;
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

__global__ __launch_bounds__(kPaperBlock) void paper_refit_kernel(
    const float *__restrict__ theta, const float *__restrict__ vd, const int32_t *__restrict__ off,
    int64_t n_points, uint32_t key0, uint32_t key1, const double2 *__restrict__ xy,
    const double *__restrict__ thresh, const unsigned long long *__restrict__ best_key,
    PaperOutputs o) {
    __shared__ double s_sum[kPaperWaves][5];
    __shared__ int s_cnt[kPaperWaves];
    const int64_t k = blockIdx.x;
    paper_refit(theta, vd, cluster_span(off, k, n_points), k, key0, key1, xy, thresh[k],
                best_key[k], o, s_sum, s_cnt);
}

// Frames whose clusters each take one workgroup of trials (at most 256), with
// no frame-wide inlier mask requested (its words are shared by neighbouring
// clusters): one launch, a workgroup per cluster, running the threshold step,
// the trials and the refit with the same device functions as the three
// kernels, so every output is theirs bit for bit.  A workgroup reads back only
// the normalised points it wrote itself, after a workgroup barrier.
__global__ __launch_bounds__(kPaperBlock) void paper_frame_kernel(
    const float *__restrict__ theta, const float *__restrict__ vd, const int32_t *__restrict__ off,
    int64_t n_points, int32_t n_hyp, uint32_t key0, uint32_t key1, double2 *__restrict__ xy,
    double *__restrict__ thresh, int32_t *__restrict__ hyp_counts, PaperOutputs o) {
    __shared__ StatsShared sh;
    __shared__ double2 s_xy[kPaperBlock];  // normalised points of clusters of <= 256 points
    __shared__ unsigned long long s_key[kPaperWaves];
    __shared__ double s_sum[kPaperWaves][5];
    __shared__ int s_cnt[kPaperWaves];
    const int64_t k = blockIdx.x;
    const Span sp = cluster_span(off, k, n_points);
    const double th = paper_stats(theta, vd, sp, k, xy, thresh, sh, s_xy);
    __syncthreads();
    // Trials read the points from LDS where they fit, else from global memory.
    unsigned long long best;
    if (paper_cluster(sp) && sp.n <= kPaperBlock)
        best = paper_score(theta, sp, k, threadIdx.x, n_hyp, key0, key1, s_xy, th, hyp_counts,
                           s_key);
    else
        best = paper_score(theta, sp, k, threadIdx.x, n_hyp, key0, key1,
                           paper_cluster(sp) ? xy + sp.lo : xy, th, hyp_counts, s_key);
    paper_refit(theta, vd, sp, k, key0, key1, xy, th, best, o, s_sum, s_cnt);
}

__global__ __launch_bounds__(kPaperBlock) void paper_clear_bits_kernel(uint32_t *__restrict__ bits,
                                                                      int64_t n_words) {
    const int64_t i = (int64_t)blockIdx.x * kPaperBlock + threadIdx.x;
    if (i < n_words) bits[i] = 0u;
}

constexpr size_t kPaperAlign = 256;
// Frames of at most this many points and clusters take the one-launch path
// (when no inlier mask is requested and n_hyp <= 256).
constexpr int64_t kPaperFrameMaxPoints = 1 << 16;
constexpr int64_t kPaperFrameMaxClusters = 1 << 16;

size_t paper_align(size_t x) { return (x + kPaperAlign - 1) / kPaperAlign * kPaperAlign; }

struct PaperLayout {
    size_t xy, thresh, best_key, total;
};

PaperLayout paper_layout(int64_t n_clusters, int64_t n_points) {
    PaperLayout L;
    size_t at = 0;
    L.xy = at; at = paper_align(at + (size_t)n_points * sizeof(double2));
    L.thresh = at; at = paper_align(at + (size_t)n_clusters * sizeof(double));
    L.best_key = at; at = paper_align(at + (size_t)n_clusters * sizeof(unsigned long long));
    L.total = at;
    return L;
}

}  // namespace

extern "C" {

size_t rv_paper_workspace_bytes(int64_t n_clusters, int64_t n_points, int32_t n_hyp) {
    if (n_clusters < 0 || n_points < 0 || n_hyp < 0) return 0;
    return paper_layout(n_clusters, n_points).total;
}

int rv_estimate_velocity_paper(const float *theta, const float *vd, const int32_t *cluster_offsets,
                               int64_t n_clusters, int64_t n_points, int32_t n_hyp, uint64_t seed,
                               float *vx, float *vy, float *heading, int32_t *n_inliers,
                               uint8_t *status, double *thresh, uint32_t *inlier_bits,
                               int32_t *hyp_counts, int32_t *best_hyp, void *workspace,
                               size_t workspace_bytes, void *stream) {
    g_error[0] = '\0';
    if (n_hyp < 1 || n_hyp > RV_MAX_HYP)
        return fail(RV_ERR_INVALID_ARG, "n_hyp must be in [1, %d]", RV_MAX_HYP);
    if (n_clusters < 0 || n_clusters > INT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "n_clusters must be in [0, 2^31 - 1]");
    if (n_points < 0 || n_points > INT32_MAX)
        return fail(RV_ERR_INVALID_ARG, "n_points must be in [0, 2^31 - 1]");
    if (cluster_offsets == nullptr) return fail(RV_ERR_INVALID_ARG, "cluster_offsets is NULL");
    if (n_points > 0 && (theta == nullptr || vd == nullptr))
        return fail(RV_ERR_INVALID_ARG, "theta or vd is NULL");
    if (n_clusters > 0 && (vx == nullptr || vy == nullptr || heading == nullptr ||
                           n_inliers == nullptr || status == nullptr))
        return fail(RV_ERR_INVALID_ARG, "a required output is NULL");
    const PaperLayout L = paper_layout(n_clusters, n_points);
    if (workspace == nullptr || workspace_bytes < L.total)
        return fail(RV_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.total,
                    workspace == nullptr ? (size_t)0 : workspace_bytes);
    if (((uintptr_t)workspace % kPaperAlign) != 0)
        return fail(RV_ERR_WORKSPACE, "workspace must be %zu-byte aligned", kPaperAlign);
    if (n_clusters == 0) return RV_OK;
    const int64_t bpc = ((int64_t)n_hyp + kPaperBlock - 1) / kPaperBlock;
    if (n_clusters * bpc > INT32_MAX) return fail(RV_ERR_INVALID_ARG, "n_clusters * n_hyp too large");
    char *ws = (char *)workspace;
    double2 *xy = (double2 *)(ws + L.xy);
    double *th = thresh != nullptr ? thresh : (double *)(ws + L.thresh);
    unsigned long long *best_key = (unsigned long long *)(ws + L.best_key);
    const uint32_t key0 = (uint32_t)(seed & 0xFFFFFFFFu), key1 = (uint32_t)(seed >> 32);
    hipStream_t st = (hipStream_t)stream;
    PaperOutputs o;
    o.vx = vx;
    o.vy = vy;
    o.heading = heading;
    o.n_inliers = n_inliers;
    o.status = status;
    o.best = best_hyp;
    o.bits = inlier_bits;
    // Stage events (rv_stage_timing): stats and mask clearing, scoring, refit;
    // the one-launch path counts wholly as scoring.
    TimedCall tc;
    const bool timed = take_timed_call(tc);
    if (timed) (void)hipEventRecord(tc.ev[0], st);
    if (inlier_bits == nullptr && n_hyp <= kPaperBlock && n_points <= kPaperFrameMaxPoints &&
        n_clusters <= kPaperFrameMaxClusters) {
        if (timed) (void)hipEventRecord(tc.ev[1], st);
        hipLaunchKernelGGL(paper_frame_kernel, dim3((unsigned)n_clusters), dim3(kPaperBlock), 0, st,
                           theta, vd, cluster_offsets, n_points, n_hyp, key0, key1, xy, th,
                           hyp_counts, o);
        if (timed) {
            (void)hipEventRecord(tc.ev[2], st);
            (void)hipEventRecord(tc.ev[3], st);
            keep_timed_call(tc);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(RV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
        return RV_OK;
    }
    if (inlier_bits != nullptr) {
        const int64_t n_words = (n_points + 31) / 32;
        if (n_words > 0)
            hipLaunchKernelGGL(paper_clear_bits_kernel,
                               dim3((unsigned)((n_words + kPaperBlock - 1) / kPaperBlock)),
                               dim3(kPaperBlock), 0, st, inlier_bits, n_words);
    }
    hipLaunchKernelGGL(paper_stats_kernel, dim3((unsigned)n_clusters), dim3(kPaperBlock), 0, st,
                       theta, vd, cluster_offsets, n_points, xy, th, best_key);
    if (timed) (void)hipEventRecord(tc.ev[1], st);
    hipLaunchKernelGGL(paper_score_kernel, dim3((unsigned)(n_clusters * bpc)), dim3(kPaperBlock), 0,
                       st, theta, cluster_offsets, n_points, n_hyp, (int32_t)bpc, key0, key1,
                       (const double2 *)xy, (const double *)th, best_key, hyp_counts);
    if (timed) (void)hipEventRecord(tc.ev[2], st);
    hipLaunchKernelGGL(paper_refit_kernel, dim3((unsigned)n_clusters), dim3(kPaperBlock), 0, st,
                       theta, vd, cluster_offsets, n_points, key0, key1, (const double2 *)xy,
                       (const double *)th, (const unsigned long long *)best_key, o);
    if (timed) {
        (void)hipEventRecord(tc.ev[3], st);
        keep_timed_call(tc);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RV_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return RV_OK;
}

}  // extern "C"
