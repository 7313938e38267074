/*
 * rv_oracle_paper.c -- plain FP64 CPU oracle of the paper-literal variant of
 * the RANSAC inlier kernel (Sec. 3.1, Alg. 1, Eq. 5) followed by the
 * least-squares kernel (Sec. 3.2, Eq. 7, Alg. 2, Eq. 8).
 *
 * TEST INFRASTRUCTURE ONLY, like rv_oracle.c: only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the GPU path shares
 * nothing with it.
 *
 * Per cluster k (points [off[k], off[k+1]); a point with a non-finite azimuth
 * or Doppler value takes no part in any step):
 *   1. normalise (Alg. 1's normalize(), unspecified in the paper; read as a
 *      per-cluster min-max map of each coordinate onto [0, 1]):
 *        x = (theta - theta_min) / (theta_max - theta_min),
 *        y = (v_d - v_min) / (v_max - v_min),
 *      a coordinate whose span is zero maps to 0;
 *   2. threshold (Eq. 5, read as the median absolute deviation that the text
 *      names): med = median(y), thresh = median(|y - med|); the median of an
 *      even count is the mean (a + b) / 2 of the two middle values;
 *   3. hypothesis h: the seed pair (i, j) drawn exactly as in rv_oracle.c
 *      (Philox4x32-10, key = seed, counter = (h, k, 0, 0)); it is invalid when
 *      |theta_j - theta_i| < 1e-3 rad; otherwise the line through the two
 *      normalised seeds: m = (y_j - y_i) / (x_j - x_i), c = y_i - m x_i;
 *   4. distance of a point, as Alg. 1 writes it with aa = -m, bb = 1, cc = -c:
 *        distn = (aa x + bb y) + cc,  distd = sqrt(aa^2 + bb^2),
 *        dist = |distn / distd|;
 *      the point is an inlier when dist <= thresh (Alg. 1's test);
 *   5. the valid hypothesis with the most inliers is kept (ties: lowest h);
 *   6. least squares on its inliers as in rv_oracle.c (normal equations of
 *      v_d = vx cos(theta) + vy sin(theta)), heading = atan2(vy, vx).
 *
 * Arithmetic: every step in FP64 exactly as written (compile with
 * -ffp-contract=off, no fast-math); cos/sin are the host libm's.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void oracle_draw_pair(uint64_t seed, uint32_t h, uint32_t k, int64_t n, int64_t *i, int64_t *j);

enum {
    PO_OK = 0,
    PO_TOO_FEW_POINTS = 1,
    PO_ALL_DEGENERATE = 2,
    PO_SINGULAR_REFIT = 3,
    PO_BAD_OFFSETS = 4,
};

static const double PO_MIN_SEED_SEPARATION = 1e-3;

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Median of n >= 1 values (sorted in place). */
double oracle_median(double *v, int64_t n)
{
    qsort(v, (size_t)n, sizeof(double), cmp_double);
    if (n % 2 == 1)
        return v[n / 2];
    return (v[n / 2 - 1] + v[n / 2]) / 2.0;
}

/* The min-max normalisation of step 1 for one coordinate. */
static void normalise(const float *a, const uint8_t *ok, int64_t n, double *out)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t p = 0; p < n; ++p) {
        if (!ok[p])
            continue;
        double t = (double)a[p];
        if (t < lo) lo = t;
        if (t > hi) hi = t;
    }
    double span = hi - lo;
    for (int64_t p = 0; p < n; ++p)
        out[p] = !ok[p] ? NAN : (span > 0.0 ? ((double)a[p] - lo) / span : 0.0);
}

/* Line of hypothesis h through normalised seeds i, j (step 3). */
struct line {
    double m, c, distd;
};

static struct line make_line(const double *x, const double *y, int64_t i, int64_t j)
{
    struct line L;
    L.m = (y[j] - y[i]) / (x[j] - x[i]);
    L.c = y[i] - L.m * x[i];
    double aa = -L.m, bb = 1.0;
    L.distd = sqrt(aa * aa + bb * bb);
    return L;
}

/* Step 4: Alg. 1's perpendicular distance. */
static double line_distance(const struct line *L, double x, double y)
{
    double aa = -L->m, bb = 1.0, cc = -L->c;
    double distn = (aa * x + bb * y) + cc;
    return fabs(distn / L->distd);
}

/*
 * The paper-literal estimate of every cluster.  Arrays sized n_clusters:
 * vx, vy, heading, thresh (FP64), n_inliers, status, best_hyp; inlier_mask
 * (n_points bytes) and the per-hypothesis arrays hyp_valid, hyp_count
 * (n_clusters * n_hyp) are nullable.  Returns 0, or -1 for bad arguments.
 */
int oracle_estimate_velocity_paper(const float *theta, const float *vd, const int32_t *offsets,
                                   int64_t n_clusters, int64_t n_points, int32_t n_hyp,
                                   uint64_t seed, double *vx, double *vy, double *heading,
                                   double *thresh, int32_t *n_inliers, uint8_t *status,
                                   int32_t *best_hyp, uint8_t *inlier_mask, uint8_t *hyp_valid,
                                   int32_t *hyp_count)
{
    if (n_clusters < 0 || n_points < 0 || n_hyp < 1 || offsets == NULL)
        return -1;
    if (inlier_mask)
        memset(inlier_mask, 0, (size_t)n_points);
    for (int64_t k = 0; k < n_clusters; ++k) {
        int64_t lo = offsets[k], hi = offsets[k + 1];
        vx[k] = vy[k] = heading[k] = NAN;
        thresh[k] = NAN;
        n_inliers[k] = 0;
        best_hyp[k] = -1;
        if (hyp_valid) memset(hyp_valid + k * n_hyp, 0, (size_t)n_hyp);
        if (hyp_count) for (int32_t h = 0; h < n_hyp; ++h) hyp_count[k * n_hyp + h] = 0;
        if (lo < 0 || hi < lo || hi > n_points) {
            status[k] = PO_BAD_OFFSETS;
            continue;
        }
        int64_t n = hi - lo;
        const float *th = theta + lo, *v = vd + lo;
        uint8_t *ok = malloc((size_t)(n > 0 ? n : 1));
        double *x = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double *y = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double *work = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        int64_t m_ok = 0;
        for (int64_t p = 0; p < n; ++p) {
            ok[p] = isfinite(th[p]) && isfinite(v[p]);
            m_ok += ok[p];
        }
        if (n < 2) {
            status[k] = PO_TOO_FEW_POINTS;
            goto next;
        }
        normalise(th, ok, n, x);
        normalise(v, ok, n, y);
        if (m_ok > 0) {
            int64_t w = 0;
            for (int64_t p = 0; p < n; ++p)
                if (ok[p]) work[w++] = y[p];
            double med = oracle_median(work, w);
            w = 0;
            for (int64_t p = 0; p < n; ++p)
                if (ok[p]) work[w++] = fabs(y[p] - med);
            thresh[k] = oracle_median(work, w);
        }
        {
            int64_t best = -1, best_count = -1;
            for (int32_t h = 0; h < n_hyp; ++h) {
                int64_t i, j;
                oracle_draw_pair(seed, (uint32_t)h, (uint32_t)k, n, &i, &j);
                int valid = ok[i] && ok[j] &&
                            fabs((double)th[j] - (double)th[i]) >= PO_MIN_SEED_SEPARATION;
                if (!valid)
                    continue;
                struct line L = make_line(x, y, i, j);
                int64_t count = 0;
                for (int64_t p = 0; p < n; ++p)
                    if (ok[p] && line_distance(&L, x[p], y[p]) <= thresh[k])
                        count += 1;
                if (hyp_valid) hyp_valid[k * n_hyp + h] = 1;
                if (hyp_count) hyp_count[k * n_hyp + h] = (int32_t)count;
                if (count > best_count) {
                    best_count = count;
                    best = h;
                }
            }
            if (best < 0) {
                status[k] = PO_ALL_DEGENERATE;
                goto next;
            }
            best_hyp[k] = (int32_t)best;
            int64_t i, j;
            oracle_draw_pair(seed, (uint32_t)best, (uint32_t)k, n, &i, &j);
            struct line L = make_line(x, y, i, j);
            double scc = 0.0, scs = 0.0, sss = 0.0, scv = 0.0, ssv = 0.0;
            int64_t n_in = 0;
            for (int64_t p = 0; p < n; ++p) {
                if (!ok[p] || !(line_distance(&L, x[p], y[p]) <= thresh[k]))
                    continue;
                if (inlier_mask) inlier_mask[lo + p] = 1;
                n_in += 1;
                double t = (double)th[p], c = cos(t), s = sin(t), dv = (double)v[p];
                scc += c * c;
                scs += c * s;
                sss += s * s;
                scv += c * dv;
                ssv += s * dv;
            }
            n_inliers[k] = (int32_t)n_in;
            double det = scc * sss - scs * scs;
            if (n_in < 2 || !(det > 0.0)) {
                status[k] = PO_SINGULAR_REFIT;
                goto next;
            }
            vx[k] = (sss * scv - scs * ssv) / det;
            vy[k] = (scc * ssv - scs * scv) / det;
            heading[k] = atan2(vy[k], vx[k]);
            status[k] = PO_OK;
        }
    next:
        free(ok);
        free(x);
        free(y);
        free(work);
    }
    return 0;
}

/* Step 4 alone, for tests: Alg. 1's distance of (px, py) to the line through
   (x1, y1) and (x2, y2). */
double oracle_paper_line_distance(double x1, double y1, double x2, double y2, double px, double py)
{
    double xs[2] = {x1, x2}, ys[2] = {y1, y2};
    struct line L = make_line(xs, ys, 0, 1);
    return line_distance(&L, px, py);
}
