/*
 * rv_oracle.c -- plain, slow, FP64 CPU oracle of the per-cluster velocity and
 * heading estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The estimator itself
 * never calls it; it shares no code, header or table with the GPU path.
 *
 * What it computes, per cluster k of a CSR frame (points [off[k], off[k+1])):
 *
 *   Sec. 3.1 (Alg. 1, parallel RANSAC), as the velocity-profile variant:
 *     - a hypothesis h is a pair of distinct seed points (i, j) of the cluster,
 *       drawn from the counter-based generator Philox4x32-10 (Salmon et al.,
 *       SC'11) with key = seed and counter = (h, k, 0, 0);
 *     - the pair fixes (vx_h, vy_h) by solving the 2x2 system of Eq. 6 written
 *       for the two seeds (Cramer's rule);
 *     - every point of the cluster is scored: it is an inlier of h when its
 *       residual |v_d - vx_h cos(theta) - vy_h sin(theta)| is below tau;
 *     - the hypothesis with the most inliers is kept (ties: lowest h).
 *   Sec. 3.2 (Eq. 7, Alg. 2, least-squares kernel):
 *     - (vx, vy) = A^+ v_r on the kept hypothesis's inliers, A having rows
 *       (cos theta, sin theta); A^+ is the Moore-Penrose pseudoinverse, i.e. the
 *       least-squares solution, computed from the 2x2 normal equations;
 *   Eq. 8 / Alg. 2:
 *     - heading = atan2(vy, vx), the quadrant-correct form of arctan(vy/vx).
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes):  the inner model is the velocity profile of Eq. 6 rather than
 * Alg. 1's normalised line fit; tau is one fixed value per call; the inlier
 * test is strict (<); a pair is degenerate when |theta_j - theta_i| < 1e-3 rad
 * and such a hypothesis never wins; a point with a non-finite azimuth or
 * Doppler value is never an inlier; clusters with fewer than two points, with
 * no valid hypothesis, or with a singular refit get a status flag and NaN
 * outputs.
 *
 * Arithmetic: inputs are float32 and are promoted exactly to double; cos/sin
 * are the host libm's; tau is promoted from its float32 value.  Compile with
 * -ffp-contract=off and without fast-math so every expression is evaluated as
 * written.
 *
 * Per-hypothesis tolerance bands (test aid): count_lo / count_hi count points
 * with |r| < tau - w and |r| < tau + w, where for hypothesis h and point p
 *   w = max(band_abs, band_rel * (|v_p| + tau + 3|vx_h cos| + 3|vy_h sin|)).
 * A float32 evaluation of the residual lands between the two counts when its
 * error is below w.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- status codes (per cluster) ---------------------------------------- */
enum {
    OR_CLUSTER_OK = 0,
    OR_CLUSTER_TOO_FEW_POINTS = 1,
    OR_CLUSTER_ALL_DEGENERATE = 2,
    OR_CLUSTER_SINGULAR_REFIT = 3,
    OR_CLUSTER_BAD_OFFSETS = 4,
};

/* Minimum azimuth separation of a valid seed pair, radians. */
static const double MIN_SEED_SEPARATION = 1e-3;

/* ---- Philox4x32-10 ------------------------------------------------------
 * Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11.  State: four 32-bit counter words and two 32-bit key words.  One
 * round multiplies counter words 0 and 2 by the two round multipliers (full
 * 64-bit products), and the new counter is
 *   (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)).
 * Between rounds the key is advanced by the two Weyl constants.  Ten rounds.
 */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ---- seed pair of a hypothesis (Alg. 1: two random indices per trial) ----
 * First index: floor(u0 * n / 2^32).  Second: floor(u1 * (n-1) / 2^32), then
 * shifted up by one when it is at or above the first, so the two differ.
 */
void oracle_map_pair(uint32_t u0, uint32_t u1, int64_t n, int64_t *i, int64_t *j)
{
    uint64_t a = ((uint64_t)u0 * (uint64_t)n) >> 32;
    uint64_t b = ((uint64_t)u1 * (uint64_t)(n - 1)) >> 32;
    if (b >= a)
        b = b + 1;
    *i = (int64_t)a;
    *j = (int64_t)b;
}

void oracle_draw_pair(uint64_t seed, uint32_t h, uint32_t k, int64_t n, int64_t *i, int64_t *j)
{
    uint32_t ctr[4] = {h, k, 0u, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t u[4];
    oracle_philox4x32_10(ctr, key, u);
    oracle_map_pair(u[0], u[1], n, i, j);
}

/* ---- one frame ----------------------------------------------------------- */
struct job {
    const float *theta, *vd;
    const int32_t *offsets;
    int64_t n_clusters, n_points;
    int32_t n_hyp;
    double tau;
    uint64_t seed;
    const int64_t *cluster_ids;  /* NULL: result r is cluster r */
    int64_t n_results;
    double near_window, band_abs, band_rel;
    double *vx, *vy, *heading;
    int32_t *n_inliers, *n_near_tau, *best_hyp;
    uint8_t *status;
    uint8_t *inlier_mask;
    uint8_t *hyp_valid;
    int32_t *hyp_i, *hyp_j;
    double *hyp_vx, *hyp_vy;
    int32_t *hyp_count, *hyp_count_lo, *hyp_count_hi;
    /* work distribution: results in order of decreasing cluster size */
    int64_t *schedule;
    int64_t next;  /* next schedule slot, taken atomically */
    pthread_mutex_t lock;
};

static void fill_failed(struct job *J, int64_t r, uint8_t st)
{
    J->vx[r] = NAN;
    J->vy[r] = NAN;
    J->heading[r] = NAN;
    J->n_inliers[r] = 0;
    J->status[r] = st;
    if (J->n_near_tau) J->n_near_tau[r] = 0;
    if (J->best_hyp) J->best_hyp[r] = -1;
}

static int64_t cluster_of(const struct job *J, int64_t r)
{
    return J->cluster_ids ? J->cluster_ids[r] : r;
}

/* Bounds of cluster k; returns 0 when its offsets are inconsistent. */
static int cluster_bounds(const struct job *J, int64_t k, int64_t *lo, int64_t *hi)
{
    int64_t a = J->offsets[k], b = J->offsets[k + 1];
    if (a < 0 || b < a || b > J->n_points)
        return 0;
    *lo = a;
    *hi = b;
    return 1;
}

/* Result of the least-squares refit of one cluster. */
struct fit {
    double vx, vy, heading;
    int32_t n_inliers, n_near;
    uint8_t status;
};

/* Normal-equation sums of the least-squares refit (Sec. 3.2, Eq. 7):
   A^T A = [[scc, scs], [scs, sss]] and A^T v_d = (scv, ssv). */
struct sums {
    double scc, scs, sss, scv, ssv;
};

static void add_point(struct sums *S, double c, double s, double v)
{
    S->scc += c * c;
    S->scs += c * s;
    S->sss += s * s;
    S->scv += c * v;
    S->ssv += s * v;
}

/* Solves the 2x2 normal equations and takes the heading (Eq. 8, atan2). */
static void solve_sums(const struct sums *S, int64_t n_in, struct fit *f)
{
    double det = S->scc * S->sss - S->scs * S->scs;
    if (n_in < 2 || !(det > 0.0)) {
        f->vx = NAN;
        f->vy = NAN;
        f->heading = NAN;
        f->status = OR_CLUSTER_SINGULAR_REFIT;
        return;
    }
    f->vx = (S->sss * S->scv - S->scs * S->ssv) / det;
    f->vy = (S->scc * S->ssv - S->scs * S->scv) / det;
    f->heading = atan2(f->vy, f->vx);
    f->status = OR_CLUSTER_OK;
}

/*
 * Least-squares refit on the inliers of hypothesis (hvx, hvy) (Sec. 3.2,
 * Eq. 7, Alg. 2): every finite point with |v_d - hvx cos - hvy sin| < tau
 * joins the inlier set, the normal equations (A^T A) v = A^T v_d are summed
 * over it and solved, and the heading is atan2(vy, vx) (Eq. 8).  mask and
 * near_mask (n bytes each, nullable) receive the inlier set and the points
 * within near_window of tau.
 */
static void refit(const float *vd, const double *c, const double *s, const uint8_t *ok,
                  int64_t n, double hvx, double hvy, double tau, double near_window,
                  uint8_t *mask, uint8_t *near_mask, struct fit *f)
{
    struct sums S = {0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t n_in = 0, n_near = 0;
    for (int64_t p = 0; p < n; ++p) {
        if (mask) mask[p] = 0;
        if (near_mask) near_mask[p] = 0;
        if (!ok[p])
            continue;
        double v = (double)vd[p];
        double res = fabs(v - hvx * c[p] - hvy * s[p]);
        if (fabs(res - tau) <= near_window) {
            n_near += 1;
            if (near_mask) near_mask[p] = 1;
        }
        if (!(res < tau))
            continue;
        n_in += 1;
        if (mask) mask[p] = 1;
        add_point(&S, c[p], s[p], v);
    }
    f->n_inliers = (int32_t)n_in;
    f->n_near = (int32_t)n_near;
    solve_sums(&S, n_in, f);
}

static void estimate_cluster(struct job *J, int64_t r, double *c, double *s, uint8_t *ok)
{
    int64_t k = cluster_of(J, r);
    int64_t H = J->n_hyp;
    int64_t lo, hi;
    double tau = J->tau;

    /* Debug arrays start as "invalid" so early exits leave them defined. */
    for (int64_t h = 0; h < H; ++h) {
        int64_t q = r * H + h;
        if (J->hyp_valid) J->hyp_valid[q] = 0;
        if (J->hyp_i) J->hyp_i[q] = -1;
        if (J->hyp_j) J->hyp_j[q] = -1;
        if (J->hyp_vx) J->hyp_vx[q] = NAN;
        if (J->hyp_vy) J->hyp_vy[q] = NAN;
        if (J->hyp_count) J->hyp_count[q] = 0;
        if (J->hyp_count_lo) J->hyp_count_lo[q] = 0;
        if (J->hyp_count_hi) J->hyp_count_hi[q] = 0;
    }

    if (!cluster_bounds(J, k, &lo, &hi)) {
        fill_failed(J, r, OR_CLUSTER_BAD_OFFSETS);
        return;
    }
    int64_t n = hi - lo;
    const float *th = J->theta + lo;
    const float *vd = J->vd + lo;
    if (J->inlier_mask)
        memset(J->inlier_mask + lo, 0, (size_t)n);
    if (n < 2) {
        fill_failed(J, r, OR_CLUSTER_TOO_FEW_POINTS);
        return;
    }

    /* The rows (cos theta, sin theta) of the design matrix A (Sec. 3.2). */
    for (int64_t p = 0; p < n; ++p) {
        double t = (double)th[p];
        c[p] = cos(t);
        s[p] = sin(t);
        ok[p] = isfinite(th[p]) && isfinite(vd[p]);
    }

    /* RANSAC trials (Sec. 3.1, Alg. 1). */
    int64_t best_h = -1;
    int64_t best_count = -1;
    double best_vx = 0.0, best_vy = 0.0;
    for (int64_t h = 0; h < H; ++h) {
        int64_t i, j;
        oracle_draw_pair(J->seed, (uint32_t)h, (uint32_t)k, n, &i, &j);
        int valid = ok[i] && ok[j] &&
                    fabs((double)th[j] - (double)th[i]) >= MIN_SEED_SEPARATION;
        int64_t q = r * H + h;
        if (J->hyp_i) J->hyp_i[q] = (int32_t)i;
        if (J->hyp_j) J->hyp_j[q] = (int32_t)j;
        if (!valid)
            continue;

        /* Eq. 6 for the two seeds, solved by Cramer's rule. */
        double vi = (double)vd[i], vj = (double)vd[j];
        double det = c[i] * s[j] - s[i] * c[j];
        double hvx = (vi * s[j] - vj * s[i]) / det;
        double hvy = (c[i] * vj - c[j] * vi) / det;

        /* Score every point of the cluster. */
        int64_t count = 0, count_lo = 0, count_hi = 0;
        for (int64_t p = 0; p < n; ++p) {
            if (!ok[p])
                continue;
            double v = (double)vd[p];
            double res = fabs(v - hvx * c[p] - hvy * s[p]);
            if (res < tau)
                count += 1;
            if (J->hyp_count_lo || J->hyp_count_hi) {
                double w = J->band_rel * (fabs(v) + tau + 3.0 * fabs(hvx * c[p]) +
                                          3.0 * fabs(hvy * s[p]));
                if (w < J->band_abs)
                    w = J->band_abs;
                if (res < tau - w)
                    count_lo += 1;
                if (res < tau + w)
                    count_hi += 1;
            }
        }
        if (J->hyp_valid) J->hyp_valid[q] = 1;
        if (J->hyp_vx) J->hyp_vx[q] = hvx;
        if (J->hyp_vy) J->hyp_vy[q] = hvy;
        if (J->hyp_count) J->hyp_count[q] = (int32_t)count;
        if (J->hyp_count_lo) J->hyp_count_lo[q] = (int32_t)count_lo;
        if (J->hyp_count_hi) J->hyp_count_hi[q] = (int32_t)count_hi;

        /* The trial with the most inliers is kept; the first one wins ties. */
        if (count > best_count) {
            best_count = count;
            best_h = h;
            best_vx = hvx;
            best_vy = hvy;
        }
    }
    if (J->best_hyp) J->best_hyp[r] = (int32_t)best_h;
    if (best_h < 0) {
        fill_failed(J, r, OR_CLUSTER_ALL_DEGENERATE);
        return;
    }

    struct fit f;
    refit(J->vd + lo, c, s, ok, n, best_vx, best_vy, tau, J->near_window,
          J->inlier_mask ? J->inlier_mask + lo : NULL, NULL, &f);
    J->vx[r] = f.vx;
    J->vy[r] = f.vy;
    J->heading[r] = f.heading;
    J->n_inliers[r] = f.n_inliers;
    J->status[r] = f.status;
    if (J->n_near_tau) J->n_near_tau[r] = f.n_near;
}

static int64_t cluster_size(const struct job *J, int64_t r)
{
    int64_t lo, hi, k = cluster_of(J, r);
    return cluster_bounds(J, k, &lo, &hi) ? hi - lo : 0;
}

static const struct job *sort_job;  /* qsort has no context argument */

static int by_size_desc(const void *a, const void *b)
{
    int64_t ra = *(const int64_t *)a, rb = *(const int64_t *)b;
    int64_t na = cluster_size(sort_job, ra), nb = cluster_size(sort_job, rb);
    if (na != nb)
        return na > nb ? -1 : 1;
    return ra < rb ? -1 : (ra > rb);
}

static void *worker(void *arg)
{
    struct job *J = (struct job *)arg;
    int64_t cap = 0;
    double *c = NULL, *s = NULL;
    uint8_t *ok = NULL;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t slot = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (slot >= J->n_results)
            break;
        int64_t r = J->schedule[slot];
        int64_t n = cluster_size(J, r);
        if (n > cap) {
            cap = n;
            free(c); free(s); free(ok);
            c = (double *)malloc((size_t)cap * sizeof(double));
            s = (double *)malloc((size_t)cap * sizeof(double));
            ok = (uint8_t *)malloc((size_t)cap);
        }
        estimate_cluster(J, r, c, s, ok);
    }
    free(c); free(s); free(ok);
    return NULL;
}

/*
 * Estimate (vx, vy, heading) for every listed cluster.  All pointers are host
 * memory.  Per-result arrays have n_results entries (n_results = n_ids when
 * cluster_ids is given, else n_clusters); per-hypothesis arrays have
 * n_results * n_hyp entries; inlier_mask has n_points entries (only the
 * listed clusters' points are written).  Nullable: cluster_ids, n_near_tau,
 * best_hyp, inlier_mask and every hyp_* array.
 * Returns 0, or -1 for invalid arguments.
 */
int oracle_estimate_velocity(
    const float *theta, const float *vd, const int32_t *offsets,
    int64_t n_clusters, int64_t n_points, int32_t n_hyp, float tau, uint64_t seed,
    const int64_t *cluster_ids, int64_t n_ids,
    double near_window, double band_abs, double band_rel,
    double *vx, double *vy, double *heading, int32_t *n_inliers, uint8_t *status,
    int32_t *n_near_tau, int32_t *best_hyp, uint8_t *inlier_mask,
    uint8_t *hyp_valid, int32_t *hyp_i, int32_t *hyp_j, double *hyp_vx, double *hyp_vy,
    int32_t *hyp_count, int32_t *hyp_count_lo, int32_t *hyp_count_hi,
    int n_threads)
{
    if (n_clusters < 0 || n_points < 0 || n_hyp < 1 || !(tau > 0.0f) || !isfinite(tau))
        return -1;
    if (!offsets || !vx || !vy || !heading || !n_inliers || !status)
        return -1;
    if (n_points > 0 && (!theta || !vd))
        return -1;
    int64_t n_results = cluster_ids ? n_ids : n_clusters;
    if (n_results < 0)
        return -1;
    if (cluster_ids)
        for (int64_t r = 0; r < n_ids; ++r)
            if (cluster_ids[r] < 0 || cluster_ids[r] >= n_clusters)
                return -1;

    struct job J;
    memset(&J, 0, sizeof J);
    J.theta = theta; J.vd = vd; J.offsets = offsets;
    J.n_clusters = n_clusters; J.n_points = n_points; J.n_hyp = n_hyp;
    J.tau = (double)tau; J.seed = seed;
    J.cluster_ids = cluster_ids; J.n_results = n_results;
    J.near_window = near_window; J.band_abs = band_abs; J.band_rel = band_rel;
    J.vx = vx; J.vy = vy; J.heading = heading; J.n_inliers = n_inliers;
    J.status = status; J.n_near_tau = n_near_tau; J.best_hyp = best_hyp;
    J.inlier_mask = inlier_mask;
    J.hyp_valid = hyp_valid; J.hyp_i = hyp_i; J.hyp_j = hyp_j;
    J.hyp_vx = hyp_vx; J.hyp_vy = hyp_vy;
    J.hyp_count = hyp_count; J.hyp_count_lo = hyp_count_lo; J.hyp_count_hi = hyp_count_hi;
    if (n_results == 0)
        return 0;

    J.schedule = (int64_t *)malloc((size_t)n_results * sizeof(int64_t));
    for (int64_t r = 0; r < n_results; ++r)
        J.schedule[r] = r;
    sort_job = &J;
    qsort(J.schedule, (size_t)n_results, sizeof(int64_t), by_size_desc);
    pthread_mutex_init(&J.lock, NULL);

    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > 256)
        n_threads = 256;
    pthread_t tids[256];
    int started = 0;
    for (int t = 1; t < n_threads; ++t)
        if (pthread_create(&tids[started], NULL, worker, &J) == 0)
            started += 1;
    worker(&J);
    for (int t = 0; t < started; ++t)
        pthread_join(tids[t], NULL);

    pthread_mutex_destroy(&J.lock);
    free(J.schedule);
    return 0;
}

/*
 * Exhaustive search over every unordered valid pair of one cluster (test aid
 * for small clusters).  best_pairs (n*n bytes, nullable) marks each pair (i, j)
 * whose hypothesis reaches the best count, in both orders.  Returns the best
 * count, or -1 when no pair is valid.
 */
int32_t oracle_all_pairs_best(const float *theta, const float *vd, int32_t n, float tau,
                              uint8_t *best_pairs, int32_t *pair_count)
{
    double t64 = (double)tau;
    double *c = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *s = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    uint8_t *ok = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    for (int32_t p = 0; p < n; ++p) {
        c[p] = cos((double)theta[p]);
        s[p] = sin((double)theta[p]);
        ok[p] = isfinite(theta[p]) && isfinite(vd[p]);
    }
    int32_t best = -1;
    for (int pass = 0; pass < 2; ++pass) {
        for (int32_t i = 0; i < n; ++i) {
            for (int32_t j = i + 1; j < n; ++j) {
                int32_t count = -1;
                if (ok[i] && ok[j] &&
                    fabs((double)theta[j] - (double)theta[i]) >= MIN_SEED_SEPARATION) {
                    double vi = (double)vd[i], vj = (double)vd[j];
                    double det = c[i] * s[j] - s[i] * c[j];
                    double hvx = (vi * s[j] - vj * s[i]) / det;
                    double hvy = (c[i] * vj - c[j] * vi) / det;
                    count = 0;
                    for (int32_t p = 0; p < n; ++p)
                        if (ok[p] && fabs((double)vd[p] - hvx * c[p] - hvy * s[p]) < t64)
                            count += 1;
                }
                if (pass == 0) {
                    if (count > best)
                        best = count;
                    if (pair_count) {
                        pair_count[i * n + j] = count;
                        pair_count[j * n + i] = count;
                    }
                } else if (best_pairs) {
                    uint8_t m = (count >= 0 && count == best) ? 1 : 0;
                    best_pairs[i * n + j] = m;
                    best_pairs[j * n + i] = m;
                }
            }
            if (pass == 1 && best_pairs)
                best_pairs[i * n + i] = 0;
        }
    }
    free(c); free(s); free(ok);
    return best;
}

/*
 * The steps after selection for a given hypothesis h of cluster k: its seed
 * pair and 2x2 solve, then the refit on its inliers.  Used to check a result
 * built on another hypothesis than the oracle's own choice.  mask and
 * near_mask have one byte per point of the cluster (nullable).  Returns 0, -1
 * for invalid arguments, or -2 when hypothesis h is degenerate.
 */
int oracle_fit_hypothesis(const float *theta, const float *vd, const int32_t *offsets,
                          int64_t n_clusters, int64_t n_points, float tau, uint64_t seed,
                          int64_t k, int64_t h, double near_window, double *vx, double *vy,
                          double *heading, int32_t *n_inliers, int32_t *n_near, uint8_t *status,
                          uint8_t *mask, uint8_t *near_mask)
{
    if (k < 0 || k >= n_clusters || h < 0 || h > 0xFFFFFFFFLL || !(tau > 0.0f))
        return -1;
    int64_t lo = offsets[k], hi = offsets[k + 1];
    if (lo < 0 || hi < lo || hi > n_points || hi - lo < 2)
        return -1;
    int64_t n = hi - lo;
    const float *th = theta + lo;
    const float *v = vd + lo;
    double *c = (double *)malloc((size_t)n * sizeof(double));
    double *s = (double *)malloc((size_t)n * sizeof(double));
    uint8_t *ok = (uint8_t *)malloc((size_t)n);
    for (int64_t p = 0; p < n; ++p) {
        c[p] = cos((double)th[p]);
        s[p] = sin((double)th[p]);
        ok[p] = isfinite(th[p]) && isfinite(v[p]);
    }
    int64_t i, j;
    oracle_draw_pair(seed, (uint32_t)h, (uint32_t)k, n, &i, &j);
    int rc = 0;
    if (!(ok[i] && ok[j] && fabs((double)th[j] - (double)th[i]) >= MIN_SEED_SEPARATION)) {
        rc = -2;
    } else {
        double vi = (double)v[i], vj = (double)v[j];
        double det = c[i] * s[j] - s[i] * c[j];
        double hvx = (vi * s[j] - vj * s[i]) / det;
        double hvy = (c[i] * vj - c[j] * vi) / det;
        struct fit f;
        refit(v, c, s, ok, n, hvx, hvy, (double)tau, near_window, mask, near_mask, &f);
        *vx = f.vx;
        *vy = f.vy;
        *heading = f.heading;
        *n_inliers = f.n_inliers;
        *n_near = f.n_near;
        *status = f.status;
    }
    free(c); free(s); free(ok);
    return rc;
}

/*
 * Least-squares refit (Sec. 3.2, Eq. 7, Alg. 2) and heading (Eq. 8) of one
 * cluster of n points on a GIVEN inlier set: point p is used when mask[p] is
 * nonzero and its azimuth and Doppler value are finite.  The sums run in point
 * order, as in the oracle's own refit, so on the oracle's own mask the result
 * is the same bit for bit.  Used to check a refit whose inlier set differs from
 * the oracle's classification at points within rounding of tau.  status is
 * OR_CLUSTER_OK or OR_CLUSTER_SINGULAR_REFIT.  Returns 0, or -1 for invalid
 * arguments.
 */
int oracle_refit_mask(const float *theta, const float *vd, const uint8_t *mask, int64_t n,
                      double *vx, double *vy, double *heading, int32_t *n_inliers,
                      uint8_t *status)
{
    if (n < 0 || (n > 0 && (!theta || !vd || !mask)) || !vx || !vy || !heading ||
        !n_inliers || !status)
        return -1;
    struct sums S = {0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t n_in = 0;
    for (int64_t p = 0; p < n; ++p) {
        if (!mask[p] || !isfinite(theta[p]) || !isfinite(vd[p]))
            continue;
        double t = (double)theta[p];
        n_in += 1;
        add_point(&S, cos(t), sin(t), (double)vd[p]);
    }
    struct fit f;
    solve_sums(&S, n_in, &f);
    *vx = f.vx;
    *vy = f.vy;
    *heading = f.heading;
    *n_inliers = (int32_t)n_in;
    *status = f.status;
    return 0;
}
