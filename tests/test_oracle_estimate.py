"""Pins of the oracle's estimator against closed forms, library routines and
invariants (CPU only).

The paper prints no accuracy values or worked example, so nothing here is a
paper number; every pin is something the mathematics fixes:
  * a hand-worked cluster with exact arithmetic (tests/golden/strict_tau_example.txt);
  * noise-free clusters: each hypothesis and the refit recover the truth within
    the error bound that float32 rounding of v_d implies (Cramer / least squares);
  * the refit equals numpy.linalg.lstsq and pinv (the paper's comparator) on
    the same inlier set, and the refit on a given inlier set equals the
    oracle's own refit on its mask (bitwise) and lstsq on other masks;
  * noise-free clusters with outliers: the inlier set is exactly the true one;
  * small clusters: RANSAC's best count equals an exhaustive all-pairs search;
  * rotation, power-of-two scaling, sign flip, reflection, batch independence;
  * degenerate and non-finite inputs;
  * statistics against ground truth, and sklearn's RANSACRegressor.
"""
import math
import os

import numpy as np
import pytest

from paper_2012_12618_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
U32 = 2.0**-24  # unit roundoff of float32


def _frame_from_clusters(clusters):
    """clusters: list of (theta array, vd array) -> (theta, vd, offsets)."""
    th = np.concatenate([np.asarray(c[0], dtype=np.float32) for c in clusters]) if clusters else np.zeros(0, np.float32)
    vd = np.concatenate([np.asarray(c[1], dtype=np.float32) for c in clusters]) if clusters else np.zeros(0, np.float32)
    off = np.zeros(len(clusters) + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(c[0]) for c in clusters])
    return th, vd, off


def _noiseless_cluster(rng, n, vx, vy, lo_deg=-60, hi_deg=60):
    th = np.deg2rad(rng.uniform(lo_deg, hi_deg, n)).astype(np.float32)
    t = th.astype(np.float64)
    vd = (vx * np.cos(t) + vy * np.sin(t)).astype(np.float32)
    return th, vd


def _read_golden(name):
    vals = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *rest = line.split()
            vals[key] = rest
    return vals


# --------------------------------------------------------------------------
# hand-worked example
# --------------------------------------------------------------------------
def test_strict_tau_worked_example(oracle_mod):
    g = _read_golden("strict_tau_example.txt")
    th = np.array([float(x) for x in g["theta"]], dtype=np.float32)
    vd = np.array([float(x) for x in g["vd"]], dtype=np.float32)
    tau = float(g["tau"][0])
    off = np.array([0, len(th)], dtype=np.int32)
    r = oracle_mod.estimate_velocity(th, vd, off, 64, tau, seed=7, debug=True)
    assert r.status[0] == oracle_mod.CLUSTER_OK
    assert r.n_inliers[0] == int(g["n_inliers"][0])
    assert list(r.inlier_mask) == [int(x) for x in g["inlier_mask"]]
    assert abs(r.vx[0] - float(g["vx"][0])) < 1e-14
    assert abs(r.vy[0] - math.tan(0.25)) < 1e-14
    assert abs(r.heading[0] - float(g["heading"][0])) < 1e-14
    assert r.n_near_tau[0] == int(g["n_near_tau"][0])
    # every valid hypothesis contains D (index 3) and scores 3 or 2
    valid = r.hyp_valid[0].astype(bool)
    assert valid.any()
    assert np.all((r.hyp_i[0][valid] == 3) | (r.hyp_j[0][valid] == 3))
    assert set(r.hyp_count[0][valid].tolist()) <= {2, 3}
    # the kept hypothesis is the first valid one with count 3
    first = int(np.flatnonzero(valid & (r.hyp_count[0] == 3))[0])
    assert r.best_hyp[0] == first


# --------------------------------------------------------------------------
# noise-free recovery (closed forms with the float32 input rounding bound)
# --------------------------------------------------------------------------
def test_noiseless_hypotheses_and_refit_recover_truth(oracle_mod):
    rng = np.random.default_rng(1)
    truths = [(12.5, -3.25), (-29.0, 17.0), (0.5, 0.0), (-7.0, -28.0), (30.0, 30.0)]
    clusters = [_noiseless_cluster(rng, n, vx, vy) for (vx, vy), n in zip(truths, [40, 100, 9, 250, 3])]
    th, vd, off = _frame_from_clusters(clusters)
    H = 200
    r = oracle_mod.estimate_velocity(th, vd, off, H, 0.15, seed=99, debug=True)
    for k, (vx, vy) in enumerate(truths):
        lo, hi = off[k], off[k + 1]
        t = th[lo:hi].astype(np.float64)
        v = vd[lo:hi].astype(np.float64)
        assert r.status[k] == oracle_mod.CLUSTER_OK
        assert r.n_inliers[k] == hi - lo            # every point is an inlier
        valid = r.hyp_valid[k].astype(bool)
        first_valid = int(np.flatnonzero(valid)[0])
        assert r.best_hyp[k] == first_valid         # all tie at n: lowest h wins
        assert np.all(r.hyp_count[k][valid] == hi - lo)
        # Cramer's rule with perturbed right-hand side: |dvx|, |dvy| <=
        # (|dv_i| + |dv_j|) / |sin(theta_j - theta_i)|, |dv| <= 2^-24 |v|.
        for h in np.flatnonzero(valid):
            i, j = r.hyp_i[k, h], r.hyp_j[k, h]
            bound = U32 * (abs(v[i]) + abs(v[j])) / abs(math.sin(t[j] - t[i])) * 1.01 + 1e-12
            assert abs(r.hyp_vx[k, h] - vx) <= bound
            assert abs(r.hyp_vy[k, h] - vy) <= bound
        # Least squares with perturbed data: |dx| <= ||A^+||_2 ||dv||_2.
        A = np.stack([np.cos(t), np.sin(t)], axis=1)
        dv = U32 * np.abs(v)
        bound = np.linalg.norm(np.linalg.pinv(A), 2) * np.linalg.norm(dv) * 1.01 + 1e-12
        assert math.hypot(r.vx[k] - vx, r.vy[k] - vy) <= bound
        assert abs(math.remainder(r.heading[k] - math.atan2(vy, vx), 2 * math.pi)) < 1e-5


def test_refit_on_a_given_mask(oracle_mod):
    # The refit on a caller's inlier set (used when a GPU mask differs from the
    # oracle's at points within rounding of tau): on the oracle's own mask it is
    # the oracle's refit bit for bit (same sums in the same order); on other
    # masks it equals numpy.linalg.lstsq; non-finite points are skipped; fewer
    # than two points or one azimuth only is singular.
    frame, H, tau = synth.make_workload("small")
    r = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=21)
    rng = np.random.default_rng(5)
    for k in range(frame.n_clusters):
        lo, hi = frame.offsets[k], frame.offsets[k + 1]
        th, vd = frame.theta[lo:hi], frame.vd[lo:hi]
        own = oracle_mod.refit_on_mask(th, vd, r.inlier_mask[lo:hi])
        assert own.n_inliers == r.n_inliers[k] and own.status == r.status[k]
        assert (own.vx, own.vy, own.heading) == (r.vx[k], r.vy[k], r.heading[k])
        m = rng.random(hi - lo) < 0.6
        m[:2] = True
        f = oracle_mod.refit_on_mask(th, vd, m)
        t = th.astype(np.float64)[m]
        A = np.stack([np.cos(t), np.sin(t)], axis=1)
        x = np.linalg.lstsq(A, vd.astype(np.float64)[m], rcond=None)[0]
        assert f.n_inliers == m.sum() and f.status == oracle_mod.CLUSTER_OK
        assert abs(f.vx - x[0]) <= 1e-10 * (1 + abs(x[0]))
        assert abs(f.vy - x[1]) <= 1e-10 * (1 + abs(x[1]))
        assert abs(math.remainder(f.heading - math.atan2(x[1], x[0]), 2 * math.pi)) <= 1e-10
    th = np.array([0.1, 0.4, 0.7, np.nan, 0.3], np.float32)
    vd = np.array([1.0, 2.0, 3.0, 4.0, np.inf], np.float32)
    f = oracle_mod.refit_on_mask(th, vd, np.ones(5, bool))
    g = oracle_mod.refit_on_mask(th[:3], vd[:3], np.ones(3, bool))
    assert f.n_inliers == 3 and (f.vx, f.vy) == (g.vx, g.vy)
    assert oracle_mod.refit_on_mask(th, vd, np.array([1, 0, 0, 0, 0])).status == \
        oracle_mod.CLUSTER_SINGULAR_REFIT
    same = np.full(4, 0.25, np.float32)
    assert oracle_mod.refit_on_mask(same, vd[:4], np.ones(4, bool)).status == \
        oracle_mod.CLUSTER_SINGULAR_REFIT


def test_heading_quadrants(oracle_mod):
    rng = np.random.default_rng(2)
    truths = [(10, 10), (-10, 10), (-10, -10), (10, -10), (-10, 1e-3), (-10, -1e-3), (0.0, 5.0), (0.0, -5.0)]
    clusters = [_noiseless_cluster(rng, 60, vx, vy) for vx, vy in truths]
    th, vd, off = _frame_from_clusters(clusters)
    r = oracle_mod.estimate_velocity(th, vd, off, 64, 0.15, seed=3)
    for k, (vx, vy) in enumerate(truths):
        assert abs(math.remainder(r.heading[k] - math.atan2(vy, vx), 2 * math.pi)) < 1e-4
    # headings near +/-pi land on the correct side
    assert r.heading[4] > 3.0 and r.heading[5] < -3.0


def test_refit_equals_lstsq_and_pinv_on_the_mask(oracle_mod):
    frame, H, tau = synth.make_workload("small")
    r = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=11)
    for k in range(frame.n_clusters):
        lo, hi = frame.offsets[k], frame.offsets[k + 1]
        m = r.inlier_mask[lo:hi].astype(bool)
        assert m.sum() == r.n_inliers[k]
        t = frame.theta[lo:hi].astype(np.float64)[m]
        v = frame.vd[lo:hi].astype(np.float64)[m]
        A = np.stack([np.cos(t), np.sin(t)], axis=1)
        x_ls = np.linalg.lstsq(A, v, rcond=None)[0]
        x_pi = np.linalg.pinv(A) @ v
        got = np.array([r.vx[k], r.vy[k]])
        scale = max(1.0, np.abs(x_ls).max())
        assert np.abs(got - x_ls).max() <= 1e-10 * scale
        assert np.abs(got - x_pi).max() <= 1e-10 * scale
        assert r.heading[k] == math.atan2(r.vy[k], r.vx[k])


def test_noiseless_with_outliers_finds_exact_inlier_set(oracle_mod):
    spec = synth.FrameSpec(48, "uniform", 30, 150, p_uniform=0.20, p_band=0.10, sigma=0.0)
    frame = synth.make_frame(spec, seed=21)
    tau = 0.15
    r = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, 256, tau, seed=5)
    checked = 0
    for k in range(frame.n_clusters):
        lo, hi = frame.offsets[k], frame.offsets[k + 1]
        t = frame.theta[lo:hi].astype(np.float64)
        v = frame.vd[lo:hi].astype(np.float64)
        true_in = frame.kind[lo:hi] == 0
        dist = np.abs(v - frame.truth_vx[k] * np.cos(t) - frame.truth_vy[k] * np.sin(t))
        if np.any(dist[~true_in] < 2 * tau):
            continue  # an outlier happens to sit on the profile: exactness not implied
        checked += 1
        assert np.array_equal(r.inlier_mask[lo:hi].astype(bool), true_in)
        A = np.stack([np.cos(t[true_in]), np.sin(t[true_in])], axis=1)
        x = np.linalg.lstsq(A, v[true_in], rcond=None)[0]
        assert abs(r.vx[k] - x[0]) < 1e-10 and abs(r.vy[k] - x[1]) < 1e-10
    assert checked >= 40


# --------------------------------------------------------------------------
# exhaustive search on small clusters
# --------------------------------------------------------------------------
def test_ransac_best_equals_all_pairs_search(oracle_mod):
    rng = np.random.default_rng(4)
    clusters = []
    for _ in range(40):
        n = int(rng.integers(3, 13))
        vx, vy = rng.uniform(-30, 30, 2)
        th, vd = _noiseless_cluster(rng, n, vx, vy)
        vd = vd + rng.normal(0, 0.08, n).astype(np.float32)
        out = rng.random(n) < 0.3
        vd[out] = rng.uniform(-40, 40, out.sum()).astype(np.float32)
        clusters.append((th, vd))
    th, vd, off = _frame_from_clusters(clusters)
    H = 4096  # every unordered pair of <= 12 points is drawn with probability ~ 1 - 1e-25
    r = oracle_mod.estimate_velocity(th, vd, off, H, 0.15, seed=8, debug=True)
    for k in range(len(clusters)):
        lo, hi = off[k], off[k + 1]
        best, best_pairs, _ = oracle_mod.all_pairs_best(th[lo:hi], vd[lo:hi], 0.15)
        h = r.best_hyp[k]
        assert r.hyp_count[k, h] == best
        assert best_pairs[r.hyp_i[k, h], r.hyp_j[k, h]]


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------
def _dyadic_frame(seed, n_clusters=24, phi_room=0.5):
    """Azimuths on a 2^-16 rad grid inside +/-(1 - phi_room) rad."""
    rng = np.random.default_rng(seed)
    clusters = []
    lim = int((1.0 - phi_room) * 2**16)
    for _ in range(n_clusters):
        n = int(rng.integers(10, 120))
        th = (rng.integers(-lim, lim + 1, n) * 2.0**-16).astype(np.float32)
        vx, vy = rng.uniform(-30, 30, 2)
        t = th.astype(np.float64)
        vd = vx * np.cos(t) + vy * np.sin(t) + rng.normal(0, 0.05, n)
        out = rng.random(n) < 0.25
        vd[out] = rng.uniform(-40, 40, out.sum())
        clusters.append((th, vd.astype(np.float32)))
    return _frame_from_clusters(clusters)


def test_rotation_rotates_the_estimate(oracle_mod):
    th, vd, off = _dyadic_frame(31)
    H, tau, seed = 256, 0.15, 77
    base = oracle_mod.estimate_velocity(th, vd, off, H, tau, seed)
    for m in (1, -5000, 17001, 32767):
        phi = m * 2.0**-16
        th2 = (th.astype(np.float64) + phi).astype(np.float32)
        assert np.array_equal(th2.astype(np.float64), th.astype(np.float64) + phi)  # exact shift
        rot = oracle_mod.estimate_velocity(th2, vd, off, H, tau, seed)
        assert np.array_equal(rot.best_hyp, base.best_hyp)
        assert np.array_equal(rot.n_inliers, base.n_inliers)
        assert np.array_equal(rot.inlier_mask, base.inlier_mask)
        c, s = math.cos(phi), math.sin(phi)
        ex = c * base.vx - s * base.vy
        ey = s * base.vx + c * base.vy
        assert np.abs(rot.vx - ex).max() < 1e-9 and np.abs(rot.vy - ey).max() < 1e-9
        dh = np.remainder(rot.heading - base.heading - phi + math.pi, 2 * math.pi) - math.pi
        assert np.abs(dh).max() < 1e-9


@pytest.mark.parametrize("k2", [-3, 1, 5])
def test_power_of_two_scaling_is_bitwise(oracle_mod, k2):
    frame, H, tau = synth.make_workload("small")
    base = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=4, debug=True)
    f = 2.0**k2
    tau_s = float(np.float32(tau)) * f  # exactly the float32 tau scaled
    sc = oracle_mod.estimate_velocity(frame.theta, (frame.vd * f).astype(np.float32), frame.offsets,
                                      H, tau_s, seed=4, debug=True)
    assert np.array_equal(sc.inlier_mask, base.inlier_mask)
    assert np.array_equal(sc.n_inliers, base.n_inliers)
    assert np.array_equal(sc.best_hyp, base.best_hyp)
    assert np.array_equal(sc.hyp_count, base.hyp_count)
    assert np.array_equal(sc.vx, base.vx * f) and np.array_equal(sc.vy, base.vy * f)
    assert np.array_equal(sc.heading, base.heading)


def test_sign_flip_is_bitwise(oracle_mod):
    frame, H, tau = synth.make_workload("small")
    base = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=9)
    neg = oracle_mod.estimate_velocity(frame.theta, -frame.vd, frame.offsets, H, tau, seed=9)
    assert np.array_equal(neg.inlier_mask, base.inlier_mask)
    assert np.array_equal(neg.vx, -base.vx) and np.array_equal(neg.vy, -base.vy)
    assert all(h == math.atan2(-y, -x) for h, x, y in zip(neg.heading, base.vx, base.vy))
    dh = np.remainder(neg.heading - base.heading, 2 * math.pi)
    assert np.abs(dh - math.pi).max() < 1e-12


def test_reflection_is_bitwise(oracle_mod):
    frame, H, tau = synth.make_workload("small")
    t = frame.theta.astype(np.float64)
    # the host libm is odd/even symmetric on these inputs (precondition of the pin)
    assert np.array_equal(np.sin(-t), -np.sin(t)) and np.array_equal(np.cos(-t), np.cos(t))
    base = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=13)
    ref = oracle_mod.estimate_velocity(-frame.theta, frame.vd, frame.offsets, H, tau, seed=13)
    assert np.array_equal(ref.inlier_mask, base.inlier_mask)
    assert np.array_equal(ref.vx, base.vx) and np.array_equal(ref.vy, -base.vy)
    assert np.array_equal(ref.heading, -base.heading)


def test_results_independent_of_other_clusters(oracle_mod):
    frame, H, tau = synth.make_workload("small")
    base = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=21)
    # append clusters after the frame
    extra = synth.make_frame(synth.FrameSpec(10, "uniform", 5, 300), seed=99)
    both = synth.concat_frames([frame, extra])
    r2 = oracle_mod.estimate_velocity(both.theta, both.vd, both.offsets, H, tau, seed=21)
    K = frame.n_clusters
    for name in ("vx", "vy", "heading", "n_inliers", "best_hyp", "status"):
        assert np.array_equal(getattr(r2, name)[:K], getattr(base, name)), name
    # subset evaluation keeps each cluster's stream (keyed by its index)
    ids = np.array([5, 63, 0, 17])
    sub = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=21, cluster_ids=ids)
    assert np.array_equal(sub.vx, base.vx[ids]) and np.array_equal(sub.n_inliers, base.n_inliers[ids])
    # thread count does not change anything
    one = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=21, n_threads=1)
    assert np.array_equal(one.vx, base.vx) and np.array_equal(one.inlier_mask, base.inlier_mask)


# --------------------------------------------------------------------------
# degenerate and non-finite inputs
# --------------------------------------------------------------------------
def test_degenerate_clusters(oracle_mod):
    rng = np.random.default_rng(6)
    good = _noiseless_cluster(rng, 30, 3.0, -4.0)
    same_theta = (np.full(20, 0.3, np.float32), rng.uniform(-5, 5, 20).astype(np.float32))
    clusters = [([], []), ([0.1], [1.0]), good, same_theta, ([0.1, 0.1005], [1.0, 2.0])]
    th, vd, off = _frame_from_clusters(clusters)
    r = oracle_mod.estimate_velocity(th, vd, off, 32, 0.15, seed=1, debug=True)
    C = oracle_mod
    assert list(r.status) == [C.CLUSTER_TOO_FEW_POINTS, C.CLUSTER_TOO_FEW_POINTS, C.CLUSTER_OK,
                              C.CLUSTER_ALL_DEGENERATE, C.CLUSTER_ALL_DEGENERATE]
    for k in (0, 1, 3, 4):
        assert math.isnan(r.vx[k]) and math.isnan(r.vy[k]) and math.isnan(r.heading[k])
        assert r.n_inliers[k] == 0
    assert r.best_hyp[0] == -1 and r.best_hyp[3] == -1
    assert not r.hyp_valid[3].any()


def test_non_finite_points_are_never_inliers(oracle_mod):
    rng = np.random.default_rng(7)
    th, vd = _noiseless_cluster(rng, 50, 5.0, 2.0)
    th = th.copy(); vd = vd.copy()
    th[3] = np.nan; vd[10] = np.inf; vd[11] = np.nan; th[12] = -np.inf
    off = np.array([0, 50], np.int32)
    r = oracle_mod.estimate_velocity(th, vd, off, 128, 0.15, seed=2, debug=True)
    assert r.status[0] == oracle_mod.CLUSTER_OK
    assert r.n_inliers[0] == 46
    assert not r.inlier_mask[[3, 10, 11, 12]].any()
    bad = {3, 10, 11, 12}
    for h in range(128):
        if r.hyp_i[0, h] in bad or r.hyp_j[0, h] in bad:
            assert r.hyp_valid[0, h] == 0
    assert abs(r.vx[0] - 5.0) < 1e-4 and abs(r.vy[0] - 2.0) < 1e-4


def test_bad_offsets_are_flagged(oracle_mod):
    th = np.linspace(-1, 1, 40).astype(np.float32)
    vd = np.cos(th).astype(np.float32)
    off = np.array([0, 20, 10, 45], np.int32)  # decreasing, then past the end
    r = oracle_mod.estimate_velocity(th, vd, off, 16, 0.15, seed=1)
    assert r.status[0] == oracle_mod.CLUSTER_OK
    assert r.status[1] == oracle_mod.CLUSTER_BAD_OFFSETS
    assert r.status[2] == oracle_mod.CLUSTER_BAD_OFFSETS


def test_invalid_arguments(oracle_mod):
    th = np.zeros(4, np.float32)
    off = np.array([0, 4], np.int32)
    for H, tau in [(0, 0.15), (8, 0.0), (8, float("nan")), (8, float("inf")), (8, -1.0)]:
        with pytest.raises(ValueError):
            oracle_mod.estimate_velocity(th, th, off, H, tau, seed=0)


# --------------------------------------------------------------------------
# statistics against ground truth
# --------------------------------------------------------------------------
def test_error_statistics_match_least_squares_theory(oracle_mod):
    spec = synth.FrameSpec(400, "uniform", 40, 200, p_uniform=0.2, sigma=0.05)
    frame = synth.make_frame(spec, seed=41)
    r = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, 256, 0.15, seed=3)
    z = []
    for k in range(frame.n_clusters):
        lo, hi = frame.offsets[k], frame.offsets[k + 1]
        m = r.inlier_mask[lo:hi].astype(bool)
        t = frame.theta[lo:hi].astype(np.float64)[m]
        A = np.stack([np.cos(t), np.sin(t)], axis=1)
        cov = 0.05**2 * np.linalg.inv(A.T @ A)
        e = np.array([r.vx[k] - frame.truth_vx[k], r.vy[k] - frame.truth_vy[k]])
        z.append(float(e @ np.linalg.solve(cov, e)))
    z = np.array(z)
    # e^T cov^-1 e ~ chi-square(2) (mean 2) up to the truncation of the noise at tau;
    # truncation at 3 sigma shrinks it slightly.
    assert 1.3 < z.mean() < 2.4, z.mean()
    assert np.quantile(z, 0.99) < 20


def test_comparable_to_sklearn_ransac(oracle_mod):
    sklearn = pytest.importorskip("sklearn.linear_model")
    frame, H, tau = synth.make_workload("small")
    r = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=1)
    ours, theirs = [], []
    for k in range(frame.n_clusters):
        lo, hi = frame.offsets[k], frame.offsets[k + 1]
        t = frame.theta[lo:hi].astype(np.float64)
        X = np.stack([np.cos(t), np.sin(t)], axis=1)
        y = frame.vd[lo:hi].astype(np.float64)
        m = sklearn.RANSACRegressor(sklearn.LinearRegression(fit_intercept=False), min_samples=2,
                                    residual_threshold=tau, max_trials=H, random_state=k)
        m.fit(X, y)
        est = m.estimator_.coef_
        theirs.append(math.hypot(est[0] - frame.truth_vx[k], est[1] - frame.truth_vy[k]))
        ours.append(math.hypot(r.vx[k] - frame.truth_vx[k], r.vy[k] - frame.truth_vy[k]))
    ours, theirs = np.median(ours), np.median(theirs)
    assert ours < 0.05 and theirs < 0.05
    assert 0.5 < ours / theirs < 2.0


def test_fit_hypothesis_reproduces_the_kept_hypothesis(oracle_mod):
    frame, H, tau = synth.make_workload("small")
    r = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed=17, debug=True)
    for k in (0, 7, 63):
        f = oracle_mod.fit_hypothesis(frame.theta, frame.vd, frame.offsets, tau, 17, k, r.best_hyp[k])
        lo, hi = frame.offsets[k], frame.offsets[k + 1]
        assert f.vx == r.vx[k] and f.vy == r.vy[k] and f.heading == r.heading[k]
        assert f.n_inliers == r.n_inliers[k] and f.n_near_tau == r.n_near_tau[k]
        assert np.array_equal(f.mask, r.inlier_mask[lo:hi])
        # another valid hypothesis: its mask is what its count says
        h2 = int(np.flatnonzero(r.hyp_valid[k])[-1])
        g = oracle_mod.fit_hypothesis(frame.theta, frame.vd, frame.offsets, tau, 17, k, h2)
        assert g.n_inliers == r.hyp_count[k, h2]
    # a degenerate hypothesis is reported as such
    th = np.full(6, 0.2, np.float32)
    assert oracle_mod.fit_hypothesis(th, th, np.array([0, 6], np.int32), 0.15, 1, 0, 0) is None
