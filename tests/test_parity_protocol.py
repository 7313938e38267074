"""The GPU-versus-oracle acceptance protocol itself (tests/parity.py), on the CPU.

Outputs shaped like the GPU's are built from the oracle and then altered the way
a float32 path may legitimately differ (a count inside the band, a mask bit
flipped at a point the oracle flags near tau, with the refit redone on that
mask) or the way a broken path would (a count outside the band, a flipped bit
away from tau, a refit that does not match the mask it reports).  The checker
must accept the first kind, reject the second, and count what it accepted.
The inputs are the hand-worked clusters of tests/golden/tau_band_example.txt
(Sec. 3.1, Alg. 1 inlier test; Sec. 3.2, Eq. 7 refit).
"""
import numpy as np
import pytest

import parity
from paper_2012_12618_amd import synth
from test_oracle_band import _clusters, _pair_hypotheses

H, SEED = 2048, 0x5EED


@pytest.fixture(scope="module")
def frame(oracle_mod):
    tau, clusters = _clusters()
    # Cluster B gains eight points on its profile (vx = 1, vy = tan 0.25) at
    # theta = -0.5, so that hypotheses on that profile win clearly and the kept
    # one has points within 1e-5 of tau (under a hypothesis seeded by another
    # theta = 0 point the extra points lie about 0.26 m/s off its profile).
    b = clusters[1]
    t_extra = np.full(8, -0.5, np.float32)
    v_extra = (np.cos(-0.5) + np.tan(0.25) * np.sin(-0.5)) * np.ones(8)
    b["theta"] = np.concatenate([b["theta"], t_extra])
    b["vd"] = np.concatenate([b["vd"], v_extra.astype(np.float32)])
    th = np.concatenate([c["theta"] for c in clusters])
    vd = np.concatenate([c["vd"] for c in clusters])
    off = np.cumsum([0] + [len(c["theta"]) for c in clusters]).astype(np.int32)
    o = oracle_mod.estimate_velocity(th, vd, off, H, tau, SEED, debug=True)
    return th, vd, off, tau, o


def _as_gpu(o):
    return {"vx": o.vx.astype(np.float32), "vy": o.vy.astype(np.float32),
            "heading": o.heading.astype(np.float32), "n_inliers": o.n_inliers.copy(),
            "status": o.status.copy(), "n_near_tau": o.n_near_tau.copy(),
            "best_hyp": o.best_hyp.copy(), "hyp_counts": o.hyp_count.ravel().copy(),
            "mask": o.inlier_mask.astype(bool)}


def test_oracle_outputs_pass(frame):
    th, vd, off, tau, o = frame
    st = parity.check(th, vd, off, H, tau, SEED, _as_gpu(o), o)
    assert st["hyp_count_differs"] == 0 and st["hyp_rel_band_only"] == 0
    assert st["mask_diff_points"] == 0 and st["refit_on_gpu_mask"] == 0


def test_counts_inside_the_band_are_counted(frame):
    th, vd, off, tau, o = frame
    g = _as_gpu(o)
    hs = _pair_hypotheses(o, 0)  # cluster A: count 6, band [3, 8], absolute-only band [5, 7]
    gc = g["hyp_counts"].reshape(-1, H)
    gc[0, hs[0]] = 8   # inside the band only through its relative term
    gc[0, hs[1]] = 7   # inside the absolute 1e-5 band
    st = parity.check(th, vd, off, H, tau, SEED, g, o)
    assert st["hyp_count_differs"] == 2
    assert st["hyp_rel_band_only"] == 1
    gc[0, hs[2]] = 9   # outside the band
    with pytest.raises(AssertionError, match="outside the band"):
        parity.check(th, vd, off, H, tau, SEED, g, o)


def _near_point(oracle_mod, frame, k):
    th, vd, off, tau, o = frame
    f = oracle_mod.fit_hypothesis(th, vd, off, tau, SEED, k, int(o.best_hyp[k]))
    near = np.flatnonzero(f.near_mask)
    far = np.flatnonzero(~f.near_mask.astype(bool) & ~f.mask.astype(bool))
    return near, far


def test_mask_difference_near_tau_is_refit_on_the_gpu_mask(oracle_mod, frame):
    th, vd, off, tau, o = frame
    k = 1  # cluster B: four points within 1e-5 of tau under the pair (S, P)
    near, far = _near_point(oracle_mod, frame, k)
    assert near.size > 0 and far.size > 0
    lo, hi = int(off[k]), int(off[k + 1])
    g = _as_gpu(o)
    g["mask"][lo + near[0]] = not g["mask"][lo + near[0]]
    gm = g["mask"][lo:hi]
    g["n_inliers"][k] = int(gm.sum())
    # the oracle's refit on the other mask is not within 1e-4 of this one
    with pytest.raises(AssertionError, match="dv"):
        parity.check(th, vd, off, H, tau, SEED, g, o)
    mf = oracle_mod.refit_on_mask(th[lo:hi], vd[lo:hi], gm)
    g["vx"][k], g["vy"][k], g["heading"][k] = mf.vx, mf.vy, mf.heading
    st = parity.check(th, vd, off, H, tau, SEED, g, o)
    assert st["mask_diff_points"] == 1 and st["refit_on_gpu_mask"] == 1
    # a flipped bit at a point far from tau is an error
    g2 = _as_gpu(o)
    g2["mask"][lo + far[0]] = True
    with pytest.raises(AssertionError, match="not near tau"):
        parity.check(th, vd, off, H, tau, SEED, g2, o)


def test_velocity_bound_includes_the_float32_rounding(oracle_mod):
    # One hypothesis per cluster: some refits pass through two nearly collinear
    # points and give thousands of m/s, whose float32 outputs cannot lie within
    # 1e-4 of the FP64 refit.  The oracle's own results rounded to float32 pass;
    # an error beyond the bound fails.
    rng = np.random.default_rng(7003)  # the shape drawn by the GPU random-shape case 3
    lo = int(rng.integers(2, 40))
    spec = synth.FrameSpec(int(rng.integers(1, 120)), "loguniform", lo, int(rng.integers(lo, 1500)),
                           p_uniform=float(rng.uniform(0.0, 0.5)),
                           p_band=float(rng.uniform(0.0, 0.3)), sigma=float(rng.uniform(0.01, 0.2)))
    f = synth.make_frame(spec, 7103)
    tau = float(np.float32(0.15))
    o = oracle_mod.estimate_velocity(f.theta, f.vd, f.offsets, 1, tau, 0x7003, debug=True)
    speed = np.abs(np.nan_to_num(o.vx)) + np.abs(np.nan_to_num(o.vy))
    k = int(np.argmax(speed))
    big = max(abs(o.vx[k]), abs(o.vy[k]))
    assert big > 1700 and o.status[k] == 0
    g = _as_gpu(o)
    assert max(abs(float(g["vx"][k]) - o.vx[k]), abs(float(g["vy"][k]) - o.vy[k])) > parity.V_TOL \
        or np.spacing(np.float32(big)) / 2 > parity.V_TOL
    parity.check(f.theta, f.vd, f.offsets, 1, tau, 0x7003, g, o)
    g2 = _as_gpu(o)
    worse = 2 * parity.v_tolerance(o.vx[k], o.vy[k])
    if abs(o.vx[k]) >= abs(o.vy[k]):
        g2["vx"][k] = np.float32(o.vx[k] + worse)
    else:
        g2["vy"][k] = np.float32(o.vy[k] + worse)
    with pytest.raises(AssertionError, match="dv"):
        parity.check(f.theta, f.vd, f.offsets, 1, tau, 0x7003, g2, o)
