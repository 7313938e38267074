"""Pins of the oracle's tolerance machinery around the strict inlier test of
Sec. 3.1, Alg. 1 (CPU only).

The GPU parity protocol accepts a float32 count that differs from the FP64 count
when it stays inside the oracle's per-hypothesis band [count_lo, count_hi], and
an inlier-mask difference only at points the oracle flags within the near-tau
window.  These tests fix both: the band's absolute and relative half-widths and
the window width, on hand-worked clusters (tests/golden/tau_band_example.txt)
whose residuals are exact, and the band's centre (with zero width the band is
the count itself).  A tenfold change of either module constant, or of the
relative coefficient, changes a hand-worked count.
"""
import os
from fractions import Fraction

import numpy as np

from paper_2012_12618_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _value(text: str) -> float:
    """'128+9829/65536', '0x1.266516p+0' or a plain decimal, exactly."""
    if text.startswith("0x"):
        return float.fromhex(text)
    for op in ("+", "-"):
        head, sep, tail = text.partition(op)
        if sep and head:
            num, _, den = tail.partition("/")
            frac = Fraction(int(num), int(den))
            return float(Fraction(head) + (frac if op == "+" else -frac))
    return float(Fraction(text))


def _clusters():
    out, cur, tau = [], None, None
    with open(os.path.join(HERE, "golden", "tau_band_example.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *rest = line.split()
            if key == "tau":
                tau = float(rest[0])
            elif key == "cluster":
                cur = {"name": rest[0]}
                out.append(cur)
            else:
                cur[key] = rest
    for c in out:
        c["theta"] = np.array([_value(x) for x in c["theta"]], dtype=np.float32)
        vd = np.array([_value(x) for x in c["vd"]], dtype=np.float64)
        assert np.all(vd.astype(np.float32).astype(np.float64) == vd), "fixture values not float32"
        c["vd"] = vd.astype(np.float32)
    return tau, out


def _pair_hypotheses(r, row):
    """Indices of the hypotheses drawn from the seed pair (0, 1), either order."""
    i, j = r.hyp_i[row], r.hyp_j[row]
    return np.flatnonzero(((i == 0) & (j == 1)) | ((i == 1) & (j == 0)))


def test_band_counts_and_near_window_hand_worked(oracle_mod):
    tau, clusters = _clusters()
    th = np.concatenate([c["theta"] for c in clusters])
    vd = np.concatenate([c["vd"] for c in clusters])
    off = np.cumsum([0] + [len(c["theta"]) for c in clusters]).astype(np.int32)
    H, seed = 2048, 0x5EED
    # default tolerance arguments: the module constants are what is pinned
    r = oracle_mod.estimate_velocity(th, vd, off, H, tau, seed, debug=True)
    for k, c in enumerate(clusters):
        hs = _pair_hypotheses(r, k)
        assert hs.size >= 4, f"cluster {c['name']}: the seed pair was drawn {hs.size} times"
        assert np.all(r.hyp_valid[k, hs] == 1)
        assert np.all(r.hyp_vx[k, hs] == float(c["hyp_vx"][0])), c["name"]
        assert np.all(r.hyp_count[k, hs] == int(c["count"][0])), c["name"]
        assert np.all(r.hyp_count_lo[k, hs] == int(c["count_lo"][0])), (
            c["name"], r.hyp_count_lo[k, hs][:4])
        assert np.all(r.hyp_count_hi[k, hs] == int(c["count_hi"][0])), (
            c["name"], r.hyp_count_hi[k, hs][:4])
        # the refit of that hypothesis: its inlier set and the near-tau flags
        f = oracle_mod.fit_hypothesis(th, vd, off, tau, seed, k, int(hs[0]))
        assert f is not None
        assert f.n_inliers == int(c["n_inliers"][0])
        assert f.n_near_tau == int(c["n_near_tau"][0]), (c["name"], f.n_near_tau)
        assert f.mask.tolist() == [int(x) for x in c["inlier_mask"]]
        assert f.near_mask.tolist() == [int(x) for x in c["near_mask"]]


def test_zero_band_is_the_count(oracle_mod):
    # With zero width both band edges are the strict count itself, for every
    # hypothesis of the small workload (and 0 for the invalid ones).
    frame, H, tau = synth.make_workload("small")
    seed = synth.ransac_seed("small")
    r = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed,
                                     debug=True, band_abs=0.0, band_rel=0.0)
    assert np.array_equal(r.hyp_count_lo, r.hyp_count)
    assert np.array_equal(r.hyp_count_hi, r.hyp_count)
    # and the default band brackets it
    d = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed,
                                     debug=True)
    assert np.array_equal(d.hyp_count, r.hyp_count)
    assert np.all(d.hyp_count_lo <= d.hyp_count) and np.all(d.hyp_count <= d.hyp_count_hi)
    assert np.any(d.hyp_count_lo < d.hyp_count_hi), "no hypothesis of the workload is ambiguous"
