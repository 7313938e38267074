"""GPU: the paper-literal variant (rv_estimate_velocity_paper) against its FP64
oracle (rv_oracle_paper.c).

Both sides evaluate the same FP64 expressions in the same order (no
contraction), so thresholds, per-trial counts, kept trials and inlier masks
must be identical bit for bit; the refit's sums run in different orders, so
vx, vy and heading (float32 outputs) agree within 1e-4.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import parity  # noqa: E402
from paper_2012_12618_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2012_12618_amd import binding

    binding.load_library()
    return binding


def _run(rv, theta, vd, offsets, H, seed, label, bits=True):
    # With the frame-wide mask requested the call takes the three kernels; without
    # it, frames of at most 65,536 points and clusters with H <= 256 take one launch.
    print(f"[gpu] rv_estimate_velocity_paper {label} K={len(offsets) - 1} N={len(theta)} H={H} "
          f"bits={bits}", flush=True)
    t = torch.from_numpy(np.ascontiguousarray(theta, np.float32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(vd, np.float32)).cuda()
    o = torch.from_numpy(np.ascontiguousarray(offsets, np.int32)).cuda()
    r = rv.rv_estimate_velocity_paper(t, v, o, H, seed, want_bits=bits, debug=True)
    torch.cuda.synchronize()
    g = {k: x.cpu().numpy() for k, x in r.items() if not k.startswith("_")}
    if bits:
        g["mask"] = parity.unpack_bits(g["inlier_bits"], len(theta))
    return g


def _compare(g, o, offsets, H, skip=()):
    K = len(offsets) - 1
    keep = np.array([k not in skip for k in range(K)], bool)
    assert np.array_equal(g["status"][keep], o.status[keep])
    th_g, th_o = g["thresh"][keep], o.thresh[keep]
    assert np.array_equal(np.isnan(th_g), np.isnan(th_o))
    assert np.array_equal(th_g[~np.isnan(th_g)], th_o[~np.isnan(th_o)])  # bit for bit
    assert np.array_equal(g["best_hyp"][keep], o.best_hyp[keep])
    assert np.array_equal(g["n_inliers"][keep], o.n_inliers[keep])
    hc = g["hyp_counts"].reshape(K, H)
    assert np.array_equal(hc[keep], o.hyp_count[keep])
    for k in np.flatnonzero(keep) if "mask" in g else ():
        a, b = offsets[k], offsets[k + 1]
        assert np.array_equal(g["mask"][a:b], o.inlier_mask[a:b]), k
    ok = keep & (o.status == 0)
    for key in ("vx", "vy"):
        assert np.max(np.abs(g[key][ok] - o.__dict__[key][ok]), initial=0.0) <= 1e-4, key
    dh = np.abs(np.angle(np.exp(1j * (g["heading"][ok].astype(np.float64) - o.heading[ok]))))
    assert np.max(dh, initial=0.0) <= 1e-4
    bad = keep & (o.status != 0)
    assert np.all(np.isnan(g["vx"][bad]))


@pytest.mark.parametrize("clusters,points", [(8, 100), (16, 150), (32, 100), (64, 150)])
def test_table_shapes(rv, oracle_mod, clusters, points):
    spec = synth.FrameSpec(n_clusters=clusters, size_kind="fixed", size_lo=points, size_hi=points,
                           p_uniform=0.2)
    f = synth.make_frame(spec, 100 + clusters + points)
    H, seed = 256, synth.ransac_seed("paper", clusters * 1000 + points)
    g = _run(rv, f.theta, f.vd, f.offsets, H, seed, f"table {clusters}x{points}")
    o = oracle_mod.estimate_velocity_paper(f.theta, f.vd, f.offsets, H, seed, debug=True)
    _compare(g, o, f.offsets, H)


def test_small_and_dense_like_frames(rv, oracle_mod):
    f, _, _ = synth.make_workload("small")
    for H, seed in ((64, 1), (300, 2)):
        g = _run(rv, f.theta, f.vd, f.offsets, H, seed, f"small H={H}")
        o = oracle_mod.estimate_velocity_paper(f.theta, f.vd, f.offsets, H, seed, debug=True)
        _compare(g, o, f.offsets, H)
    spec = synth.FrameSpec(n_clusters=48, size_kind="loguniform", size_lo=8, size_hi=4096,
                           p_uniform=0.15, p_band=0.15)
    f = synth.make_frame(spec, 77)
    g = _run(rv, f.theta, f.vd, f.offsets, 128, 5, "loguniform to 4096")
    o = oracle_mod.estimate_velocity_paper(f.theta, f.vd, f.offsets, 128, 5, debug=True)
    _compare(g, o, f.offsets, 128)


@pytest.mark.parametrize("case", range(4))
def test_drawn_shapes(rv, oracle_mod, case):
    # Frames of drawn shape (cluster count, sizes up to the variant's limit,
    # outliers, noise, H) against the variant's own oracle, on both paths.
    rng = np.random.default_rng(9500 + case)
    lo = int(rng.integers(2, 40))
    spec = synth.FrameSpec(int(rng.integers(1, 100)), ("uniform", "loguniform")[case % 2], lo,
                           int(rng.integers(lo, 4097)), p_uniform=float(rng.uniform(0, 0.5)),
                           p_band=float(rng.uniform(0, 0.3)), sigma=float(rng.uniform(0.01, 0.2)))
    f = synth.make_frame(spec, 9600 + case)
    H = int(rng.choice([1, 50, 256, 600]))
    seed = 9700 + case
    o = oracle_mod.estimate_velocity_paper(f.theta, f.vd, f.offsets, H, seed, debug=True)
    for bits in (True, False):
        g = _run(rv, f.theta, f.vd, f.offsets, H, seed, f"drawn {case} bits={bits}", bits=bits)
        _compare(g, o, f.offsets, H)


def _edge_frame(rv):
    # one point, equal azimuths, a NaN point, zero Doppler span, an empty
    # cluster, a cluster of RV_PAPER_MAX_POINTS points and one above the limit
    rng = np.random.default_rng(4)
    big = rv.RV_PAPER_MAX_POINTS
    theta = np.concatenate([np.array([0.1, 0.2, 0.2, 0.2, 0.3, np.nan, 0.5, 0.6, 0.7], np.float32),
                            rng.uniform(-1, 1, big + big + 1).astype(np.float32)])
    vd = np.concatenate([np.array([1.0, 2.0, 3.0, 4.0, 1.0, 1.0, 2.0, 2.0, 2.0], np.float32),
                         rng.uniform(-9, 9, big + big + 1).astype(np.float32)])
    off = np.array([0, 1, 4, 6, 9, 9, 9 + big, 9 + 2 * big + 1], np.int32)
    return theta, vd, off


def test_hand_worked_example_and_edge_cases(rv, oracle_mod):
    vals = {}
    for line in open(os.path.join(HERE, "golden", "paper_variant_example.txt")):
        if line.strip() and not line.startswith("#"):
            key, *rest = line.split()
            vals[key] = [float(x) for x in rest]
    theta = np.array(vals["theta"], np.float32)
    vd = np.array(vals["vd"], np.float32)
    g = _run(rv, theta, vd, np.array([0, 5], np.int32), 64, 3, "golden")
    assert g["thresh"][0] == pytest.approx(vals["thresh"][0], abs=1e-15)
    assert list(g["mask"]) == [int(x) for x in vals["mask"]]
    theta, vd, off = _edge_frame(rv)
    g = _run(rv, theta, vd, off, 96, 8, "edges")
    o = oracle_mod.estimate_velocity_paper(theta, vd, off, 96, 8, debug=True)
    assert g["status"][6] == rv.RV_CLUSTER_TOO_LARGE
    _compare(g, o, off, 96, skip=(6,))
    bad = np.array([0, 5, 3, 9], np.int32)
    g = _run(rv, theta[:9], vd[:9], bad, 16, 1, "bad offsets")
    assert g["status"][1] == rv.RV_CLUSTER_BAD_OFFSETS


def _ties_frame():
    # Doppler values on a coarse grid (many equal normalised values, so the
    # medians fall on ties), odd and even counts of usable points, non-finite
    # points, a majority of equal values (threshold 0: every trial takes the
    # literal test), and sizes on both sides of 256 points (ranks below,
    # bitonic sorts above).
    rng = np.random.default_rng(12)
    sizes = [2, 3, 4, 5, 17, 64, 127, 128, 129, 200, 255, 256, 257, 300, 511, 1024]
    thetas, vds = [], []
    for i, n in enumerate(sizes):
        th = rng.uniform(-1.0, 1.0, n).astype(np.float32)
        vd = (np.round(rng.uniform(-6, 6, n) * 2) / 2).astype(np.float32)
        if i % 3 == 1 and n > 4:
            vd[: n // 2 + 1] = 1.5  # more than half equal: the MAD is 0
        if i % 4 == 2 and n > 3:
            vd[1] = np.nan
            th[2] = np.inf
        thetas.append(th)
        vds.append(vd)
    theta = np.concatenate(thetas)
    vd = np.concatenate(vds)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    return theta, vd, off


def test_ties_sizes_around_the_rank_limit(rv, oracle_mod):
    theta, vd, off = _ties_frame()
    for H, seed in ((64, 21), (256, 22)):
        g = _run(rv, theta, vd, off, H, seed, f"ties H={H}")
        o = oracle_mod.estimate_velocity_paper(theta, vd, off, H, seed, debug=True)
        _compare(g, o, off, H)
        assert np.count_nonzero(o.thresh == 0.0) >= 3


@pytest.mark.parametrize("H", [1, 64, 256, 257])
def test_one_launch_path_matches_three_kernels(rv, oracle_mod, H):
    frames = []
    for clusters, points in ((8, 100), (64, 150)):
        spec = synth.FrameSpec(n_clusters=clusters, size_kind="fixed", size_lo=points,
                               size_hi=points, p_uniform=0.2)
        f = synth.make_frame(spec, 300 + clusters + points)
        frames.append((f"table {clusters}x{points}", f.theta, f.vd, f.offsets))
    frames.append(("ties",) + _ties_frame())
    spec = synth.FrameSpec(n_clusters=48, size_kind="loguniform", size_lo=2, size_hi=4096,
                           p_uniform=0.15, p_band=0.15)
    f = synth.make_frame(spec, 78)
    frames.append(("loguniform to 4096", f.theta, f.vd, f.offsets))
    bad = np.array([0, 5, 3, 9, 9], np.int32)  # a decreasing offset and an empty cluster
    frames.append(("bad offsets", f.theta[:9], f.vd[:9], bad))
    frames.append(("edges",) + _edge_frame(rv))
    for label, theta, vd, off in frames:
        seed = 40 + H
        a = _run(rv, theta, vd, off, H, seed, label, bits=True)
        b = _run(rv, theta, vd, off, H, seed, label, bits=False)
        if label == "bad offsets":
            # After a decreasing offset the next range overlaps an earlier one;
            # only the status flags are defined there.
            assert np.array_equal(a["status"], b["status"])
            assert a["status"][1] == rv.RV_CLUSTER_BAD_OFFSETS
            continue
        for key in ("vx", "vy", "heading", "thresh"):
            assert np.array_equal(a[key].view(np.uint8), b[key].view(np.uint8)), (label, key)
        for key in ("n_inliers", "status", "hyp_counts", "best_hyp"):
            assert np.array_equal(a[key], b[key]), (label, key)
        o = oracle_mod.estimate_velocity_paper(theta, vd, off, H, seed, debug=True)
        skip = ()
        if label == "edges":
            assert b["status"][6] == rv.RV_CLUSTER_TOO_LARGE
            skip = (6,)
        _compare(b, o, off, H, skip=skip)


def test_preallocated_outputs_match_fresh_ones(rv):
    f = synth.table_frame(16, 150)
    t = torch.from_numpy(f.theta).cuda()
    v = torch.from_numpy(f.vd).cuda()
    o = torch.from_numpy(f.offsets).cuda()
    for bits in (False, True):
        out = rv.allocate_paper_outputs(f.n_clusters, f.n_points, 256, t.device, want_bits=bits,
                                        debug=True)
        for seed in (5, 6):
            print(f"[gpu] rv_estimate_velocity_paper preallocated bits={bits} seed={seed}", flush=True)
            a = rv.rv_estimate_velocity_paper(t, v, o, 256, seed, out=out)
            b = rv.rv_estimate_velocity_paper(t, v, o, 256, seed, want_bits=bits, debug=True)
            torch.cuda.synchronize()
            assert set(a) == set(b)
            for key in a:
                x, y = a[key].cpu().numpy(), b[key].cpu().numpy()
                assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), (bits, seed, key)
