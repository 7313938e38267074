"""GPU parity: the HIP estimator (through the C ABI) against the FP64 oracle.

Acceptance protocol in tests/parity.py.  Cases: the two full-size workloads
("small": 64 clusters, H = 256; "dense": 4096 clusters of log-uniform size in
[8, 4096], H = 1024, the benchmark's launch configuration), random small
frames over several hypothesis counts, cluster sizes around every register-row
and register-pass boundary, one 65,536-point cluster, a frame of 70,000 small
clusters (beyond the dispatch planner's limit), empty and degenerate
clusters, non-finite points and inconsistent offsets; then bitwise invariants
of the GPU path (power-of-two scaling, sign flip, reflection, determinism,
independence from the other clusters of the frame) and the device Philox stream.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import parity  # noqa: E402
from paper_2012_12618_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2012_12618_amd import binding

    binding.load_library()  # raises if the HIP library is missing
    return binding


def _frame_from_clusters(clusters):
    th = np.concatenate([np.asarray(c[0], np.float32) for c in clusters]) if clusters else np.zeros(0, np.float32)
    vd = np.concatenate([np.asarray(c[1], np.float32) for c in clusters]) if clusters else np.zeros(0, np.float32)
    off = np.zeros(len(clusters) + 1, np.int32)
    off[1:] = np.cumsum([len(c[0]) for c in clusters])
    return th, vd, off


def _cluster(rng, n, outlier_frac=0.2, sigma=0.05):
    vx, vy = rng.uniform(-30, 30, 2)
    th = np.deg2rad(rng.uniform(-60, 60, n)).astype(np.float32)
    t = th.astype(np.float64)
    v = vx * np.cos(t) + vy * np.sin(t) + rng.normal(0, sigma, n)
    out = rng.random(n) < outlier_frac
    v[out] = rng.uniform(-40, 40, out.sum())
    return th, v.astype(np.float32)


def _parity(oracle_mod, name, theta, vd, offsets, H, tau, seed, **kw):
    g = parity.run_gpu(theta, vd, offsets, H, tau, seed, label=name)
    o = oracle_mod.estimate_velocity(theta, vd, offsets, H, tau, seed, debug=True)
    stats = parity.check(theta, vd, offsets, H, tau, seed, g, o, **kw)
    parity.report(name, stats)
    return g, o, stats


def test_device_philox_matches_oracle(rv, oracle_mod):
    rng = np.random.default_rng(5)
    n = 4096
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[:64] = 0
    key[:64] = 0
    ctr[:64, 0] = np.arange(64)
    print(f"[gpu] rv_philox4x32_10 n={n}", flush=True)
    got = rv.rv_philox4x32_10(torch.from_numpy(ctr.view(np.int32)).cuda(),
                              torch.from_numpy(key.view(np.int32)).cuda()).cpu().numpy().view(np.uint32)
    for t in range(n):
        assert np.array_equal(got[t], oracle_mod.philox4x32_10(ctr[t], key[t])), t


def test_parity_small_workload(rv, oracle_mod):
    frame, H, tau = synth.make_workload("small")
    _parity(oracle_mod, "small", frame.theta, frame.vd, frame.offsets, H, tau, synth.ransac_seed("small"))


def test_parity_dense_workload(rv, oracle_mod):
    frame, H, tau = synth.make_workload("dense")
    seed = synth.ransac_seed("dense")
    g, o, stats = _parity(oracle_mod, "dense", frame.theta, frame.vd, frame.offsets, H, tau, seed)
    # the benchmark's configuration (no debug outputs) gives the same results bitwise
    g2 = parity.run_gpu(frame.theta, frame.vd, frame.offsets, H, tau, seed, debug=False, bits=False,
                        label="dense-nodebug")
    for name in ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau"):
        assert np.array_equal(g2[name], g[name], equal_nan=name in ("vx", "vy", "heading")), name


@pytest.mark.parametrize("H", [1, 7, 64, 65, 256, 300, 1024])
def test_parity_random_frames(rv, oracle_mod, H):
    rng = np.random.default_rng(1000 + H)
    sizes = rng.integers(2, 301, size=40)
    clusters = [_cluster(rng, int(n)) for n in sizes]
    th, vd, off = _frame_from_clusters(clusters)
    _parity(oracle_mod, f"random-H{H}", th, vd, off, H, 0.15, 0xABCD0000 + H)


@pytest.mark.parametrize("case", range(6))
def test_parity_random_shapes(rv, oracle_mod, case):
    # Frames of the synthetic generator with drawn shapes: cluster count, size
    # law and range, outlier fractions (uniform and micro-Doppler band), noise,
    # H and tau.
    rng = np.random.default_rng(7000 + case)
    lo = int(rng.integers(2, 40))
    spec = synth.FrameSpec(int(rng.integers(1, 120)), ("uniform", "loguniform")[case % 2], lo,
                           int(rng.integers(lo, 1500)), p_uniform=float(rng.uniform(0.0, 0.5)),
                           p_band=float(rng.uniform(0.0, 0.3)), sigma=float(rng.uniform(0.01, 0.2)))
    frame = synth.make_frame(spec, 7100 + case)
    H = int(rng.choice([1, 33, 256, 513, 1024]))
    tau = float(np.float32(rng.choice([0.05, 0.15, 0.4])))
    _parity(oracle_mod, f"random-shape-{case}", frame.theta, frame.vd, frame.offsets, H, tau,
            0x7000 + case)


def test_parity_many_hypotheses(rv, oracle_mod):
    # H = 70,000 (hypothesis indexes above 2^16 in the Philox counter and in the
    # selection key; 274 scoring workgroups per cluster) on a few clusters.
    rng = np.random.default_rng(77)
    clusters = [_cluster(rng, n) for n in (2, 40, 130, 700)]
    th, vd, off = _frame_from_clusters(clusters)
    _parity(oracle_mod, "H70000", th, vd, off, 70_000, 0.15, 0x70000)


def test_parity_row_and_pass_boundaries(rv, oracle_mod):
    rng = np.random.default_rng(77)
    sizes = [2, 3, 63, 64, 65, 127, 128, 129, 1023, 1024, 1025, 1088, 2047, 2048, 2049, 3000]
    clusters = [_cluster(rng, n, outlier_frac=0.3) for n in sizes]
    th, vd, off = _frame_from_clusters(clusters)
    _parity(oracle_mod, "boundaries", th, vd, off, 257, 0.15, 42)


def test_parity_one_large_cluster(rv, oracle_mod):
    rng = np.random.default_rng(78)
    th, vd = _cluster(rng, 65536, outlier_frac=0.4)
    _parity(oracle_mod, "large-cluster", th, vd, np.array([0, 65536], np.int32), 128, 0.15, 9)


def test_parity_more_clusters_than_the_planner_orders(rv, oracle_mod):
    # Above 65,536 clusters the single-frame path scores in index order and
    # refits every cluster with a whole workgroup (no dispatch plan); the
    # hypothesis thread count grows with the cluster count (Sec. 3.1, Eq. 4).
    spec = synth.FrameSpec(70000, "uniform", 2, 64, p_uniform=0.2)
    frame = synth.make_frame(spec, seed=70)
    H, tau, seed = 64, 0.15, 0x70000
    g, o, stats = _parity(oracle_mod, "70k-clusters", frame.theta, frame.vd, frame.offsets, H, tau,
                          seed)
    assert stats["clusters"] == 70000
    # the same frame through the batched entry point: bitwise the same outputs
    dev = "cuda:0"
    t = torch.from_numpy(frame.theta).to(dev)
    v = torch.from_numpy(frame.vd).to(dev)
    off = torch.from_numpy(frame.offsets).to(dev)
    fo = torch.tensor([0, frame.n_clusters], dtype=torch.int32, device=dev)
    seeds = torch.tensor([seed], dtype=torch.int64, device=dev)
    print(f"[gpu] rv_estimate_velocity_batch 70k-clusters K={frame.n_clusters} H={H}", flush=True)
    b = rv.rv_estimate_velocity_batch(t, v, off, fo, seeds, H, tau, want_bits=True, debug=True)
    torch.cuda.synchronize()
    for name in ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau", "best_hyp",
                 "hyp_counts", "inlier_bits"):
        got = b[name].cpu().numpy()
        assert np.array_equal(got, g[name], equal_nan=name in ("vx", "vy", "heading")), name


def test_reused_outputs_too_small_are_refused(rv):
    # Outputs allocated for H = 256 reused with H = 1024, or for a smaller
    # frame: the binding raises before any launch.
    frame, H, tau = synth.make_workload("small")
    dev = torch.device("cuda:0")
    t = torch.from_numpy(frame.theta).to(dev)
    v = torch.from_numpy(frame.vd).to(dev)
    off = torch.from_numpy(frame.offsets).to(dev)
    out = rv.allocate_outputs(frame.n_clusters, frame.n_points, 256, dev, debug=True)
    with pytest.raises(ValueError, match="hyp_counts"):
        rv.rv_estimate_velocity(t, v, off, 1024, tau, 1, out=out)
    small = rv.allocate_outputs(frame.n_clusters - 1, frame.n_points, 256, dev)
    with pytest.raises(ValueError, match="vx"):
        rv.rv_estimate_velocity(t, v, off, 256, tau, 1, out=small)
    ok = rv.rv_estimate_velocity(t, v, off, 256, tau, 1, out=out)
    torch.cuda.synchronize()
    assert int((ok["status"] == 0).sum()) > 0


def test_parity_narrow_azimuth_clusters(rv, oracle_mod):
    spec = synth.FrameSpec(64, "uniform", 20, 400, p_uniform=0.2, theta_spread_deg=3.0)
    frame = synth.make_frame(spec, seed=55)
    _parity(oracle_mod, "narrow-azimuth", frame.theta, frame.vd, frame.offsets, 512, 0.15, 55)


def test_edge_cases(rv, oracle_mod):
    rng = np.random.default_rng(8)
    good = _cluster(rng, 50)
    nan_cl = _cluster(rng, 60)
    nan_cl[0][[1, 5]] = np.nan
    nan_cl[1][[7]] = np.inf
    nan_cl[1][[9]] = np.nan
    same = (np.full(30, 0.25, np.float32), rng.uniform(-3, 3, 30).astype(np.float32))
    close = (np.array([0.1, 0.1005, 0.1002], np.float32), np.array([1, 2, 3], np.float32))
    clusters = [([], []), ([0.3], [2.0]), good, same, nan_cl, close, ([0.0, 0.5], [1.0, 1.0])]
    th, vd, off = _frame_from_clusters(clusters)
    _parity(oracle_mod, "edge", th, vd, off, 96, 0.15, 3)

    # empty frame and a frame whose clusters are all empty
    g = parity.run_gpu(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(1, np.int32), 16, 0.15, 1,
                       label="empty")
    assert g["vx"].shape == (0,)
    g = parity.run_gpu(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(4, np.int32), 16, 0.15, 1,
                       label="empty-clusters")
    assert list(g["status"]) == [1, 1, 1]

    # inconsistent offsets: flagged, nothing outside [0, N) touched
    th = np.linspace(-1, 1, 40).astype(np.float32)
    vd = (3 * np.cos(th) - 2 * np.sin(th)).astype(np.float32)
    off = np.array([0, 20, 10, 45, 40], np.int32)
    g = parity.run_gpu(th, vd, off, 32, 0.15, 5, label="bad-offsets")
    o = oracle_mod.estimate_velocity(th, vd, off, 32, 0.15, 5)
    assert list(g["status"]) == list(o.status) == [0, 4, 4, 4]


def test_gpu_invariants_bitwise(rv):
    frame, H, tau = synth.make_workload("small")
    seed = 0x1234
    base = parity.run_gpu(frame.theta, frame.vd, frame.offsets, H, tau, seed, label="inv-base")
    again = parity.run_gpu(frame.theta, frame.vd, frame.offsets, H, tau, seed, label="inv-again")
    for name in ("vx", "vy", "heading", "n_inliers", "best_hyp", "hyp_counts", "inlier_bits"):
        assert np.array_equal(again[name], base[name]), f"not deterministic: {name}"
    # power-of-two scaling of v_d and tau
    for k2 in (-2, 3):
        f = 2.0**k2
        tau_s = float(np.float32(tau)) * f  # exactly the float32 tau scaled
        sc = parity.run_gpu(frame.theta, frame.vd * np.float32(f), frame.offsets, H, tau_s, seed, label=f"scale{k2}")
        assert np.array_equal(sc["hyp_counts"], base["hyp_counts"])
        assert np.array_equal(sc["inlier_bits"], base["inlier_bits"])
        assert np.array_equal(sc["vx"], base["vx"] * np.float32(f))
        assert np.array_equal(sc["vy"], base["vy"] * np.float32(f))
        assert np.array_equal(sc["heading"], base["heading"])
    # sign flip
    neg = parity.run_gpu(frame.theta, -frame.vd, frame.offsets, H, tau, seed, label="sign")
    assert np.array_equal(neg["hyp_counts"], base["hyp_counts"])
    assert np.array_equal(neg["vx"], -base["vx"]) and np.array_equal(neg["vy"], -base["vy"])
    dh = np.remainder(neg["heading"].astype(np.float64) - base["heading"], 2 * math.pi)
    assert np.abs(dh - math.pi).max() < 1e-6
    # reflection theta -> -theta
    ref = parity.run_gpu(-frame.theta, frame.vd, frame.offsets, H, tau, seed, label="reflect")
    assert np.array_equal(ref["hyp_counts"], base["hyp_counts"])
    assert np.array_equal(ref["vx"], base["vx"]) and np.array_equal(ref["vy"], -base["vy"])
    assert np.array_equal(ref["heading"], -base["heading"])


def test_results_independent_of_other_clusters(rv):
    frame, H, tau = synth.make_workload("small")
    seed = 77
    base = parity.run_gpu(frame.theta, frame.vd, frame.offsets, H, tau, seed, bits=False, label="mix-base")
    extra = synth.make_frame(synth.FrameSpec(300, "loguniform", 2, 3000, p_band=0.2), seed=5)
    both = synth.concat_frames([frame, extra])
    mixed = parity.run_gpu(both.theta, both.vd, both.offsets, H, tau, seed, bits=False, label="mix-appended")
    K = frame.n_clusters
    for name in ("vx", "vy", "heading", "n_inliers", "best_hyp", "n_near_tau"):
        assert np.array_equal(mixed[name][:K], base[name]), name
    assert np.array_equal(mixed["hyp_counts"][:K * H], base["hyp_counts"])
    # change every other cluster's data: clusters 0 and 5 keep their results
    vd2 = frame.vd.copy()
    for k in range(frame.n_clusters):
        if k not in (0, 5):
            lo, hi = frame.offsets[k], frame.offsets[k + 1]
            vd2[lo:hi] = vd2[lo:hi][::-1]
    other = parity.run_gpu(frame.theta, vd2, frame.offsets, H, tau, seed, bits=False, label="mix-changed")
    for k in (0, 5):
        assert other["vx"][k] == base["vx"][k] and other["n_inliers"][k] == base["n_inliers"][k]


def test_stage_timing_and_errors(rv):
    frame, H, tau = synth.make_workload("small")
    t = torch.from_numpy(frame.theta).cuda()
    v = torch.from_numpy(frame.vd).cuda()
    o = torch.from_numpy(frame.offsets).cuda()
    rv.rv_stage_timing(True)
    try:
        print("[gpu] stage timing x3", flush=True)
        for _ in range(3):
            rv.rv_estimate_velocity(t, v, o, H, tau, 1)
        ms, n = rv.rv_stage_times()
    finally:
        rv.rv_stage_timing(False)
    assert n == 3 and all(x > 0 for x in ms)
    out = rv.allocate_outputs(frame.n_clusters, frame.n_points, H, "cuda:0")
    out["workspace"] = out["workspace"][:100]
    with pytest.raises(rv.RVError) as e:
        rv.rv_estimate_velocity(t, v, o, H, tau, 1, out=out)
    assert e.value.code == rv.RV_ERR_WORKSPACE
    with pytest.raises(rv.RVError) as e:
        rv.rv_estimate_velocity(t, v, o, 0, tau, 1)
    assert e.value.code == rv.RV_ERR_INVALID_ARG
    torch.cuda.synchronize()


def test_parity_precision_stress_shape(rv, oracle_mod):
    """Clusters of the precision-stress configuration (65,536 points each, 40 %
    micro-Doppler band outliers, 4096 hypotheses), every output checked."""
    spec = synth.FrameSpec(8, "fixed", 65536, 65536, p_uniform=0.0, p_band=0.4)
    frame = synth.make_frame(spec, seed=505)
    _parity(oracle_mod, "stress-65536x4096", frame.theta, frame.vd, frame.offsets, 4096, 0.15, 505)


def test_side_stream_call_keeps_its_workspace(rv):
    """A call on a non-current stream with binding-allocated buffers: the
    workspace dropped on return must not be handed to the current stream's
    next allocation while the side stream still uses it."""
    frame, H, tau = synth.make_workload("small")
    seed = synth.ransac_seed("small")
    t = torch.from_numpy(frame.theta).cuda()
    v = torch.from_numpy(frame.vd).cuda()
    o = torch.from_numpy(frame.offsets).cuda()
    ref = rv.rv_estimate_velocity(t, v, o, H, tau, seed)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    print("[gpu] rv_estimate_velocity on a side stream", flush=True)
    for rep in range(3):
        got = rv.rv_estimate_velocity(t, v, o, H, tau, seed, stream=side)
        junk = torch.full((1 << 22,), float("nan"), device="cuda")  # current stream
        junk.add_(1.0)
        side.synchronize()
        torch.cuda.synchronize()
        for k in ("vx", "vy", "heading", "n_inliers", "status"):
            assert torch.equal(torch.nan_to_num(got[k].float(), 7.0), torch.nan_to_num(ref[k].float(), 7.0)), (rep, k)


def _small_frames():
    """Frames that take the one-launch path when no inlier mask is requested."""
    rng = np.random.default_rng(321)
    small, H, tau = synth.make_workload("small")
    yield "small-workload", small.theta, small.vd, small.offsets, H, tau, synth.ransac_seed("small")
    for H in (1, 7, 64, 65, 256):
        sizes = rng.integers(2, 301, size=40)
        th, vd, off = _frame_from_clusters([_cluster(rng, int(n)) for n in sizes])
        yield f"random-H{H}", th, vd, off, H, 0.15, 0x5A11 + H
    sizes = [2, 3, 63, 64, 65, 1023, 1024, 1025, 2049, 3000]
    th, vd, off = _frame_from_clusters([_cluster(rng, n, outlier_frac=0.3) for n in sizes])
    yield "row-and-pass-boundaries", th, vd, off, 256, 0.15, 4242
    good = _cluster(rng, 50)
    nan_cl = _cluster(rng, 60)
    nan_cl[0][[1, 5]] = np.nan
    nan_cl[1][[7, 9]] = np.inf
    same = (np.full(30, 0.25, np.float32), rng.uniform(-3, 3, 30).astype(np.float32))
    th, vd, off = _frame_from_clusters([([], []), ([0.3], [2.0]), good, same, nan_cl,
                                        ([0.0, 0.5], [1.0, 1.0])])
    yield "edge-clusters", th, vd, off, 200, 0.15, 77
    bad = off.copy()
    bad[3] = bad[4] + 5  # inconsistent offsets for two clusters
    yield "bad-offsets", th, vd, bad, 64, 0.15, 78


def test_small_frame_path_matches_three_kernel_path(rv, oracle_mod):
    """Without an inlier mask, small frames (<= 65,536 points, <= 256 hypotheses)
    run as one fused launch; every output equals the three-kernel path's
    (taken when the mask is requested) bitwise, and the oracle's by the protocol."""
    for name, th, vd, off, H, tau, seed in _small_frames():
        fused = parity.run_gpu(th, vd, off, H, tau, seed, debug=True, bits=False, label=f"{name}-fused")
        three = parity.run_gpu(th, vd, off, H, tau, seed, debug=True, bits=True, label=f"{name}-3k")
        for k in ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau", "hyp_counts", "best_hyp"):
            assert np.array_equal(fused[k], three[k], equal_nan=k in ("vx", "vy", "heading")), (name, k)
        if name != "bad-offsets":
            o = oracle_mod.estimate_velocity(th, vd, off, H, tau, seed, debug=True)
            parity.report(f"{name}-fused", parity.check(th, vd, off, H, tau, seed, fused, o))


def test_prepared_call_matches_the_plain_call(rv):
    f, n_hyp, tau = synth.make_workload("small")
    t = torch.from_numpy(f.theta).cuda()
    v = torch.from_numpy(f.vd).cuda()
    o = torch.from_numpy(f.offsets).cuda()
    out = rv.allocate_outputs(f.n_clusters, f.n_points, n_hyp, t.device, want_near=True,
                              debug=True)
    prepared = rv.PreparedEstimate(t, v, o, n_hyp, tau, out)
    for seed in (11, 12):
        print(f"[gpu] rv_estimate_velocity prepared seed={seed}", flush=True)
        a = {k: x.clone() for k, x in prepared(seed).items()}
        b = rv.rv_estimate_velocity(t, v, o, n_hyp, tau, seed, want_near=True, debug=True)
        torch.cuda.synchronize()
        assert set(a) == set(b)
        for key in a:
            x, y = a[key].cpu().numpy(), b[key].cpu().numpy()
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), (seed, key)
