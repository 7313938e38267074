"""GPU: the FP16 residual form of the batched path (tuning.fp16_min_points).

* every output except hyp_counts is bitwise the float32 form's, whatever
  clusters take the FP16 form (it changes how the best hypothesis is found,
  never which one);
* hyp_counts of an FP16-form cluster holds the FP16 counts, which are upper
  bounds of the float32 counts; clusters below the threshold keep the float32
  counts;
* inputs that stress the exact re-count: noiseless clusters where every valid
  hypothesis ties (more than 64 candidates per workgroup), ill-conditioned
  clusters (huge hypotheses, some beyond the FP16 range), non-finite points,
  duplicate azimuths (all hypotheses degenerate), two-point clusters;
* the precision-stress shape at full size (512 clusters of 65,536 points, 40 %
  micro-Doppler band outliers, 4096 hypotheses): FP16 form bitwise the float32
  form, and the parity protocol against the FP64 oracle on sampled clusters,
  with the error of each sampled result printed;
* the FP16 form captured in a HIP graph (replays with eager work and new
  contents in between) and inside the frame server.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import parity  # noqa: E402
from paper_2012_12618_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau", "best_hyp", "inlier_bits")


@pytest.fixture(scope="module")
def rv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2012_12618_amd import binding

    binding.load_library()
    return binding


def _run(rv, frame, frame_offsets, seeds, H, tau, fp16_min, label):
    t = rv.rv_tuning_default()
    t.fp16_min_points = fp16_min
    t.lanes_max_points = 0  # small clusters too take the FP16 form (lanes would take precedence)
    print(f"[gpu] batch fp16_min={fp16_min} {label} K={frame.n_clusters} N={frame.n_points} H={H}",
          flush=True)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    res = rv.rv_estimate_velocity_batch(dev(frame.theta), dev(frame.vd), dev(frame.offsets),
                                        dev(frame_offsets), dev(seeds.view(np.int64)), H, tau,
                                        tuning=t, want_bits=True, debug=True)
    torch.cuda.synchronize()
    return {k: x.cpu().numpy() for k, x in res.items()}


def _compare(frame, H, g32, g16, fp16_min, label):
    for k in KEYS:
        assert np.array_equal(g16[k], g32[k], equal_nan=k in ("vx", "vy", "heading")), (label, k)
    sizes = frame.sizes()
    c32 = g32["hyp_counts"].reshape(-1, H)
    c16 = g16["hyp_counts"].reshape(-1, H)
    in_fp16 = (sizes >= max(fp16_min, 2)) if fp16_min > 0 else np.zeros_like(sizes, bool)
    assert np.array_equal(c16[~in_fp16], c32[~in_fp16]), label
    assert np.all(c16[in_fp16] >= c32[in_fp16]), label
    if in_fp16.any():
        eq = float(np.mean(c16[in_fp16] == c32[in_fp16]))
        print(f"[fp16] {label}: {int(in_fp16.sum())} clusters in the FP16 form, "
              f"{eq:.4f} of their FP16 counts equal the float32 counts", flush=True)


def _single_frame(frame, label_seed):
    fo = np.array([0, frame.n_clusters], np.int32)
    seeds = np.array([synth.frame_seed("precision", label_seed)], np.uint64)
    return fo, seeds


@pytest.mark.parametrize("fp16_min", [2, 300, 1500])
def test_fp16_form_equals_float32_form(rv, fp16_min):
    batch, H, tau = synth.make_batch_workload("batched", n_frames=4)
    g32 = _run(rv, batch.frame, batch.frame_offsets, batch.seeds, H, tau, 0, "float32")
    g16 = _run(rv, batch.frame, batch.frame_offsets, batch.seeds, H, tau, fp16_min, "fp16")
    _compare(batch.frame, H, g32, g16, fp16_min, f"batched-4 fp16_min={fp16_min}")


def _stress_frame():
    """Clusters chosen to drive the exact re-count and the FP16 range guard."""
    rng = np.random.default_rng(77)
    th_l, v_l, sizes = [], [], []

    def add(th, v):
        th_l.append(np.asarray(th, np.float32))
        v_l.append(np.asarray(v, np.float32))
        sizes.append(len(th))

    # noiseless, no outliers: every valid hypothesis has the full count (ties everywhere)
    for n in (300, 2000):
        th = np.deg2rad(rng.uniform(-60, 60, n)).astype(np.float32)
        t = th.astype(np.float64)
        add(th, 12.0 * np.cos(t) - 7.0 * np.sin(t))
    # ill-conditioned: a 0.5 degree azimuth window, so seed pairs are near-collinear
    # and many hypotheses are huge; uniform outliers make some beyond 2^14 m/s
    for n in (700, 3000):
        th = np.deg2rad(20.0 + rng.uniform(-0.25, 0.25, n)).astype(np.float32)
        t = th.astype(np.float64)
        v = 5.0 * np.cos(t) + 3.0 * np.sin(t) + rng.normal(0, 0.05, n)
        out = rng.random(n) < 0.3
        v[out] = rng.uniform(-40, 40, out.sum())
        add(th, v)
    # non-finite points sprinkled into a normal cluster
    n = 1200
    th = np.deg2rad(rng.uniform(-60, 60, n)).astype(np.float32)
    t = th.astype(np.float64)
    v = -20.0 * np.cos(t) + 9.0 * np.sin(t) + rng.normal(0, 0.05, n)
    v = v.astype(np.float32)
    v[::37] = np.nan
    th[5::41] = np.inf
    add(th, v)
    # every azimuth equal: all hypotheses degenerate
    add(np.full(500, 0.3, np.float32), rng.uniform(-5, 5, 500))
    # two points
    add([0.1, 0.9], [1.0, 2.0])
    # large velocities near the edge of the FP16 range of the offsets
    n = 1500
    th = np.deg2rad(rng.uniform(-60, 60, n)).astype(np.float32)
    t = th.astype(np.float64)
    add(th, 9000.0 * np.cos(t) - 8000.0 * np.sin(t) + rng.normal(0, 0.05, n))
    offsets = np.zeros(len(sizes) + 1, np.int32)
    offsets[1:] = np.cumsum(sizes)
    k = len(sizes)
    return synth.Frame(theta=np.concatenate(th_l), vd=np.concatenate(v_l), offsets=offsets,
                       truth_vx=np.zeros(k), truth_vy=np.zeros(k),
                       kind=np.zeros(int(offsets[-1]), np.int8))


@pytest.mark.parametrize("case", range(6))
def test_fp16_form_equals_float32_form_random_shapes(rv, case):
    # One frame of drawn shape (sizes, outliers, noise, H, tau) in the FP16 form
    # for every cluster of at least two points against the float32 form.
    rng = np.random.default_rng(8000 + case)
    lo = int(rng.integers(2, 60))
    spec = synth.FrameSpec(int(rng.integers(1, 80)), ("uniform", "loguniform")[case % 2], lo,
                           int(rng.integers(lo, 6000)), p_uniform=float(rng.uniform(0.0, 0.6)),
                           p_band=float(rng.uniform(0.0, 0.4)), sigma=float(rng.uniform(0.01, 0.3)))
    frame = synth.make_frame(spec, 8100 + case)
    H = int(rng.choice([1, 64, 257, 1024]))
    tau = float(np.float32(rng.choice([0.02, 0.15, 1.0])))
    fo, seeds = _single_frame(frame, 8200 + case)
    g32 = _run(rv, frame, fo, seeds, H, tau, 0, f"float32 shape {case}")
    g16 = _run(rv, frame, fo, seeds, H, tau, 2, f"fp16 shape {case}")
    _compare(frame, H, g32, g16, 2, f"random shape {case} H={H} tau={tau}")


def test_fp16_form_on_stress_clusters(rv, oracle_mod):
    frame = _stress_frame()
    fo, seeds = _single_frame(frame, 1)
    for H in (512, 1000):
        g32 = _run(rv, frame, fo, seeds, H, 0.15, 0, f"stress H={H}")
        g16 = _run(rv, frame, fo, seeds, H, 0.15, 2, f"stress H={H}")
        _compare(frame, H, g32, g16, 2, f"stress H={H}")
    # the float32 form (hence the FP16 form) against the oracle on these clusters
    g32["mask"] = parity.unpack_bits(g32["inlier_bits"], frame.n_points)
    o = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, 0.15, int(seeds[0]),
                                     debug=True)
    stats = parity.check(frame.theta, frame.vd, frame.offsets, H, 0.15, int(seeds[0]), g32, o)
    parity.report("fp16-stress-clusters", stats)


def test_fp16_rejects_negative_threshold(rv):
    batch, H, tau = synth.make_batch_workload("served", n_frames=1)
    t = rv.rv_tuning_default()
    t.fp16_min_points = -1
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    with pytest.raises(rv.RVError) as e:
        rv.rv_estimate_velocity_batch(dev(batch.frame.theta), dev(batch.frame.vd),
                                      dev(batch.frame.offsets), dev(batch.frame_offsets),
                                      dev(batch.seeds.view(np.int64)), H, tau, tuning=t)
    assert e.value.code == rv.RV_ERR_INVALID_ARG


def test_fp16_precision_stress_full_size(rv, oracle_mod):
    """512 clusters x 65,536 points, 40 % band outliers, H = 4096: the FP16 form
    against the float32 form (every cluster) and the FP64 oracle (sampled)."""
    frame, H, tau = synth.make_workload("precision")
    fo = np.array([0, frame.n_clusters], np.int32)
    seeds = np.array([synth.ransac_seed("precision")], np.uint64)
    g32 = _run(rv, frame, fo, seeds, H, tau, 0, "precision float32")
    g16 = _run(rv, frame, fo, seeds, H, tau, 1024, "precision fp16")
    _compare(frame, H, g32, g16, 1024, "precision-512x65536")
    ids = [0, 255, 511]
    o = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, int(seeds[0]),
                                     cluster_ids=ids, debug=True)
    g32["mask"] = parity.unpack_bits(g32["inlier_bits"], frame.n_points)
    stats = parity.check(frame.theta, frame.vd, frame.offsets, H, tau, int(seeds[0]), g32, o,
                         cluster_ids=ids)
    parity.report("fp16-precision-sampled", stats)
    for i, k in enumerate(ids):
        print(f"[fp16] cluster {k}: vx {g16['vx'][k]:.6f} (oracle {o.vx[i]:.6f}, "
              f"err {abs(g16['vx'][k] - o.vx[i]):.2e}), vy {g16['vy'][k]:.6f} (oracle {o.vy[i]:.6f}, "
              f"err {abs(g16['vy'][k] - o.vy[i]):.2e}), heading err "
              f"{abs(np.remainder(g16['heading'][k] - o.heading[i] + np.pi, 2 * np.pi) - np.pi):.2e}, "
              f"inliers {g16['n_inliers'][k]} (oracle {o.n_inliers[i]})", flush=True)


def test_fp16_form_in_a_captured_graph(rv):
    """Graph replays of the FP16 form, with eager work and new contents between
    replays, equal the eager float32 form bitwise (every output but hyp_counts)."""
    batch, H, tau = synth.make_batch_workload("served", n_frames=3)
    f = batch.frame
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    t, v, o = dev(f.theta), dev(f.vd), dev(f.offsets)
    fo, sd = dev(batch.frame_offsets), dev(batch.seeds.view(np.int64))
    K, N, F = f.n_clusters, f.n_points, batch.n_frames
    t16 = rv.rv_tuning_default()
    t16.fp16_min_points = 64
    t16.lanes_max_points = 0
    eager = rv.allocate_batch_outputs(F, K, N, H, "cuda:0", want_bits=True, debug=True)
    replay = rv.allocate_batch_outputs(F, K, N, H, "cuda:0", want_bits=True, debug=True)
    print(f"[gpu] rv_graph_capture_batch fp16_min=64 F={F} K={K} N={N} H={H}", flush=True)
    graph = rv.rv_graph_capture_batch(t, v, o, fo, sd, H, tau, replay, tuning=t16)
    try:
        for rep in range(3):
            if rep == 1:
                v.neg_()
            if rep == 2:
                sd.add_(11)
            rv.rv_estimate_velocity_batch(t, v, o, fo, sd, H, tau, out=eager)  # float32 form
            _ = torch.ones(1000, device="cuda").sum().item()
            torch.cuda.synchronize()
            print(f"[gpu] fp16 graph replay {rep}", flush=True)
            graph.launch()
            torch.cuda.synchronize()
            for k in KEYS:
                a, b = eager[k].cpu().numpy(), replay[k].cpu().numpy()
                assert np.array_equal(a, b, equal_nan=k in ("vx", "vy", "heading")), (rep, k)
            assert np.all(replay["hyp_counts"].cpu().numpy() >= eager["hyp_counts"].cpu().numpy())
    finally:
        graph.destroy()


def test_server_with_fp16_form_matches_single_frames(rv):
    """A frame server whose tuning enables the FP16 form answers every frame
    with the float32 single-frame results."""
    batch, H, tau = synth.make_batch_workload("served", n_frames=4)
    frames = [batch.frame_slice(f) for f in range(batch.n_frames)]
    cfg = rv.rv_server_config_default()
    cfg.n_hyp, cfg.tau = H, tau
    cfg.max_batch_frames, cfg.n_streams = 2, 2
    cfg.tuning.fp16_min_points = 128
    print(f"[gpu] server fp16_min=128 frames={len(frames)}", flush=True)
    server = rv.RVServer(cfg)
    try:
        seeds = [synth.frame_seed("served", 900 + i) for i in range(len(frames))]
        tickets = [server.submit(f.theta, f.vd, f.offsets, s) for f, s in zip(frames, seeds)]
        got = [server.result(tk) for tk in tickets]
    finally:
        server.destroy()
    for f, s, g in zip(frames, seeds, got):
        alone = parity.run_gpu(f.theta, f.vd, f.offsets, H, tau, s, debug=False, bits=False,
                               label="fp16-server-alone")
        for k in ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau"):
            assert np.array_equal(g[k], alone[k], equal_nan=k in ("vx", "vy", "heading")), k
