"""GPU: the batched form (many frames, one launch sequence, persistent scoring).

* every cluster's outputs are bitwise those of a single-frame call on its frame
  (with that frame's seed), including per-hypothesis counts and inlier bits;
* parity with the oracle per frame (tests/parity.py protocol);
* tuning (register rows per size bucket, persistent grid size, the size up to
  which clusters score with lanes = hypotheses) never changes a result bit; the
  lanes = hypotheses form equals the rows form on every cluster size it takes,
  edge clusters and hypothesis counts included;
* a captured HIP graph replayed several times, with eager work and
  synchronisations between replays and new input contents, matches the eager
  call every time;
* empty frames, empty batches and degenerate clusters.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import parity  # noqa: E402
from paper_2012_12618_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau", "best_hyp")


@pytest.fixture(scope="module")
def rv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2012_12618_amd import binding

    binding.load_library()
    return binding


def _dev(batch):
    f = batch.frame
    return (torch.from_numpy(f.theta).cuda(), torch.from_numpy(f.vd).cuda(),
            torch.from_numpy(f.offsets).cuda(), torch.from_numpy(batch.frame_offsets).cuda(),
            torch.from_numpy(batch.seeds.view(np.int64)).cuda())


def _run_batch(rv, batch, H, tau, label, tuning=None, bits=True):
    print(f"[gpu] rv_estimate_velocity_batch {label} F={batch.n_frames} K={batch.frame.n_clusters} "
          f"N={batch.frame.n_points} H={H}", flush=True)
    t, v, o, fo, sd = _dev(batch)
    res = rv.rv_estimate_velocity_batch(t, v, o, fo, sd, H, tau, tuning=tuning, want_bits=bits,
                                        debug=True)
    torch.cuda.synchronize()
    out = {k: x.cpu().numpy() for k, x in res.items()}
    if bits:
        out["mask"] = parity.unpack_bits(out["inlier_bits"], batch.frame.n_points)
    return out


def _with_edge_frames(batch):
    """Insert an empty frame and a frame of tiny/degenerate clusters."""
    frames = [batch.frame_slice(f) for f in range(batch.n_frames)]
    tiny = synth.Frame(
        theta=np.array([0.1, 0.2, 0.3, 0.3, 0.3, -0.5, 0.4], np.float32),
        vd=np.array([1.0, 2.0, 0.5, 0.6, 0.7, 3.0, 3.1], np.float32),
        offsets=np.array([0, 1, 2, 5, 7, 7], np.int32),
        truth_vx=np.zeros(5), truth_vy=np.zeros(5), kind=np.zeros(7, np.int8))
    empty = synth.Frame(theta=np.zeros(0, np.float32), vd=np.zeros(0, np.float32),
                        offsets=np.zeros(1, np.int32), truth_vx=np.zeros(0), truth_vy=np.zeros(0),
                        kind=np.zeros(0, np.int8))
    frames = frames[:2] + [empty, tiny] + frames[2:]
    fo = np.zeros(len(frames) + 1, np.int64)
    fo[1:] = np.cumsum([f.n_clusters for f in frames])
    seeds = np.array([synth.frame_seed("batched", 100 + i) for i in range(len(frames))], np.uint64)
    return synth.Batch(frame=synth.concat_frames(frames), frame_offsets=fo.astype(np.int32), seeds=seeds)


def test_batch_equals_single_frames(rv):
    b0, H, tau = synth.make_batch_workload("batched", n_frames=5)
    batch = _with_edge_frames(b0)
    g = _run_batch(rv, batch, H, tau, "vs-single")
    fo = batch.frame_offsets
    for f in range(batch.n_frames):
        fr = batch.frame_slice(f)
        c0, c1 = int(fo[f]), int(fo[f + 1])
        p0 = int(batch.frame.offsets[c0])
        s = parity.run_gpu(fr.theta, fr.vd, fr.offsets, H, tau, int(batch.seeds[f]), label=f"frame{f}")
        for k in KEYS:
            assert np.array_equal(g[k][c0:c1], s[k], equal_nan=k in ("vx", "vy", "heading")), (f, k)
        assert np.array_equal(g["hyp_counts"][c0 * H:c1 * H], s["hyp_counts"]), f
        assert np.array_equal(g["mask"][p0:p0 + fr.n_points], s["mask"]), f


@pytest.mark.parametrize("case", range(3))
def test_batch_of_drawn_shapes_equals_single_frames(rv, case):
    # Frames of drawn shapes (cluster count, size law and range, outliers,
    # noise) in one batch with drawn lanes and rows tuning: every output of
    # every frame equals its single-frame call's bit for bit.
    rng = np.random.default_rng(9000 + case)
    frames = []
    for f in range(int(rng.integers(2, 9))):
        lo = int(rng.integers(2, 50))
        spec = synth.FrameSpec(int(rng.integers(0, 150)), ("uniform", "loguniform")[f % 2], lo,
                               int(rng.integers(lo, 3000)), p_uniform=float(rng.uniform(0, 0.5)),
                               p_band=float(rng.uniform(0, 0.3)), sigma=float(rng.uniform(0.01, 0.2)))
        frames.append(synth.make_frame(spec, 9100 + 10 * case + f))
    fo = np.zeros(len(frames) + 1, np.int64)
    fo[1:] = np.cumsum([fr.n_clusters for fr in frames])
    seeds = np.array([synth.frame_seed("batched", 9200 + 10 * case + i) for i in range(len(frames))],
                     np.uint64)
    batch = synth.Batch(frame=synth.concat_frames(frames), frame_offsets=fo.astype(np.int32),
                        seeds=seeds)
    H = int(rng.choice([1, 100, 256, 700]))
    tau = float(np.float32(rng.choice([0.05, 0.15, 0.5])))
    tuning = rv.rv_tuning_default()
    tuning.lanes_max_points = int(rng.choice([0, 32, 64, 256]))
    for b in range(len(tuning.rows_max)):
        tuning.rows_max[b] = int(rng.integers(1, 17))
    g = _run_batch(rv, batch, H, tau, f"drawn-{case}", tuning=tuning)
    for f, fr in enumerate(frames):
        c0, c1 = int(fo[f]), int(fo[f + 1])
        p0 = int(batch.frame.offsets[c0])
        s = parity.run_gpu(fr.theta, fr.vd, fr.offsets, H, tau, int(seeds[f]), label=f"drawn{case}-{f}")
        for k in KEYS:
            assert np.array_equal(g[k][c0:c1], s[k], equal_nan=k in ("vx", "vy", "heading")), (f, k)
        assert np.array_equal(g["hyp_counts"][c0 * H:c1 * H], s["hyp_counts"]), f
        assert np.array_equal(g["mask"][p0:p0 + fr.n_points], s["mask"]), f


def test_batch_parity_with_oracle(rv, oracle_mod):
    batch, H, tau = synth.make_batch_workload("served", n_frames=3)
    g = _run_batch(rv, batch, H, tau, "oracle")
    fo = batch.frame_offsets
    for f in range(batch.n_frames):
        fr = batch.frame_slice(f)
        c0, c1 = int(fo[f]), int(fo[f + 1])
        p0 = int(batch.frame.offsets[c0])
        sub = {k: g[k][c0:c1] for k in KEYS}
        sub["hyp_counts"] = g["hyp_counts"][c0 * H:c1 * H]
        sub["mask"] = g["mask"][p0:p0 + fr.n_points]
        o = oracle_mod.estimate_velocity(fr.theta, fr.vd, fr.offsets, H, tau, int(batch.seeds[f]), debug=True)
        stats = parity.check(fr.theta, fr.vd, fr.offsets, H, tau, int(batch.seeds[f]), sub, o)
        parity.report(f"batch-frame{f}", stats)


def test_tuning_never_changes_results(rv):
    batch, H, tau = synth.make_batch_workload("batched", n_frames=4)
    base = _run_batch(rv, batch, H, tau, "tune-default")
    for rows, per_cu, lanes in (([1] * 8, 1, 0), ([4, 4, 8, 8, 12, 12, 16, 16], 3, 256),
                                ([16, 2, 3, 5, 7, 9, 11, 13], 0, 130)):
        t = rv.RVTuning.from_dict({"rows_max": rows, "blocks_per_cu": per_cu,
                                   "lanes_max_points": lanes})
        g = _run_batch(rv, batch, H, tau, f"tune-{per_cu}-{lanes}", tuning=t)
        for k in KEYS + ("hyp_counts", "inlier_bits"):
            assert np.array_equal(g[k], base[k], equal_nan=k in ("vx", "vy", "heading")), k


@pytest.mark.parametrize("H", [1, 64, 300, 512])
def test_lanes_form_equals_rows_form(rv, H):
    # Clusters of 2..300 points (every size up to the LDS tile of 256 and past
    # it), with outliers, non-finite points, equal azimuths and two-point
    # clusters, scored with lanes = hypotheses up to 256 points against the
    # rows form everywhere: every output and every hypothesis count bitwise.
    rng = np.random.default_rng(300 + H)
    clusters = []
    for n in list(range(2, 70)) + [95, 127, 128, 129, 200, 255, 256, 257, 300]:
        vx, vy = rng.uniform(-30, 30, 2)
        th = np.deg2rad(rng.uniform(-60, 60, n)).astype(np.float32)
        v = vx * np.cos(th.astype(np.float64)) + vy * np.sin(th.astype(np.float64))
        v = v + rng.normal(0, 0.05, n)
        out = rng.random(n) < 0.25
        v[out] = rng.uniform(-40, 40, out.sum())
        clusters.append((th, v.astype(np.float32)))
    th, v = clusters[10]
    th[3], v[5] = np.nan, np.inf
    clusters.append((np.full(20, 0.3, np.float32), rng.uniform(-2, 2, 20).astype(np.float32)))
    theta = np.concatenate([c[0] for c in clusters])
    vd = np.concatenate([c[1] for c in clusters])
    off = np.zeros(len(clusters) + 1, np.int32)
    off[1:] = np.cumsum([len(c[0]) for c in clusters])
    half = len(clusters) // 2
    frame = synth.Frame(theta=theta, vd=vd, offsets=off, truth_vx=np.zeros(len(clusters)),
                        truth_vy=np.zeros(len(clusters)), kind=np.zeros(len(theta), np.int8))
    batch = synth.Batch(frame=frame, frame_offsets=np.array([0, half, len(clusters)], np.int32),
                        seeds=np.array([0x1A2B, 0x3C4D5E6F7], np.uint64))
    rows = rv.RVTuning.from_dict({"rows_max": [16] * 8, "lanes_max_points": 0})
    lanes = rv.RVTuning.from_dict({"rows_max": [16] * 8, "lanes_max_points": 256})
    a = _run_batch(rv, batch, H, 0.15, f"rows-H{H}", tuning=rows)
    b = _run_batch(rv, batch, H, 0.15, f"lanes-H{H}", tuning=lanes)
    for k in KEYS + ("hyp_counts", "inlier_bits"):
        assert np.array_equal(a[k], b[k], equal_nan=k in ("vx", "vy", "heading")), k
    assert int((a["status"] == 0).sum()) > len(clusters) // 2


def test_graph_replays_match_eager(rv):
    batch, H, tau = synth.make_batch_workload("served", n_frames=4)
    t, v, o, fo, sd = _dev(batch)
    K, N, F = batch.frame.n_clusters, batch.frame.n_points, batch.n_frames
    eager_out = rv.allocate_batch_outputs(F, K, N, H, "cuda:0", want_bits=True, debug=True)
    graph_out = rv.allocate_batch_outputs(F, K, N, H, "cuda:0", want_bits=True, debug=True)
    print(f"[gpu] rv_graph_capture_batch F={F} K={K} N={N} H={H}", flush=True)
    graph = rv.rv_graph_capture_batch(t, v, o, fo, sd, H, tau, graph_out)
    try:
        for rep in range(4):
            if rep == 2:  # new contents in the captured buffers: sign-flipped Doppler values
                v.neg_()
            if rep == 3:
                sd.add_(7)
            rv.rv_estimate_velocity_batch(t, v, o, fo, sd, H, tau, out=eager_out)
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work in between
            torch.cuda.synchronize()
            print(f"[gpu] graph replay {rep}", flush=True)
            graph.launch()
            torch.cuda.synchronize()
            for k in KEYS + ("hyp_counts", "inlier_bits"):
                a, b = eager_out[k].cpu().numpy(), graph_out[k].cpu().numpy()
                assert np.array_equal(a, b, equal_nan=k in ("vx", "vy", "heading")), (rep, k)
    finally:
        graph.destroy()


def test_batch_edge_cases(rv):
    # no clusters at all
    t = torch.zeros(0, device="cuda")
    o = torch.zeros(1, dtype=torch.int32, device="cuda")
    fo = torch.zeros(2, dtype=torch.int32, device="cuda")
    sd = torch.zeros(1, dtype=torch.int64, device="cuda")
    r = rv.rv_estimate_velocity_batch(t, t, o, fo, sd, 64, 0.15)
    assert r["vx"].numel() == 0
    # argument errors
    b, H, tau = synth.make_batch_workload("served", n_frames=2)
    tt, vv, oo, ffo, ssd = _dev(b)
    with pytest.raises(ValueError):
        rv.rv_estimate_velocity_batch(tt, vv, oo, ffo, ssd[:1], H, tau)
    bad = rv.RVTuning.from_dict({"rows_max": [0] * 8, "blocks_per_cu": 0})
    with pytest.raises(rv.RVError):
        rv.rv_estimate_velocity_batch(tt, vv, oo, ffo, ssd, H, tau, tuning=bad)


def test_autotuned_setting_gives_identical_results(rv):
    from paper_2012_12618_amd import tuner

    batch, H, tau = synth.make_batch_workload("batched", n_frames=3)
    t, v, o, fo, sd = _dev(batch)
    print("[gpu] autotune batched F=3", flush=True)
    tune, report = tuner.autotune(t, v, o, fo, sd, H, tau, offsets_host=batch.frame.offsets, reps=2)
    assert report["best_ms"] > 0 and len(report["trials"]) >= 2
    a = _run_batch(rv, batch, H, tau, "autotuned", tuning=tune)
    b = _run_batch(rv, batch, H, tau, "default")
    for k in KEYS + ("hyp_counts", "inlier_bits"):
        assert np.array_equal(a[k], b[k], equal_nan=k in ("vx", "vy", "heading")), k


def test_full_batch_in_bench_configuration(rv, oracle_mod):
    """The full batched workload (256 frames) as the benchmark runs it (captured
    graph, no debug outputs): equal bit for bit to an eager debug call, and in
    parity with the oracle on 12 frames spread over the batch."""
    batch, H, tau = synth.make_batch_workload("batched")
    t, v, o, fo, sd = _dev(batch)
    K, N, F = batch.frame.n_clusters, batch.frame.n_points, batch.n_frames
    print(f"[gpu] full batch graph F={F} K={K} N={N} H={H}", flush=True)
    out = rv.allocate_batch_outputs(F, K, N, H, "cuda:0", want_near=True)
    graph = rv.rv_graph_capture_batch(t, v, o, fo, sd, H, tau, out)
    try:
        graph.launch()
        torch.cuda.synchronize()
    finally:
        graph.destroy()
    g = _run_batch(rv, batch, H, tau, "full-debug")
    for k in ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau"):
        assert np.array_equal(out[k].cpu().numpy(), g[k], equal_nan=k in ("vx", "vy", "heading")), k
    for f in np.linspace(0, F - 1, 12).astype(int):
        fr = batch.frame_slice(int(f))
        c0, c1 = int(batch.frame_offsets[f]), int(batch.frame_offsets[f + 1])
        p0 = int(batch.frame.offsets[c0])
        sub = {k: g[k][c0:c1] for k in KEYS}
        sub["hyp_counts"] = g["hyp_counts"][c0 * H:c1 * H]
        sub["mask"] = g["mask"][p0:p0 + fr.n_points]
        ref = oracle_mod.estimate_velocity(fr.theta, fr.vd, fr.offsets, H, tau, int(batch.seeds[f]),
                                           debug=True)
        parity.report(f"full-batch-frame{f}",
                      parity.check(fr.theta, fr.vd, fr.offsets, H, tau, int(batch.seeds[f]), sub, ref))
