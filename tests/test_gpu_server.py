"""GPU: the frame server (request queue, budget admission, continuous batching).

* every frame's results are bitwise those of rv_estimate_velocity on that frame
  alone with its seed, while other frames are queued and in flight, under an
  arena budget small enough that admission has to wait for memory, and every
  served frame passes the acceptance protocol against the FP64 oracle (kept
  hypothesis, inlier mask, refit, heading; Sec. 3.1-3.2);
* empty and degenerate frames go through; frames larger than the budget and
  malformed offsets are refused; a full queue answers RV_ERR_BUSY.
"""
import threading

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


def _frames():
    b, H, tau = synth.make_batch_workload("served", n_frames=6)
    frames = [b.frame_slice(f) for f in range(b.n_frames)]
    tiny = synth.Frame(theta=np.array([0.1, 0.2, 0.3, 0.3, 0.3, -0.5, 0.4], np.float32),
                       vd=np.array([1.0, 2.0, 0.5, 0.6, 0.7, 3.0, 3.1], np.float32),
                       offsets=np.array([0, 1, 2, 5, 7, 7], np.int32),
                       truth_vx=np.zeros(5), truth_vy=np.zeros(5), kind=np.zeros(7, np.int8))
    empty = synth.Frame(theta=np.zeros(0, np.float32), vd=np.zeros(0, np.float32),
                        offsets=np.zeros(1, np.int32), truth_vx=np.zeros(0), truth_vy=np.zeros(0),
                        kind=np.zeros(0, np.int8))
    return frames + [tiny, empty], H, tau


def test_results_same_alone_and_in_the_mix(rv, oracle_mod):
    frames, H, tau = _frames()
    cfg = rv.rv_server_config_default()
    cfg.n_hyp, cfg.tau = H, tau
    cfg.keep_inlier_bits = 1
    biggest = max(rv.rv_server_frame_bytes(cfg, f.n_clusters, f.n_points) for f in frames)
    cfg.hbm_budget_bytes = int(2.5 * biggest)  # at most two or three frames on the device
    cfg.max_batch_frames, cfg.n_streams = 3, 2
    jobs = [(i % len(frames), synth.frame_seed("served", 500 + i)) for i in range(24)]
    print(f"[gpu] server budget={cfg.hbm_budget_bytes} jobs={len(jobs)}", flush=True)
    server = rv.RVServer(cfg)
    try:
        tickets = [None] * len(jobs)

        def submit(part):
            for j in part:
                f = frames[jobs[j][0]]
                tickets[j] = server.submit(f.theta, f.vd, f.offsets, jobs[j][1])

        threads = [threading.Thread(target=submit, args=(range(t, len(jobs), 3),)) for t in range(3)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        got = [server.result(tk) for tk in tickets]
        st = server.stats()
    finally:
        server.destroy()
    assert st["frames_done"] == len(jobs) and st["arena_peak_bytes"] <= cfg.hbm_budget_bytes
    assert st["max_batch_frames_seen"] >= 2  # frames did share launches
    total = {}
    for j, (fi, seed) in enumerate(jobs):
        f = frames[fi]
        if f.n_clusters == 0:
            assert got[j]["vx"].size == 0
            continue
        alone = parity.run_gpu(f.theta, f.vd, f.offsets, H, tau, seed, debug=True, bits=True,
                               label=f"alone job{j}")
        for k in KEYS:
            assert np.array_equal(got[j][k], alone[k], equal_nan=k in ("vx", "vy", "heading")), (j, k)
        assert got[j]["times"]["done_ns"] >= got[j]["times"]["launched_ns"] >= got[j]["times"]["submitted_ns"]
        # the served result against the oracle (no per-hypothesis GPU counts:
        # an ambiguous selection is judged from the oracle's bands)
        g = dict(got[j])
        g["mask"] = parity.unpack_bits(g["inlier_bits"], f.n_points)
        o = oracle_mod.estimate_velocity(f.theta, f.vd, f.offsets, H, tau, seed, debug=True)
        stats = parity.check(f.theta, f.vd, f.offsets, H, tau, seed, g, o, check_hyp=False)
        for key, val in stats.items():
            total[key] = max(total.get(key, 0), val) if key.startswith("max") else total.get(key, 0) + val
    parity.report("served vs oracle", total)
    assert total["clusters"] > 0


def test_refusals(rv):
    frames, H, tau = _frames()
    f = frames[0]
    cfg = rv.rv_server_config_default()
    cfg.n_hyp, cfg.tau = H, tau
    cfg.hbm_budget_bytes = 1 << 20
    server = rv.RVServer(cfg)
    try:
        with pytest.raises(rv.RVError) as e:
            server.submit(f.theta, f.vd, f.offsets, 1)  # larger than the whole arena
        assert e.value.code == rv.RV_ERR_INVALID_ARG and "budget" in str(e.value)
        bad = np.array([0, 5, 3, 7], np.int32)
        with pytest.raises(rv.RVError):
            server.submit(np.zeros(7, np.float32), np.zeros(7, np.float32), bad, 1)
        with pytest.raises(rv.RVError):
            server.submit(np.zeros(7, np.float32), np.zeros(7, np.float32),
                          np.array([0, 3, 6], np.int32), 1)  # does not end at n_points
        with pytest.raises(rv.RVError):
            server.result(12345)
    finally:
        server.destroy()


def test_full_queue_answers_busy(rv):
    frame, H, tau = synth.make_workload("dense")
    small, _, _ = synth.make_workload("small")
    cfg = rv.rv_server_config_default()
    cfg.n_hyp, cfg.tau = 4096, tau  # the first frame keeps the only slot busy for milliseconds
    cfg.hbm_budget_bytes = 2 * rv.rv_server_frame_bytes(cfg, frame.n_clusters, frame.n_points)
    cfg.n_streams, cfg.max_waiting_frames, cfg.max_batch_frames = 1, 1, 1
    print("[gpu] server busy test", flush=True)
    server = rv.RVServer(cfg)
    try:
        t_big = server.submit(frame.theta, frame.vd, frame.offsets, 1)
        codes = []
        tks = []
        for i in range(4):
            try:
                tks.append(server.submit(small.theta, small.vd, small.offsets, 10 + i))
            except rv.RVError as e:
                codes.append(e.code)
        assert rv.RV_ERR_BUSY in codes
        assert server.stats()["busy_rejections"] == len(codes)
        server.result(t_big)
        for tk in tks:
            server.result(tk)
    finally:
        server.destroy()


def test_pinned_submit_matches_copied_submit(rv):
    # Frames held in pinned host memory and queued without a copy give every
    # output of the copied submit bit for bit; several tickets in flight read
    # the same pinned arrays.
    frames, H, tau = _frames()
    cfg = rv.rv_server_config_default()
    cfg.n_hyp, cfg.tau = H, tau
    cfg.keep_inlier_bits = 1
    cfg.max_batch_frames, cfg.n_streams = 4, 2
    pinned = [tuple(torch.from_numpy(a).pin_memory() for a in (f.theta, f.vd, f.offsets))
              for f in frames]
    jobs = [(i % len(frames), synth.frame_seed("served", 700 + i)) for i in range(16)]
    print(f"[gpu] server pinned submits jobs={len(jobs)}", flush=True)
    server = rv.RVServer(cfg)
    try:
        t_pin = [server.submit_pinned(*pinned[fi], seed) for fi, seed in jobs]
        t_cpy = [server.submit(frames[fi].theta, frames[fi].vd, frames[fi].offsets, seed)
                 for fi, seed in jobs]
        for j, (a, b) in enumerate(zip(t_pin, t_cpy)):
            ra, rb = server.result(a), server.result(b)
            for k in KEYS:
                assert np.array_equal(ra[k].view(np.uint8), rb[k].view(np.uint8)), (j, k)
        # Pageable arrays read in place give the same results (synchronous copies).
        f = frames[0]
        tp = server.submit_pinned(torch.from_numpy(f.theta), torch.from_numpy(f.vd),
                                  torch.from_numpy(f.offsets), 4242)
        tc = server.submit(f.theta, f.vd, f.offsets, 4242)
        ra, rb = server.result(tp), server.result(tc)
        for k in KEYS:
            assert np.array_equal(ra[k].view(np.uint8), rb[k].view(np.uint8)), ("pageable", k)
        with pytest.raises(ValueError, match="float32"):
            server.submit_pinned(pinned[0][0].double(), *pinned[0][1:], 1)
    finally:
        server.destroy()
