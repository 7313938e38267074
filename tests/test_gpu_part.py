"""GPU: a frame estimated in parts gives bit for bit the whole-frame call's
outputs.  rv_estimate_velocity_part (each part's clusters drawing their
hypotheses with their index in the whole frame, the part's points found
through the frame's own offsets and the part's first point) is checked on the
one-launch small-frame path and on the three-kernel path, with parts that start
on and off 32-point boundaries, and one part against the FP64 oracle by the
acceptance protocol; rv_estimate_velocity_pipelined (the frame copied from
pinned host memory part by part, each part's estimate overlapping the next
part's copy) for several part counts, with device and pinned host outputs.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import parity  # noqa: E402
from paper_2012_12618_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

PER_CLUSTER = ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau", "best_hyp")


@pytest.fixture(scope="module")
def rv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2012_12618_amd import binding

    binding.load_library()
    return binding


def _cuts(frame, n_parts):
    """Cluster boundaries that cut the frame into about n_parts parts of equal points."""
    off = frame.offsets
    want = np.linspace(0, frame.n_points, n_parts + 1)[1:-1]
    cuts = np.searchsorted(off, want)
    return sorted({0, *[int(c) for c in cuts if 0 < c < frame.n_clusters], frame.n_clusters})


def _whole(rv, frame, H, tau, seed, bits):
    print(f"[gpu] rv_estimate_velocity whole K={frame.n_clusters} N={frame.n_points} H={H}",
          flush=True)
    got = rv.rv_estimate_velocity(torch.from_numpy(frame.theta).cuda(),
                                  torch.from_numpy(frame.vd).cuda(),
                                  torch.from_numpy(frame.offsets).cuda(), H, tau, seed,
                                  want_near=True, want_bits=bits, debug=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in got.items()}


def _same(label, got, whole, c0, c1, H):
    for k in PER_CLUSTER:
        assert np.array_equal(np.asarray(got[k]).view(np.uint8), whole[k][c0:c1].view(np.uint8)), \
            (label, k)
    assert np.array_equal(got["hyp_counts"], whole["hyp_counts"][c0 * H:c1 * H]), label


def _frame(case):
    if case == "small":
        frame, H, tau = synth.make_workload("small")
        return frame, H, tau, synth.ransac_seed("small")
    spec = synth.FrameSpec(600, "loguniform", 8, 4096, p_uniform=0.15, p_band=0.15)
    return synth.make_frame(spec, 77), 1024, 0.15, 0x7707


@pytest.mark.parametrize("case", ["small", "dense-mix"])
def test_parts_match_whole_frame(rv, case):
    frame, H, tau, seed = _frame(case)
    bits = case != "small"
    whole = _whole(rv, frame, H, tau, seed, bits)
    N = frame.n_points
    whole_mask = parity.unpack_bits(whole["inlier_bits"], N) if bits else None
    d_t = torch.from_numpy(frame.theta).cuda()
    d_v = torch.from_numpy(frame.vd).cuda()
    d_o = torch.from_numpy(frame.offsets).cuda()
    cuts = _cuts(frame, 3 if case == "small" else 5)
    assert len(cuts) >= 3
    aligned = 0
    for c0, c1 in zip(cuts[:-1], cuts[1:]):
        p0, p1 = int(frame.offsets[c0]), int(frame.offsets[c1])
        aligned += p0 % 32 == 0
        print(f"[gpu] rv_estimate_velocity_part {case} clusters [{c0}, {c1}) points [{p0}, {p1})",
              flush=True)
        got = rv.rv_estimate_velocity_part(d_t[p0:p1], d_v[p0:p1], d_o[c0:c1 + 1], c0, p0, H, tau,
                                           seed, want_near=True, want_bits=bits, debug=True)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in got.items()}
        _same(f"part {c0}", got, whole, c0, c1, H)
        if bits:
            assert np.array_equal(parity.unpack_bits(got["inlier_bits"], p1 - p0),
                                  whole_mask[p0:p1]), c0
    if case == "dense-mix":
        assert aligned < len(cuts) - 1  # some part starts off a 32-point boundary


def test_part_against_oracle(rv, oracle_mod):
    # The oracle computes the part's clusters with their frame indexes.
    spec = synth.FrameSpec(96, "uniform", 20, 300, p_uniform=0.2)
    frame, H, tau, seed = synth.make_frame(spec, 78), 256, 0.15, 0x7808
    c0, c1 = 40, 96
    p0, p1 = int(frame.offsets[c0]), int(frame.offsets[c1])
    print(f"[gpu] rv_estimate_velocity_part oracle check clusters [{c0}, {c1})", flush=True)
    got = rv.rv_estimate_velocity_part(torch.from_numpy(frame.theta[p0:p1]).cuda(),
                                       torch.from_numpy(frame.vd[p0:p1]).cuda(),
                                       torch.from_numpy(frame.offsets[c0:c1 + 1]).cuda(), c0, p0,
                                       H, tau, seed, want_near=True, want_bits=True, debug=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    ids = np.arange(c0, c1)
    o = oracle_mod.estimate_velocity(frame.theta, frame.vd, frame.offsets, H, tau, seed,
                                     cluster_ids=ids, debug=True)
    # The protocol reads the GPU side in the whole frame's layout: the part's
    # outputs go to its clusters' frame indexes, and only those are checked.
    K = frame.n_clusters
    g = {}
    for k in PER_CLUSTER:
        full = np.zeros(K, dtype=got[k].dtype)
        full[c0:c1] = got[k]
        g[k] = full
    g["hyp_counts"] = np.zeros(K * H, dtype=np.int32)
    g["hyp_counts"][c0 * H:c1 * H] = got["hyp_counts"]
    mask = np.zeros(frame.n_points, dtype=bool)
    mask[p0:p1] = parity.unpack_bits(got["inlier_bits"], p1 - p0)
    g["mask"] = mask
    parity.report("part-oracle", parity.check(frame.theta, frame.vd, frame.offsets, H, tau, seed,
                                              g, o, cluster_ids=ids))


@pytest.mark.parametrize("case", ["small", "dense-mix"])
def test_pipelined_matches_whole_frame(rv, case):
    frame, H, tau, seed = _frame(case)
    whole = _whole(rv, frame, H, tau, seed, bits=False)
    K, N = frame.n_clusters, frame.n_points
    h_t = torch.from_numpy(frame.theta).pin_memory()
    h_v = torch.from_numpy(frame.vd).pin_memory()
    h_o = torch.from_numpy(frame.offsets).pin_memory()
    dev_in = (torch.empty(N, device="cuda"), torch.empty(N, device="cuda"),
              torch.empty(K + 1, dtype=torch.int32, device="cuda"))
    copy_stream = torch.cuda.Stream()
    for n_parts in (1, 3, 8, rv.RV_MAX_PARTS):
        for host_out in (False, True):
            out = rv.allocate_outputs(K, N, H, "cuda", want_near=True, debug=True)
            if host_out:
                out = {k: (v.cpu().pin_memory() if k != "workspace" else v) for k, v in out.items()}
            print(f"[gpu] rv_estimate_velocity_pipelined {case} parts={n_parts} "
                  f"host_out={host_out}", flush=True)
            got = rv.rv_estimate_velocity_pipelined(h_t, h_v, h_o, n_parts, H, tau, seed,
                                                    device_inputs=dev_in, out=out,
                                                    copy_stream=copy_stream)
            torch.cuda.synchronize()
            got = {k: v.cpu().numpy() for k, v in got.items()}
            _same(f"pipelined {n_parts} {host_out}", got, whole, 0, K, H)


def test_pipelined_edge_frames(rv):
    # Empty and one-point clusters at the cuts, one cluster larger than a part,
    # more parts than clusters, a frame of empty clusters only: every output as
    # the whole-frame call's, and nothing to do for a frame without clusters.
    rng = np.random.default_rng(606)

    def cluster(n):
        th = np.deg2rad(rng.uniform(-60, 60, n)).astype(np.float32)
        vx, vy = rng.uniform(-30, 30, 2)
        v = vx * np.cos(th.astype(np.float64)) + vy * np.sin(th.astype(np.float64))
        v = v + rng.normal(0, 0.05, n)
        out = rng.random(n) < 0.2
        v[out] = rng.uniform(-40, 40, out.sum())
        return th, v.astype(np.float32)

    frames = {
        "mixed": [0, 1, 5, 0, 200, 1, 3000, 2, 0, 64, 65, 0],
        "few-clusters": [700, 3, 900],
        "all-empty": [0, 0, 0, 0],
        "one-cluster": [4097],
    }
    H, tau = 96, 0.15
    copy_stream = torch.cuda.Stream()
    for name, sizes in frames.items():
        parts = [cluster(n) for n in sizes]
        th = np.concatenate([p[0] for p in parts])
        vd = np.concatenate([p[1] for p in parts])
        off = np.zeros(len(sizes) + 1, np.int32)
        off[1:] = np.cumsum(sizes)
        K, N = len(sizes), int(off[-1])
        print(f"[gpu] rv_estimate_velocity whole edge {name} K={K} N={N}", flush=True)
        whole = rv.rv_estimate_velocity(torch.from_numpy(th).cuda(), torch.from_numpy(vd).cuda(),
                                        torch.from_numpy(off).cuda(), H, tau, 0x606,
                                        want_near=True, debug=True)
        torch.cuda.synchronize()
        whole = {k: v.cpu().numpy() for k, v in whole.items()}
        h_t = torch.from_numpy(th).pin_memory()
        h_v = torch.from_numpy(vd).pin_memory()
        h_o = torch.from_numpy(off).pin_memory()
        for n_parts in (1, 2, 5, rv.RV_MAX_PARTS):
            print(f"[gpu] rv_estimate_velocity_pipelined edge {name} parts={n_parts}", flush=True)
            got = rv.rv_estimate_velocity_pipelined(h_t, h_v, h_o, n_parts, H, tau, 0x606,
                                                    debug=True, copy_stream=copy_stream)
            torch.cuda.synchronize()
            got = {k: v.cpu().numpy() for k, v in got.items()}
            _same(f"edge {name} {n_parts}", got, whole, 0, K, H)
    empty = torch.zeros(0, dtype=torch.float32).pin_memory()
    got = rv.rv_estimate_velocity_pipelined(empty, empty,
                                            torch.zeros(1, dtype=torch.int32).pin_memory(), 4,
                                            H, tau, 1, copy_stream=copy_stream)
    torch.cuda.synchronize()
    assert all(v.numel() == 0 for v in got.values())


def test_pipelined_calls_in_a_row_reuse_buffers(rv):
    # Two pipelined calls enqueued back to back on the same device buffers,
    # no synchronisation between them: the second call's copies wait for the
    # first call's estimates, so both frames' results are the whole-frame ones.
    spec = synth.FrameSpec(400, "loguniform", 8, 4096, p_uniform=0.15)
    fa, fb = synth.make_frame(spec, 201), synth.make_frame(spec, 202)
    H, tau = 1024, 0.15
    N = max(fa.n_points, fb.n_points)
    K = max(fa.n_clusters, fb.n_clusters)
    dev_in = (torch.empty(N, device="cuda"), torch.empty(N, device="cuda"),
              torch.empty(K + 1, dtype=torch.int32, device="cuda"))
    copy_stream = torch.cuda.Stream()
    outs = []
    host = []
    for f, seed in ((fa, 0x2011), (fb, 0x2022)):
        h = tuple(torch.from_numpy(a).pin_memory() for a in (f.theta, f.vd, f.offsets))
        host.append(h)  # kept alive until the stream is done
        print(f"[gpu] rv_estimate_velocity_pipelined back to back K={f.n_clusters}", flush=True)
        outs.append(rv.rv_estimate_velocity_pipelined(*h, 4, H, tau, seed, device_inputs=dev_in,
                                                      debug=True, copy_stream=copy_stream))
    torch.cuda.synchronize()
    for (f, seed), got in zip(((fa, 0x2011), (fb, 0x2022)), outs):
        whole = _whole(rv, f, H, tau, seed, bits=False)
        got = {k: v.cpu().numpy() for k, v in got.items()}
        _same(f"back-to-back {seed:#x}", got, whole, 0, f.n_clusters, H)
