"""GPU: the allocation-free entry point captured in a HIP graph (through
torch.cuda.graph) and replayed on new contents of the same input buffers, with
eager work and synchronisations between the replays: every replay gives bit for
bit the outputs of the workspace entry point on the same contents, on the
three-kernel path (frame-wide mask requested) and on the one-launch path.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2012_12618_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau", "inlier_bits", "hyp_counts",
        "best_hyp")


@pytest.fixture(scope="module")
def rv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2012_12618_amd import binding

    binding.load_library()
    return binding


def _variants(frame, n, seed):
    """n frames with the offsets of `frame`: azimuths turned and v_d re-drawn noise."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        th = (frame.theta + np.float32(0.01 * i)).astype(np.float32)
        vd = (frame.vd + rng.normal(0, 0.02, frame.vd.shape)).astype(np.float32)
        out.append((th, vd))
    return out


@pytest.mark.parametrize("case", ["three-kernel", "one-launch"])
def test_graph_replays_match_eager(rv, case):
    if case == "three-kernel":
        frame = synth.make_frame(synth.FrameSpec(200, "loguniform", 8, 1024, p_uniform=0.2), 61)
        H, tau, bits = 512, 0.15, True
    else:
        frame, H, tau = synth.make_workload("small")
        bits = False
    K, N = frame.n_clusters, frame.n_points
    t = torch.from_numpy(frame.theta).cuda()
    v = torch.from_numpy(frame.vd).cuda()
    o = torch.from_numpy(frame.offsets).cuda()
    out = rv.allocate_outputs(K, N, H, "cuda", want_near=True, want_bits=bits, debug=True)
    del out["workspace"]
    seed = 0x6161
    print(f"[gpu] noalloc eager warm-up {case} K={K} N={N}", flush=True)
    rv.rv_estimate_velocity_noalloc(t, v, o, H, tau, seed, out)  # scratch address taken here
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    print(f"[gpu] noalloc graph capture {case}", flush=True)
    with torch.cuda.graph(g):
        rv.rv_estimate_velocity_noalloc(t, v, o, H, tau, seed, out)
    torch.cuda.synchronize()
    for i, (th, vd) in enumerate(_variants(frame, 3, 62) + [(frame.theta, frame.vd)]):
        t.copy_(torch.from_numpy(th))
        v.copy_(torch.from_numpy(vd))
        torch.cuda.synchronize()
        print(f"[gpu] graph replay {i} {case}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        got = {k: out[k].cpu().numpy().copy() for k in KEYS if k in out}
        ref = rv.rv_estimate_velocity(t, v, o, H, tau, seed, want_near=True, want_bits=bits,
                                      debug=True)
        torch.cuda.synchronize()
        for k in got:
            assert np.array_equal(got[k].view(np.uint8), ref[k].cpu().numpy().view(np.uint8)), \
                (case, i, k)
    del g
