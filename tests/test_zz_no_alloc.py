"""The allocation-free entry point (rv_estimate_velocity_noalloc, through the C
ABI) against rv_estimate_velocity on the same inputs: every output bit for bit,
on two calls in a row that share the library's device scratch, the second with
a smaller frame (and a different launch path), then the smaller frame's results
against the FP64 oracle by the acceptance protocol.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import parity  # noqa: E402
from paper_2012_12618_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau", "inlier_bits", "hyp_counts",
        "best_hyp")


@pytest.fixture(scope="module")
def rv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2012_12618_amd import binding

    binding.load_library()  # raises if the HIP library is missing
    return binding


def _on_gpu(frame):
    return (torch.from_numpy(frame.theta).cuda(), torch.from_numpy(frame.vd).cuda(),
            torch.from_numpy(frame.offsets).cuda())


def _both(rv, label, frame, n_hyp, tau, seed, bits):
    t, v, o = _on_gpu(frame)
    K, N = frame.n_clusters, frame.n_points
    assert rv.rv_workspace_bytes(K, N, n_hyp) <= rv.RV_NOALLOC_SCRATCH_BYTES
    out = rv.allocate_outputs(K, N, n_hyp, t.device, want_near=True, want_bits=bits, debug=True)
    del out["workspace"]
    print(f"[gpu] rv_estimate_velocity_noalloc {label} K={K} N={N} H={n_hyp} seed={seed:#x}",
          flush=True)
    got = rv.rv_estimate_velocity_noalloc(t, v, o, n_hyp, tau, seed, out)
    torch.cuda.synchronize()
    got = {k: x.cpu().numpy() for k, x in got.items()}
    print(f"[gpu] rv_estimate_velocity {label} (reference)", flush=True)
    ref = rv.rv_estimate_velocity(t, v, o, n_hyp, tau, seed, want_near=True, want_bits=bits,
                                  debug=True)
    torch.cuda.synchronize()
    ref = {k: x.cpu().numpy() for k, x in ref.items()}
    assert set(got) == set(ref)
    for k in KEYS:
        if k in ref:
            assert np.array_equal(got[k].view(np.uint8), ref[k].view(np.uint8)), (label, k)
    return got


def test_noalloc_matches_workspace_entry_point(rv, oracle_mod):
    # First call: 512 clusters of log-uniform [8, 4096] points (the dense
    # frame's mix), H = 1024, frame-wide mask requested: the three-kernel path
    # with the dispatch planner.
    big_spec = synth.FrameSpec(512, "loguniform", 8, 4096, p_uniform=0.15, p_band=0.15)
    big = synth.make_frame(big_spec, 71)
    _both(rv, "first", big, 1024, 0.15, 0x7101, bits=True)
    # Second call, smaller, on the scratch the first one left: 64 clusters of
    # U{20..200} points, H = 256, no mask: the one-launch path.
    small, H, tau = synth.make_workload("small")
    assert small.n_points < big.n_points
    seed = synth.ransac_seed("small")
    g = _both(rv, "second", small, H, tau, seed, bits=False)
    o = oracle_mod.estimate_velocity(small.theta, small.vd, small.offsets, H, tau, seed, debug=True)
    g = dict(g)
    parity.report("noalloc-second",
                  parity.check(small.theta, small.vd, small.offsets, H, tau, seed, g, o))
    # Third call, smaller again, with the mask: the three-kernel path once more.
    mid = synth.make_frame(synth.FrameSpec(100, "loguniform", 8, 512, p_uniform=0.2), 72)
    assert mid.n_points < big.n_points
    _both(rv, "third", mid, 512, 0.15, 0x7103, bits=True)


def test_noalloc_refuses_a_frame_beyond_its_scratch(rv):
    n = 5_500_000
    assert rv.rv_workspace_bytes(1, n, 64) > rv.RV_NOALLOC_SCRATCH_BYTES
    t = torch.zeros(n, dtype=torch.float32, device="cuda")
    o = torch.tensor([0, n], dtype=torch.int32, device="cuda")
    out = rv.allocate_outputs(1, n, 64, t.device, want_near=False)
    del out["workspace"]
    print(f"[gpu] rv_estimate_velocity_noalloc oversized N={n} (refused on the host)", flush=True)
    with pytest.raises(rv.RVError, match="allocation-free") as e:
        rv.rv_estimate_velocity_noalloc(t, t, o, 64, 0.15, 1, out)
    assert e.value.code == rv.RV_ERR_WORKSPACE
