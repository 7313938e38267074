"""GPU: inputs and outputs in pinned host memory (read and written by the
kernels through their device mapping, no copies) give bit for bit the results
of the same call on device memory, on the one-launch small-frame path and on
the three-kernel path with the frame-wide mask; a prepared call estimates
smaller frames held at the start of its buffers; pageable memory is refused
before anything runs.
"""
import ctypes

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


def _pinned_outputs(rv, K, N, H, bits, debug):
    out = rv.allocate_outputs(K, N, H, "cpu", want_near=True, want_bits=bits, debug=debug)
    ws = torch.empty(max(rv.rv_workspace_bytes(K, N, H), 1), dtype=torch.uint8, device="cuda")
    out = {k: (v.pin_memory() if k != "workspace" else ws) for k, v in out.items()}
    return out


def _compare(label, host, dev):
    for k in KEYS:
        if k in dev:
            a = host[k].numpy()
            b = dev[k].cpu().numpy()
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (label, k)


@pytest.mark.parametrize("case", ["small", "three-kernel"])
def test_pinned_host_frame_matches_device_frame(rv, case):
    if case == "small":
        f, H, tau = synth.make_workload("small")
        bits, seed = False, synth.ransac_seed("small")
    else:
        f = synth.make_frame(synth.FrameSpec(300, "loguniform", 8, 2048, p_uniform=0.2), 81)
        H, tau, bits, seed = 512, 0.15, True, 0x8181
    K, N = f.n_clusters, f.n_points
    ht = torch.from_numpy(f.theta).pin_memory()
    hv = torch.from_numpy(f.vd).pin_memory()
    ho = torch.from_numpy(f.offsets).pin_memory()
    out = _pinned_outputs(rv, K, N, H, bits, debug=True)
    print(f"[gpu] rv_estimate_velocity pinned host {case} K={K} N={N} H={H}", flush=True)
    got = rv.rv_estimate_velocity(ht, hv, ho, H, tau, seed, out=out)
    torch.cuda.synchronize()
    print(f"[gpu] rv_estimate_velocity device {case}", flush=True)
    ref = rv.rv_estimate_velocity(ht.cuda(), hv.cuda(), ho.cuda(), H, tau, seed, want_near=True,
                                  want_bits=bits, debug=True)
    torch.cuda.synchronize()
    _compare(case, got, ref)


def test_prepared_call_on_smaller_frames(rv):
    frames = [synth.make_frame(synth.FrameSpec(64, "uniform", 20, 200, p_uniform=0.2), 900 + i)
              for i in range(3)]
    H, tau = 256, 0.15
    K = max(f.n_clusters for f in frames)
    N = max(f.n_points for f in frames)
    ht = torch.empty(N, dtype=torch.float32).pin_memory()
    hv = torch.empty(N, dtype=torch.float32).pin_memory()
    ho = torch.empty(K + 1, dtype=torch.int32).pin_memory()
    out = _pinned_outputs(rv, K, N, H, bits=False, debug=True)
    prep = rv.PreparedEstimate(ht, hv, ho, H, tau, out)
    for i, f in enumerate(frames):
        n, k = f.n_points, f.n_clusters
        ht[:n].numpy()[:] = f.theta
        hv[:n].numpy()[:] = f.vd
        ho[:k + 1].numpy()[:] = f.offsets
        print(f"[gpu] prepared pinned call frame {i} K={k} N={n}", flush=True)
        got = prep(7000 + i, n_points=n, n_clusters=k)
        torch.cuda.synchronize()
        got = {key: v[:k * H] if key == "hyp_counts" else v[:k] for key, v in got.items()}
        ref = rv.rv_estimate_velocity(torch.from_numpy(f.theta).cuda(), torch.from_numpy(f.vd).cuda(),
                                      torch.from_numpy(f.offsets).cuda(), H, tau, 7000 + i,
                                      want_near=True, debug=True)
        torch.cuda.synchronize()
        _compare(f"prepared-{i}", got, ref)
    with pytest.raises(ValueError, match="does not fit"):
        prep(1, n_points=N + 1, n_clusters=K)


def test_pageable_memory_is_refused(rv):
    lib = rv.load_library()
    a = np.zeros(1024, np.float32)
    d = ctypes.c_void_p()
    assert lib.rv_host_device_pointer(ctypes.c_void_p(a.ctypes.data), ctypes.byref(d)) == -1
    assert d.value is None
    assert "not pinned" in rv.rv_last_error()
    with pytest.raises(ValueError, match="pinned"):
        rv.rv_estimate_velocity(torch.zeros(10), torch.zeros(10),
                                torch.tensor([0, 10], dtype=torch.int32).pin_memory(), 4, 0.15, 1)


def test_views_map_at_their_offset(rv):
    # A view into pinned memory maps to the allocation's device address plus
    # the view's byte offset (host-side queries only).
    t = torch.empty(4096, dtype=torch.float32).pin_memory()
    base = rv.host_device_pointer(t)
    for off in (1, 5, 1000, 4095):
        assert rv.host_device_pointer(t[off:]) == base + 4 * off, off
