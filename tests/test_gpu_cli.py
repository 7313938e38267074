"""GPU: the estimator from a plain C++ program through the C ABI alone
(_lib/rv_cli: raw input files in, raw per-cluster results out, run as a child
process) gives bit for bit the results of the Python binding on the same frame;
a bad argument comes back as the library's own error text and exit status 1.
"""
import os
import subprocess

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2012_12618_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLI = os.path.join(ROOT, "paper_2012_12618_amd", "_lib", "rv_cli")


@pytest.fixture(scope="module")
def rv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    if not os.path.exists(CLI):
        pytest.fail(f"{CLI} is missing: build the library first")
    from paper_2012_12618_amd import binding

    binding.load_library()
    return binding


def _write_frame(dirname, frame):
    paths = [os.path.join(dirname, n) for n in ("theta.f32", "vd.f32", "offsets.i32")]
    np.ascontiguousarray(frame.theta, np.float32).tofile(paths[0])
    np.ascontiguousarray(frame.vd, np.float32).tofile(paths[1])
    np.ascontiguousarray(frame.offsets, np.int32).tofile(paths[2])
    return paths


def test_cli_matches_binding(rv, tmp_path):
    spec = synth.FrameSpec(300, "loguniform", 2, 2048, p_uniform=0.2, p_band=0.1)
    frame = synth.make_frame(spec, 91)
    H, tau, seed = 512, np.float32(0.15), 0x9191
    paths = _write_frame(str(tmp_path), frame)
    prefix = os.path.join(str(tmp_path), "out")
    print(f"[gpu] rv_cli K={frame.n_clusters} N={frame.n_points} H={H}", flush=True)
    res = subprocess.run([CLI, *paths, str(H), "%.9g" % tau, str(seed), prefix],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    assert res.stdout.startswith(f"clusters {frame.n_clusters} points {frame.n_points} ok ")
    got = {k: np.fromfile(f"{prefix}.{k}", dt) for k, dt in
           (("vx", np.float32), ("vy", np.float32), ("heading", np.float32),
            ("n_inliers", np.int32), ("status", np.uint8))}
    print("[gpu] rv_estimate_velocity (binding) on the same frame", flush=True)
    ref = rv.rv_estimate_velocity(torch.from_numpy(frame.theta).cuda(),
                                  torch.from_numpy(frame.vd).cuda(),
                                  torch.from_numpy(frame.offsets).cuda(), H, float(tau), seed,
                                  want_near=False)
    torch.cuda.synchronize()
    for k, a in got.items():
        b = ref[k].cpu().numpy()
        assert a.shape == b.shape, k
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), k
    assert int(res.stdout.split()[-1]) == int((got["status"] == 0).sum())


def test_cli_reports_library_errors(rv, tmp_path):
    frame = synth.make_frame(synth.FrameSpec(4, "uniform", 10, 20), 92)
    paths = _write_frame(str(tmp_path), frame)
    print("[gpu] rv_cli with n_hyp = 0 (refused on the host)", flush=True)
    res = subprocess.run([CLI, *paths, "0", "0.15", "1", os.path.join(str(tmp_path), "out")],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 1
    assert "n_hyp" in res.stderr
