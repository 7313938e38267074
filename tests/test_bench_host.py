"""CPU: host-side logic of bench.py.

* more than one GPU is refused with a message (this estimator runs on one GPU);
* the kernel-code hash ignores comments and blank lines but not code;
* a committed counter summary is read back only while the kernel code is the
  code it was taken on;
* the latency loops run every frame with a fresh seed and Python's garbage
  collector off, and turn it back on.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_code_hash_ignores_comments_only(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f() {\n    return 1;  // one\n}\n")
    b.write_text("// a header comment\n\nint f() {\n    return 1;\n}\n\n")
    c.write_text("int f() {\n    return 2;\n}\n")
    assert bench.kernel_code_sha256(str(a)) == bench.kernel_code_sha256(str(b))
    assert bench.kernel_code_sha256(str(a)) != bench.kernel_code_sha256(str(c))


def test_counter_summaries_are_read_back_only_for_their_code():
    import json
    import re

    src = os.path.join(ROOT, "paper_2012_12618_amd", "csrc", "rv.hip")
    path = os.path.join(ROOT, "profiles", "score_kernel_dense_counters.md")
    if not os.path.exists(path):
        pytest.skip("no committed counter summary")
    rec = json.loads(re.search(r"```json\n(.*?)\n```", open(path).read(), re.S).group(1))
    current = rec.get("kernel_code_sha256") == bench.kernel_code_sha256(src)
    assert (bench.profiled_traffic("dense") is not None) == current
    issue = bench.profiled_valu_issue("dense")
    assert (issue is not None) == current
    if current:
        assert 0.0 < issue["valu_instructions_per_simd_cycle"] < 1.0


def test_oracle_error_summary_per_cluster_bound():
    import numpy as np

    o_vx = np.array([10.0, -3.0, 0.5, 7.0])
    o_vy = np.array([1.0, 2.0, -0.25, 7.0])
    o_hd = np.arctan2(o_vy, o_vx)
    vx = o_vx.astype(np.float32)
    vy = o_vy.astype(np.float32)
    vy[2] = np.float32(-0.25 + 1e-6)  # one result beyond float32 rounding
    best = np.array([5, 6, 7, 8])
    o_best = np.array([5, 6, 7, 9])  # the last cluster kept another hypothesis
    e = bench.oracle_error_summary(vx, vy, np.arctan2(vy, vx).astype(np.float32), best,
                                   o_vx, o_vy, o_hd, o_best)
    assert e["clusters"] == 4 and e["same_hypothesis"] == 3
    assert e["dv_within_float32_rounding"] == 2
    assert abs(e["abs_dv_mps"]["max"] - 1e-6) < 1e-8
    assert e["abs_dheading_rad"]["max"] < 1e-5


def test_timed_frames_runs_every_frame_with_the_collector_off():
    import gc

    seen = []

    def call(i, seed):
        seen.append((i, seed, gc.isenabled()))
        return float(i)

    assert gc.isenabled()
    out = bench.timed_frames(call, "small", 5)
    assert out == [0.0, 1.0, 2.0, 3.0, 4.0]
    assert [s[0] for s in seen] == list(range(5))
    assert len({s[1] for s in seen}) == 5  # a fresh seed per frame
    assert not any(s[2] for s in seen)
    assert gc.isenabled()  # restored afterwards
