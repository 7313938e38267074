"""The C-ABI library (CPU only): it loads, exports every function include/rv.h
declares, sizes workspaces, and rejects bad arguments on the host before any
HIP call is made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rv.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2012_12618_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        from paper_2012_12618_amd import build

        build.build()
    return binding.load_library()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rv_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    assert {"rv_estimate_velocity", "rv_workspace_bytes", "rv_last_error"} <= set(names)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_header_constants_match_binding():
    from paper_2012_12618_amd import binding

    text = open(HEADER).read()
    consts = dict(re.findall(r"(RV_[A-Z_]+)\s*=\s*(-?\d+)", text))
    for name, value in consts.items():
        assert getattr(binding, name) == int(value), name
    assert "RV_MIN_SEED_SEPARATION 1e-3" in text and binding.RV_MIN_SEED_SEPARATION == 1e-3
    assert "RV_NEAR_TAU_WINDOW 1e-5" in text and binding.RV_NEAR_TAU_WINDOW == 1e-5
    assert "RV_MAX_PARTS 64" in text and binding.RV_MAX_PARTS == 64


def test_noalloc_scratch_limit(lib):
    # The allocation-free entry point refuses a frame whose workspace exceeds
    # its device scratch before any HIP call (fake pointers: never used).
    from paper_2012_12618_amd import binding

    text = open(HEADER).read()
    assert "RV_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)" in text
    assert binding.RV_NOALLOC_SCRATCH_BYTES == 96 << 20
    fake = ctypes.c_void_p(4096)
    n = 5_500_000
    assert binding.rv_workspace_bytes(1, n, 64) > binding.RV_NOALLOC_SCRATCH_BYTES
    assert binding.rv_workspace_bytes(4096, 2_723_399, 1024) <= binding.RV_NOALLOC_SCRATCH_BYTES
    rc = lib.rv_estimate_velocity_noalloc(fake, fake, fake, 1, n, 64, 0.15, 1, fake, fake, fake,
                                          fake, fake, None, None, None, None, None)
    assert rc == -2
    assert "allocation-free" in lib.rv_last_error().decode()


def test_host_device_pointer_refuses_unmapped_memory(lib):
    # NULL and pageable memory are refused on the host (-1) and leave *device NULL
    import numpy as np

    d = ctypes.c_void_p(1234)
    assert lib.rv_host_device_pointer(None, ctypes.byref(d)) == -1 and d.value is None
    a = np.zeros(16, np.float32)
    d = ctypes.c_void_p(1234)
    assert lib.rv_host_device_pointer(ctypes.c_void_p(a.ctypes.data), ctypes.byref(d)) == -1
    assert d.value is None
    assert lib.rv_host_device_pointer(ctypes.c_void_p(a.ctypes.data), None) == -1


def test_workspace_bytes(lib):
    from paper_2012_12618_amd import binding

    a = binding.rv_workspace_bytes(64, 7000, 256)
    b = binding.rv_workspace_bytes(4096, 2_700_000, 1024)
    assert 0 < a < b
    assert binding.rv_workspace_bytes(-1, 10, 8) == 0
    # 20 bytes per point (float2 + float + float2) and 12 per cluster, 256-byte aligned sections
    assert 20 * 2_700_000 + 12 * 4096 <= b <= 20 * 2_700_000 + 12 * 4096 + 6 * 256
    assert binding.rv_workspace_bytes(4096, 2_700_000, 1) == b  # independent of n_hyp
    assert b % 256 == 0


def _call(lib, **kw):
    args = dict(theta=None, vd=None, offsets=None, K=1, N=10, H=16, tau=0.15, seed=1,
                vx=None, vy=None, heading=None, n_in=None, status=None, near=None, bits=None,
                hc=None, best=None, ws=None, ws_bytes=0, stream=None)
    args.update(kw)
    P = ctypes.c_void_p
    return lib.rv_estimate_velocity(
        args["theta"], args["vd"], args["offsets"], args["K"], args["N"], args["H"], args["tau"],
        args["seed"], args["vx"], args["vy"], args["heading"], args["n_in"], args["status"],
        args["near"], args["bits"], args["hc"], args["best"], args["ws"], args["ws_bytes"],
        args["stream"])


def test_host_argument_checks(lib):
    fake = ctypes.c_void_p(4096)  # never dereferenced: the checks fail first
    ok = dict(theta=fake, vd=fake, offsets=fake, vx=fake, vy=fake, heading=fake, n_in=fake,
              status=fake)
    cases = [
        (dict(ok, H=0), -1, "n_hyp"),
        (dict(ok, H=(1 << 20) + 1), -1, "n_hyp"),
        (dict(ok, tau=0.0), -1, "tau"),
        (dict(ok, tau=float("nan")), -1, "tau"),
        (dict(ok, tau=float("inf")), -1, "tau"),
        (dict(ok, K=-1), -1, "n_clusters"),
        (dict(ok, N=-5), -1, "n_points"),
        (dict(ok, N=2**31), -1, "n_points"),
        (dict(ok, offsets=None), -1, "cluster_offsets"),
        (dict(ok, theta=None), -1, "theta"),
        (dict(ok, vx=None), -1, "output"),
        (dict(ok, status=None), -1, "output"),
        (dict(ok), -2, "workspace"),
        (dict(ok, ws=fake, ws_bytes=10), -2, "workspace"),
        (dict(ok, ws=ctypes.c_void_p(4096 + 8), ws_bytes=1 << 30), -2, "aligned"),
    ]
    for kw, code, word in cases:
        assert _call(lib, **kw) == code, kw
        assert word in lib.rv_last_error().decode()
    # nothing to do: no clusters -> OK without touching the GPU
    assert _call(lib, offsets=fake, K=0, N=0, ws=fake, ws_bytes=1 << 20) == 0
    assert lib.rv_last_error().decode() == ""


def test_binding_checks_output_sizes(lib):
    # Caller-supplied outputs smaller than what the kernels write are refused
    # on the host (host tensors stand in for device ones: only sizes matter).
    import torch

    from paper_2012_12618_amd import binding

    cpu = torch.device("cpu")
    K, N, H = 10, 1000, 256
    out = binding.allocate_outputs(K, N, H, cpu, want_bits=True, debug=True)
    assert len(binding._output_ptrs(out, cpu, K, N, H)) == 9
    for k, n, h, name in ((K, N, 1024, "hyp_counts"), (K + 1, N, H, "vx"),
                          (K, N + 32, H, "inlier_bits")):
        with pytest.raises(ValueError, match=name):
            binding._output_ptrs(out, cpu, k, n, h)
    out["best_hyp"] = out["best_hyp"][:5]
    with pytest.raises(ValueError, match="best_hyp"):
        binding._output_ptrs(out, cpu, K, N, H)


def test_philox_hook_argument_checks(lib):
    assert lib.rv_philox4x32_10(None, None, None, -1, None) == -1
    assert lib.rv_philox4x32_10(None, None, None, 0, None) == 0
    assert lib.rv_philox4x32_10(None, None, None, 5, None) == -1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2012_12618_amd import binding

    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        binding.load_library()


def test_batch_host_argument_checks(lib):
    from paper_2012_12618_amd import binding

    fake = ctypes.c_void_p(4096)
    t = binding.rv_tuning_default()
    assert list(t.rows_max) == [16] * binding.RV_TUNE_BUCKETS and t.blocks_per_cu == 0
    assert binding.rv_batch_workspace_bytes(0, 10, 10, 8) == 0
    a = binding.rv_batch_workspace_bytes(4, 100, 10000, 512)
    b = binding.rv_batch_workspace_bytes(4, 100, 20000, 512)
    assert 0 < a < b

    def call(**kw):
        args = dict(theta=fake, vd=fake, off=fake, fo=fake, seeds=fake, F=2, K=10, N=100, H=64,
                    tau=0.15, out=fake, tuning=None, ws=None, ws_bytes=0)
        args.update(kw)
        tune = args["tuning"]
        return lib.rv_estimate_velocity_batch(
            args["theta"], args["vd"], args["off"], args["fo"], args["seeds"], args["F"], args["K"],
            args["N"], args["H"], args["tau"], args["out"], args["out"], args["out"], args["out"],
            args["out"], None, None, None, None, None if tune is None else ctypes.byref(tune),
            args["ws"], args["ws_bytes"], None)

    cases = [
        (dict(F=0), -1, "n_frames"),
        (dict(seeds=None), -1, "seeds"),
        (dict(fo=None), -1, "frame_offsets"),
        (dict(H=0), -1, "n_hyp"),
        (dict(tau=-1.0), -1, "tau"),
        (dict(out=None), -1, "output"),
        (dict(), -2, "workspace"),
    ]
    for kw, code, word in cases:
        assert call(**kw) == code, kw
        assert word in lib.rv_last_error().decode()
    bad = binding.RVTuning.from_dict({"rows_max": [17] * 8, "blocks_per_cu": 0})
    assert call(tuning=bad, ws=fake, ws_bytes=1 << 30) == -1
    assert "rows_max" in lib.rv_last_error().decode()
    bad = binding.RVTuning.from_dict({"rows_max": [16] * 8, "blocks_per_cu": 0, "fp16_min_points": -1})
    assert call(tuning=bad, ws=fake, ws_bytes=1 << 30) == -1
    assert "fp16_min_points" in lib.rv_last_error().decode()
    for lanes in (-1, 257):
        bad = binding.RVTuning.from_dict({"rows_max": [16] * 8, "lanes_max_points": lanes})
        assert call(tuning=bad, ws=fake, ws_bytes=1 << 30) == -1
        assert "lanes_max_points" in lib.rv_last_error().decode()
    # the default tuning: 16 rows everywhere, grid as large as fits, no FP16 form,
    # lanes = hypotheses up to 64 points
    d = binding.rv_tuning_default()
    assert list(d.rows_max) == [16] * 8 and d.blocks_per_cu == 0 and d.fp16_min_points == 0
    assert d.lanes_max_points == 64
    assert binding.RVTuning.from_dict(d.to_dict()).to_dict() == d.to_dict()
    assert ctypes.sizeof(binding.RVTuning) == 4 * (8 + 3)
    # nothing to do
    assert call(K=0, N=0, ws=fake, ws_bytes=1 << 20) == 0
    assert lib.rv_graph_launch(None, None) == -1
    lib.rv_graph_destroy(None)


def test_server_host_checks(lib):
    from paper_2012_12618_amd import binding

    cfg = binding.rv_server_config_default()
    assert (cfg.n_hyp, cfg.max_batch_frames, cfg.n_streams) == (512, 64, 2)
    assert cfg.hbm_budget_bytes == 16 << 30
    # arena bytes of one frame: 28 per point (inputs 8, staging 20) and 69 per cluster
    # (offsets 4, descriptor 32, best key 8, outputs 25), plus 256-byte sections and queues
    b = binding.rv_server_frame_bytes(cfg, 700, 146_000)
    assert 28 * 146_000 + 69 * 700 <= b <= 28 * 146_000 + 69 * 700 + 25 * 256 + 2560
    # with the inlier masks kept: one more bit per point
    cfg.keep_inlier_bits = 1
    bm = binding.rv_server_frame_bytes(cfg, 700, 146_000)
    assert b + 146_000 // 8 <= bm <= b + 146_000 // 8 + 256
    cfg.keep_inlier_bits = 0
    assert binding.rv_server_frame_bytes(cfg, -1, 5) == 0
    h = ctypes.c_void_p()
    for field, value, word in (("n_hyp", 0, "n_hyp"), ("tau", 0.0, "tau"),
                               ("hbm_budget_bytes", 1000, "budget"),
                               ("max_batch_frames", 0, "max_batch_frames"),
                               ("n_streams", 9, "n_streams"),
                               ("max_waiting_frames", 0, "max_waiting_frames"),
                               ("tuning.fp16_min_points", -5, "fp16_min_points"),
                               ("tuning.lanes_max_points", 300, "lanes_max_points")):
        c = binding.rv_server_config_default()
        if field.startswith("tuning."):
            setattr(c.tuning, field.split(".")[1], value)
        else:
            setattr(c, field, value)
        assert lib.rv_server_create(ctypes.byref(c), ctypes.byref(h)) == -1, field
        assert word in lib.rv_last_error().decode() and not h.value
    t = ctypes.c_uint64()
    assert lib.rv_server_submit(None, None, None, None, 0, 0, 1, ctypes.byref(t)) == -1
    assert lib.rv_server_submit_pinned(None, None, None, None, 0, 0, 1, ctypes.byref(t)) == -1
    assert lib.rv_server_wait(None, 1, 0) == -1
    assert lib.rv_server_result(None, 1, None, None, None, None, None, None, None, None,
                                None) == -1
    assert lib.rv_server_stats(None, None) == -1
    lib.rv_server_destroy(None)


def test_paper_variant_host_checks(lib):
    from paper_2012_12618_amd import binding

    assert binding.rv_paper_workspace_bytes(10, 1000, 64) >= 16 * 1000 + 16 * 10
    fake = ctypes.c_void_p(4096)

    def call(**kw):
        a = dict(theta=fake, vd=fake, off=fake, K=2, N=10, H=16, out=fake, ws=None, ws_bytes=0)
        a.update(kw)
        return lib.rv_estimate_velocity_paper(a["theta"], a["vd"], a["off"], a["K"], a["N"], a["H"],
                                              1, a["out"], a["out"], a["out"], a["out"], a["out"],
                                              None, None, None, None, a["ws"], a["ws_bytes"], None)

    for kw, code, word in ((dict(H=0), -1, "n_hyp"), (dict(off=None), -1, "cluster_offsets"),
                           (dict(theta=None), -1, "theta"), (dict(out=None), -1, "output"),
                           (dict(), -2, "workspace")):
        assert call(**kw) == code, kw
        assert word in lib.rv_last_error().decode()
    assert call(K=0, N=0, ws=fake, ws_bytes=1 << 20) == 0


def test_part_first_cluster_checks(lib):
    # The part entry point refuses a cluster or point base outside its range
    # before any HIP call (fake pointers: never used).
    fake = ctypes.c_void_p(4096)

    def part(first, K=4, first_point=0):
        return lib.rv_estimate_velocity_part(fake, fake, fake, K, 100, first, first_point, 16, 0.15,
                                             1, fake, fake, fake, fake, fake, None, None, None,
                                             None, fake, 1 << 20, None)

    assert part(-1) == -1 and "first_cluster" in lib.rv_last_error().decode()
    assert part(1 << 32) == -1 and "first_cluster" in lib.rv_last_error().decode()
    assert part((1 << 32) - 2) == -1 and "2^32" in lib.rv_last_error().decode()
    assert part(0, first_point=-1) == -1 and "first_point" in lib.rv_last_error().decode()
    assert part(0, first_point=1 << 31) == -1 and "first_point" in lib.rv_last_error().decode()


def test_pipelined_host_checks(lib):
    # The pipelined entry point reads the host offsets to cut the frame: bad
    # offsets, part counts and workspaces are refused before any HIP call.
    import numpy as np

    from paper_2012_12618_amd import binding

    fake = ctypes.c_void_p(4096)
    theta = np.zeros(100, np.float32)

    def call(off, n_parts=4, n_points=100, ws_bytes=1 << 30):
        off = np.ascontiguousarray(off, np.int32)
        return lib.rv_estimate_velocity_pipelined(
            ctypes.c_void_p(theta.ctypes.data), ctypes.c_void_p(theta.ctypes.data),
            ctypes.c_void_p(off.ctypes.data), len(off) - 1, n_points, n_parts, 16, 0.15, 1, fake,
            fake, fake, fake, fake, fake, fake, fake, None, None, None, fake, ws_bytes, None,
            None)

    good = [0, 10, 40, 100]
    assert call(good, n_parts=0) == -1 and "n_parts" in lib.rv_last_error().decode()
    assert call(good, n_parts=binding.RV_MAX_PARTS + 1) == -1
    assert call([1, 10, 40, 100]) == -1 and "start at 0" in lib.rv_last_error().decode()
    assert call([0, 10, 40, 99]) == -1 and "end at n_points" in lib.rv_last_error().decode()
    assert call([0, 50, 40, 100]) == -1 and "decrease at cluster 1" in lib.rv_last_error().decode()
    assert call(good, ws_bytes=64) == -2
    assert call([0], n_points=0) == 0  # no clusters: nothing to do, nothing enqueued


def test_pipelined_binding_checks(lib):
    # The binding refuses device or strided host inputs and wrong dtypes
    # before it touches the GPU.
    import torch

    from paper_2012_12618_amd import binding

    th = torch.zeros(64, dtype=torch.float32)
    off = torch.tensor([0, 64], dtype=torch.int32)
    with pytest.raises(ValueError, match="contiguous host tensor"):
        binding.rv_estimate_velocity_pipelined(th[::2], th[::2], off, 2, 16, 0.15, 1)
    with pytest.raises(TypeError, match="float32"):
        binding.rv_estimate_velocity_pipelined(th.double(), th, off, 2, 16, 0.15, 1)
    with pytest.raises(TypeError, match="int32"):
        binding.rv_estimate_velocity_pipelined(th, th, off.long(), 2, 16, 0.15, 1)


def test_package_exports():
    # Every name the package lists resolves to the binding's object without
    # loading the library; estimate_velocity is rv_estimate_velocity.
    import paper_2012_12618_amd as rv
    from paper_2012_12618_amd import binding

    for name in rv.__all__:
        assert getattr(rv, name) is getattr(binding, name), name
    assert rv.estimate_velocity is binding.rv_estimate_velocity
