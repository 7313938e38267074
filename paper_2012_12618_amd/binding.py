"""Thin ctypes binding of ``librv.so`` (include/rv.h): argument marshalling only.

PyTorch supplies device memory and the stream; every step of the estimate runs
in the library's HIP kernels.  The library must be built (``build.py``); if it
is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "librv.so")

RV_OK = 0
RV_ERR_INVALID_ARG = -1
RV_ERR_WORKSPACE = -2
RV_ERR_HIP = -3
RV_ERR_BUSY = -4

RV_CLUSTER_OK = 0
RV_CLUSTER_TOO_FEW_POINTS = 1
RV_CLUSTER_ALL_DEGENERATE = 2
RV_CLUSTER_SINGULAR_REFIT = 3
RV_CLUSTER_BAD_OFFSETS = 4
RV_CLUSTER_TOO_LARGE = 5
RV_PAPER_MAX_POINTS = 4096

RV_MIN_SEED_SEPARATION = 1e-3
RV_NEAR_TAU_WINDOW = 1e-5
RV_MAX_HYP = 1 << 20
RV_NOALLOC_SCRATCH_BYTES = 96 << 20
RV_MAX_PARTS = 64

RV_TUNE_BUCKETS = 8

N_STAGES = 3
STAGE_NAMES = ("prep", "score", "refit")

_lib = None


class RVTuning(ctypes.Structure):
    """rv_tuning_t: register rows per pass for each cluster-size bucket, the
    persistent grid's workgroups per compute unit (0: as many as fit), the
    smallest cluster scored in the FP16 residual form (0: none) and the largest
    cluster scored with lanes = hypotheses."""

    _fields_ = [("rows_max", ctypes.c_int32 * RV_TUNE_BUCKETS), ("blocks_per_cu", ctypes.c_int32),
                ("fp16_min_points", ctypes.c_int32), ("lanes_max_points", ctypes.c_int32)]

    def to_dict(self) -> dict:
        return {"rows_max": list(self.rows_max), "blocks_per_cu": int(self.blocks_per_cu),
                "fp16_min_points": int(self.fp16_min_points),
                "lanes_max_points": int(self.lanes_max_points)}

    @classmethod
    def from_dict(cls, d: dict) -> "RVTuning":
        t = rv_tuning_default()
        for i, r in enumerate(d["rows_max"]):
            t.rows_max[i] = int(r)
        t.blocks_per_cu = int(d.get("blocks_per_cu", 0))
        t.fp16_min_points = int(d.get("fp16_min_points", 0))
        t.lanes_max_points = int(d.get("lanes_max_points", t.lanes_max_points))
        return t


class RVServerConfig(ctypes.Structure):
    """rv_server_config_t."""

    _fields_ = [("n_hyp", ctypes.c_int32), ("tau", ctypes.c_float),
                ("hbm_budget_bytes", ctypes.c_size_t), ("max_batch_frames", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("max_waiting_frames", ctypes.c_int32),
                ("keep_inlier_bits", ctypes.c_int32), ("tuning", RVTuning)]


class RVFrameTimes(ctypes.Structure):
    """rv_frame_times_t: host-clock ns since the server's creation."""

    _fields_ = [("submitted_ns", ctypes.c_int64), ("launched_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("batch_frames", ctypes.c_int32),
                ("slot", ctypes.c_int32)]


class RVServerStats(ctypes.Structure):
    """rv_server_stats_t."""

    _fields_ = [(n, ctypes.c_int64) for n in (
        "frames_submitted", "frames_done", "batches", "busy_rejections", "max_batch_frames_seen",
        "arena_bytes", "arena_peak_bytes", "pinned_bytes", "waiting_frames", "inflight_batches")]

    def to_dict(self) -> dict:
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class RVError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"rv error {code}: {message}")
        self.code = code


def load_library() -> ctypes.CDLL:
    """Load librv.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"HIP library not built: {LIB_PATH} is missing "
            "(run `python -m paper_2012_12618_amd.build` or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    lib.rv_workspace_bytes.restype = ctypes.c_size_t
    lib.rv_workspace_bytes.argtypes = [i64, i64, i32]
    lib.rv_estimate_velocity.restype = ctypes.c_int
    lib.rv_estimate_velocity.argtypes = [
        P, P, P, i64, i64, i32, ctypes.c_float, ctypes.c_uint64,
        P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P,
    ]
    lib.rv_estimate_velocity_part.restype = ctypes.c_int
    lib.rv_estimate_velocity_part.argtypes = [
        P, P, P, i64, i64, i64, i64, i32, ctypes.c_float, ctypes.c_uint64,
        P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P,
    ]
    lib.rv_estimate_velocity_pipelined.restype = ctypes.c_int
    lib.rv_estimate_velocity_pipelined.argtypes = [
        P, P, P, i64, i64, i32, i32, ctypes.c_float, ctypes.c_uint64, P, P, P,
        P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P, P,
    ]
    lib.rv_estimate_velocity_noalloc.restype = ctypes.c_int
    lib.rv_estimate_velocity_noalloc.argtypes = [
        P, P, P, i64, i64, i32, ctypes.c_float, ctypes.c_uint64,
        P, P, P, P, P, P, P, P, P, P,
    ]
    lib.rv_host_device_pointer.restype = ctypes.c_int
    lib.rv_host_device_pointer.argtypes = [P, P]
    lib.rv_last_error.restype = ctypes.c_char_p
    lib.rv_last_error.argtypes = []
    lib.rv_stage_timing.restype = ctypes.c_int
    lib.rv_stage_timing.argtypes = [ctypes.c_int]
    lib.rv_stage_times.restype = ctypes.c_int
    lib.rv_stage_times.argtypes = [P, P]
    lib.rv_philox4x32_10.restype = ctypes.c_int
    lib.rv_philox4x32_10.argtypes = [P, P, P, i64, P]
    lib.rv_tuning_default.restype = None
    lib.rv_tuning_default.argtypes = [P]
    lib.rv_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.rv_batch_workspace_bytes.argtypes = [i64, i64, i64, i32]
    batch_args = [P, P, P, P, P, i64, i64, i64, i32, ctypes.c_float,
                  P, P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t]
    lib.rv_estimate_velocity_batch.restype = ctypes.c_int
    lib.rv_estimate_velocity_batch.argtypes = batch_args + [P]
    lib.rv_graph_capture_batch.restype = ctypes.c_int
    lib.rv_graph_capture_batch.argtypes = batch_args + [P]
    lib.rv_graph_launch.restype = ctypes.c_int
    lib.rv_graph_launch.argtypes = [P, P]
    lib.rv_graph_destroy.restype = None
    lib.rv_graph_destroy.argtypes = [P]
    lib.rv_paper_workspace_bytes.restype = ctypes.c_size_t
    lib.rv_paper_workspace_bytes.argtypes = [i64, i64, i32]
    lib.rv_estimate_velocity_paper.restype = ctypes.c_int
    lib.rv_estimate_velocity_paper.argtypes = [P, P, P, i64, i64, i32, ctypes.c_uint64,
                                               P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P]
    lib.rv_server_config_default.restype = None
    lib.rv_server_config_default.argtypes = [P]
    lib.rv_server_frame_bytes.restype = ctypes.c_size_t
    lib.rv_server_frame_bytes.argtypes = [P, i64, i64]
    lib.rv_server_create.restype = ctypes.c_int
    lib.rv_server_create.argtypes = [P, P]
    lib.rv_server_submit.restype = ctypes.c_int
    lib.rv_server_submit.argtypes = [P, P, P, P, i64, i64, ctypes.c_uint64, P]
    lib.rv_server_submit_pinned.restype = ctypes.c_int
    lib.rv_server_submit_pinned.argtypes = [P, P, P, P, i64, i64, ctypes.c_uint64, P]
    lib.rv_server_wait.restype = ctypes.c_int
    lib.rv_server_wait.argtypes = [P, ctypes.c_uint64, i64]
    lib.rv_server_result.restype = ctypes.c_int
    lib.rv_server_result.argtypes = [P, ctypes.c_uint64, P, P, P, P, P, P, P, P, P]
    lib.rv_server_stats.restype = ctypes.c_int
    lib.rv_server_stats.argtypes = [P, P]
    lib.rv_server_destroy.restype = None
    lib.rv_server_destroy.argtypes = [P]
    _lib = lib
    return lib


def rv_last_error() -> str:
    return load_library().rv_last_error().decode()


def _check(code: int) -> None:
    if code != RV_OK:
        raise RVError(code, rv_last_error())


def rv_workspace_bytes(n_clusters: int, n_points: int, n_hyp: int) -> int:
    return int(load_library().rv_workspace_bytes(int(n_clusters), int(n_points), int(n_hyp)))


def host_device_pointer(t: torch.Tensor) -> int:
    """The address under which the current GPU sees a pinned host tensor's
    memory (rv_host_device_pointer); raises for pageable memory."""
    out = ctypes.c_void_p()
    _check(load_library().rv_host_device_pointer(ctypes.c_void_p(t.data_ptr()), ctypes.byref(out)))
    return int(out.value)


def _dev_ptr(t: torch.Tensor | None, dtype: torch.dtype, device: torch.device, name: str,
             numel: int | None = None, host_ok: bool = False):
    """Device pointer of a checked tensor; ``numel``: the elements the kernels
    write or read through it (a smaller tensor raises before anything runs).
    ``host_ok``: a pinned host tensor is accepted too, and the kernels then read
    or write it directly through its device mapping."""
    if t is None:
        return None
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if host_ok and t.device.type == "cpu":
        if not t.is_pinned():
            raise ValueError(f"{name}: host tensors must be pinned (pin_memory())")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if numel is not None and t.numel() < numel:
            raise ValueError(f"{name} holds {t.numel()} elements, {numel} needed")
        return ctypes.c_void_p(host_device_pointer(t)) if t.numel() > 0 else None
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, {numel} needed")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else None


def _output_ptrs(out: dict, device, n_clusters: int, n_points: int, n_hyp: int,
                 host_ok: bool = False) -> tuple:
    """The output pointers of the estimate entry points, in their C order
    (vx, vy, heading, n_inliers, status, n_near_tau, inlier_bits, hyp_counts,
    best_hyp), each checked for dtype, device, layout and size."""
    K = n_clusters
    h = host_ok
    return (
        _dev_ptr(out["vx"], torch.float32, device, "vx", K, h),
        _dev_ptr(out["vy"], torch.float32, device, "vy", K, h),
        _dev_ptr(out["heading"], torch.float32, device, "heading", K, h),
        _dev_ptr(out["n_inliers"], torch.int32, device, "n_inliers", K, h),
        _dev_ptr(out["status"], torch.uint8, device, "status", K, h),
        _dev_ptr(out.get("n_near_tau"), torch.int32, device, "n_near_tau", K, h),
        _dev_ptr(out.get("inlier_bits"), torch.int32, device, "inlier_bits", (n_points + 31) // 32, h),
        _dev_ptr(out.get("hyp_counts"), torch.int32, device, "hyp_counts", K * int(n_hyp), h),
        _dev_ptr(out.get("best_hyp"), torch.int32, device, "best_hyp", K, h),
    )


def _call_device(theta: torch.Tensor) -> torch.device:
    """The GPU a call runs on: theta's, or the current one for a pinned host theta."""
    if theta.device.type == "cuda":
        return theta.device
    if theta.is_pinned():
        return torch.device("cuda", torch.cuda.current_device())
    raise ValueError("theta must be a GPU tensor or a pinned host tensor")


def allocate_outputs(n_clusters: int, n_points: int, n_hyp: int, device, *,
                     want_near: bool = True, want_bits: bool = False, debug: bool = False) -> dict:
    """Output tensors for rv_estimate_velocity (plus the workspace)."""
    dev = torch.device(device)
    out = {
        "vx": torch.empty(n_clusters, dtype=torch.float32, device=dev),
        "vy": torch.empty(n_clusters, dtype=torch.float32, device=dev),
        "heading": torch.empty(n_clusters, dtype=torch.float32, device=dev),
        "n_inliers": torch.empty(n_clusters, dtype=torch.int32, device=dev),
        "status": torch.empty(n_clusters, dtype=torch.uint8, device=dev),
        "workspace": torch.empty(max(rv_workspace_bytes(n_clusters, n_points, n_hyp), 1),
                                 dtype=torch.uint8, device=dev),
    }
    if want_near:
        out["n_near_tau"] = torch.empty(n_clusters, dtype=torch.int32, device=dev)
    if want_bits:
        out["inlier_bits"] = torch.empty((n_points + 31) // 32, dtype=torch.int32, device=dev)
    if debug:
        out["hyp_counts"] = torch.empty(n_clusters * n_hyp, dtype=torch.int32, device=dev)
        out["best_hyp"] = torch.empty(n_clusters, dtype=torch.int32, device=dev)
    return out


def _used_on(stream, tensors) -> None:
    """Tell torch's caching allocator that ``stream`` uses these tensors, so that
    their memory is not handed out again (for instance after the workspace is
    dropped on return) before the work enqueued on ``stream`` has finished."""
    for t in tensors:
        if isinstance(t, torch.Tensor) and t.is_cuda:
            t.record_stream(stream)


def rv_estimate_velocity(theta: torch.Tensor, vd: torch.Tensor, offsets: torch.Tensor,
                         n_hyp: int, tau: float, seed: int, *, want_near: bool = True,
                         want_bits: bool = False, debug: bool = False, out: dict | None = None,
                         stream: torch.cuda.Stream | None = None, validate: bool = False) -> dict:
    """Per-cluster (vx, vy, heading, n_inliers, status) of one CSR frame.

    ``theta``/``vd``: float32 [N] on a GPU; ``offsets``: int32 [K+1] on the same
    device.  Inputs and the tensors of ``out`` may instead be pinned host
    tensors (the kernels then read and write them directly, no copies; the
    call runs on the current GPU and the workspace stays there; the caller
    keeps such tensors alive until the stream has finished with them).  Outputs (and
    the workspace) are allocated with torch unless ``out`` (from
    ``allocate_outputs``) is given.  Work is enqueued on ``stream`` (default:
    torch's current stream); the returned tensors are ready after that stream
    synchronises.  ``validate`` checks the offsets on the host first (a device
    to host copy; off by default).  Returned dict keys: vx, vy, heading,
    n_inliers, status and, when requested, n_near_tau, inlier_bits (int32 words,
    bit p%32 of word p/32 is point p), hyp_counts [K*H], best_hyp.
    """
    return _estimate(theta, vd, offsets, None, n_hyp, tau, seed, want_near, want_bits, debug,
                     out, stream, validate)


# The estimate under its short name, estimate_velocity(theta, vd, offsets, n_hyp,
# tau, seed, *, debug=False, ...): the same function.
estimate_velocity = rv_estimate_velocity


def rv_estimate_velocity_part(theta: torch.Tensor, vd: torch.Tensor, offsets: torch.Tensor,
                              first_cluster: int, first_point: int, n_hyp: int, tau: float,
                              seed: int, *, want_near: bool = True, want_bits: bool = False,
                              debug: bool = False, out: dict | None = None,
                              stream: torch.cuda.Stream | None = None) -> dict:
    """rv_estimate_velocity for a part of a larger frame: its clusters are the
    frame's clusters ``first_cluster ..``, and each draws its hypotheses with its
    index in the whole frame, so the outputs are bit for bit the whole frame's.
    ``theta`` and ``vd`` are the part's points (the frame's from ``first_point``
    on); ``offsets`` are the frame's offsets of the part's clusters (frame point
    indexes).  Other arguments and the results are those of
    rv_estimate_velocity, indexed by the part's clusters and points."""
    return _estimate(theta, vd, offsets, (int(first_cluster), int(first_point)), n_hyp, tau, seed,
                     want_near, want_bits, debug, out, stream, False)


def _estimate(theta, vd, offsets, part, n_hyp, tau, seed, want_near, want_bits, debug,
              out, stream, validate) -> dict:
    """The whole-frame entry point when ``part`` is None, else the part one
    with part = (first_cluster, first_point)."""
    lib = load_library()
    device = _call_device(theta)
    n_points = int(theta.numel())
    n_clusters = int(offsets.numel()) - 1
    if n_clusters < 0:
        raise ValueError("offsets needs n_clusters + 1 entries")
    if int(vd.numel()) != n_points:
        raise ValueError("theta and vd differ in length")
    if validate:
        off = offsets.cpu()
        if off[0] != 0 or off[-1] != n_points or bool((off[1:] < off[:-1]).any()):
            raise ValueError("offsets must start at 0, be non-decreasing and end at n_points")
    owned = out is None
    if out is None:
        out = allocate_outputs(n_clusters, n_points, n_hyp, device, want_near=want_near,
                               want_bits=want_bits, debug=debug)
    ws = out["workspace"]
    if stream is None:
        stream = torch.cuda.current_stream(device)
    inputs = (
        _dev_ptr(theta, torch.float32, device, "theta", host_ok=True),
        _dev_ptr(vd, torch.float32, device, "vd", host_ok=True),
        _dev_ptr(offsets, torch.int32, device, "offsets", host_ok=True),
        n_clusters, n_points)
    rest = (
        int(n_hyp), float(tau), int(seed) & 0xFFFFFFFFFFFFFFFF,
        *_output_ptrs(out, device, n_clusters, n_points, n_hyp, host_ok=True),
        _dev_ptr(ws, torch.uint8, device, "workspace"), int(ws.numel()),
        ctypes.c_void_p(stream.cuda_stream))
    if part is None:
        code = lib.rv_estimate_velocity(*inputs, *rest)
    else:
        code = lib.rv_estimate_velocity_part(*inputs, *part, *rest)
    _check(code)
    if owned:
        _used_on(stream, out.values())
    return {k: v for k, v in out.items() if k != "workspace"}


def rv_estimate_velocity_pipelined(theta: torch.Tensor, vd: torch.Tensor, offsets: torch.Tensor,
                                   n_parts: int, n_hyp: int, tau: float, seed: int, *,
                                   device_inputs: tuple | None = None, want_near: bool = True,
                                   debug: bool = False, out: dict | None = None,
                                   stream: torch.cuda.Stream | None = None,
                                   copy_stream: torch.cuda.Stream | None = None) -> dict:
    """One frame from host memory, copied and estimated in ``n_parts`` parts
    that shrink toward the end (rv_estimate_velocity_pipelined): each part's
    estimate on ``stream``
    overlaps the next part's copy on ``copy_stream`` (default: a new stream).
    ``theta``/``vd``/``offsets``: contiguous CPU tensors, pinned for the copies
    to overlap; ``device_inputs``: (theta, vd, offsets) device tensors of at
    least the frame's sizes that receive the copies (allocated if None).  The
    results (no inlier mask) are those of rv_estimate_velocity on the whole
    frame; ``out`` may hold device or pinned host tensors.  The caller keeps
    the host tensors alive and unchanged until ``stream`` has finished: the
    library's copies read them then, and torch's pinned-memory cache does not
    know of those copies, so it could hand freed memory out again too early."""
    lib = load_library()
    for name, t in (("theta", theta), ("vd", vd), ("offsets", offsets)):
        if t.device.type != "cpu" or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous host tensor")
    if theta.dtype != torch.float32 or vd.dtype != torch.float32 or offsets.dtype != torch.int32:
        raise TypeError("theta and vd must be float32, offsets int32")
    device = torch.device("cuda", torch.cuda.current_device())
    n_points = int(theta.numel())
    n_clusters = int(offsets.numel()) - 1
    if n_clusters < 0 or int(vd.numel()) != n_points:
        raise ValueError("offsets needs n_clusters + 1 entries; theta and vd must match")
    if device_inputs is None:
        device_inputs = (torch.empty(n_points, dtype=torch.float32, device=device),
                         torch.empty(n_points, dtype=torch.float32, device=device),
                         torch.empty(n_clusters + 1, dtype=torch.int32, device=device))
    d_t, d_v, d_o = device_inputs
    owned = out is None
    if out is None:
        out = allocate_outputs(n_clusters, n_points, n_hyp, device, want_near=want_near,
                               want_bits=False, debug=debug)
    if out.get("inlier_bits") is not None:
        raise ValueError("the pipelined form gives no inlier mask")
    if stream is None:
        stream = torch.cuda.current_stream(device)
    if copy_stream is None:
        copy_stream = torch.cuda.Stream(device=device)
    ws = out["workspace"]
    ptrs = _output_ptrs(out, device, n_clusters, n_points, n_hyp, host_ok=True)
    code = lib.rv_estimate_velocity_pipelined(
        ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(vd.data_ptr()),
        ctypes.c_void_p(offsets.data_ptr()), n_clusters, n_points, int(n_parts), int(n_hyp),
        float(tau), int(seed) & 0xFFFFFFFFFFFFFFFF,
        _dev_ptr(d_t, torch.float32, device, "theta (device)", n_points),
        _dev_ptr(d_v, torch.float32, device, "vd (device)", n_points),
        _dev_ptr(d_o, torch.int32, device, "offsets (device)", n_clusters + 1),
        *ptrs[:6], *ptrs[7:],
        _dev_ptr(ws, torch.uint8, device, "workspace"), int(ws.numel()),
        ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(copy_stream.cuda_stream))
    _check(code)
    if owned:
        _used_on(stream, out.values())
    _used_on(stream, device_inputs)
    _used_on(copy_stream, device_inputs)
    return {k: v for k, v in out.items() if k != "workspace"}


def rv_estimate_velocity_noalloc(theta: torch.Tensor, vd: torch.Tensor, offsets: torch.Tensor,
                                 n_hyp: int, tau: float, seed: int, out: dict,
                                 stream: torch.cuda.Stream | None = None) -> dict:
    """rv_estimate_velocity on the library's own device scratch: no workspace,
    and the caller's ``out`` (tensors as ``allocate_outputs`` makes them; a
    ``workspace`` entry is ignored) receives the results.  Frames needing more
    than RV_NOALLOC_SCRATCH_BYTES of workspace raise RVError; calls that share a
    GPU must not overlap (they share its scratch)."""
    lib = load_library()
    device = theta.device
    if device.type != "cuda":
        raise ValueError("theta must be a GPU tensor")
    n_points = int(theta.numel())
    n_clusters = int(offsets.numel()) - 1
    if n_clusters < 0:
        raise ValueError("offsets needs n_clusters + 1 entries")
    if int(vd.numel()) != n_points:
        raise ValueError("theta and vd differ in length")
    if stream is None:
        stream = torch.cuda.current_stream(device)
    _check(lib.rv_estimate_velocity_noalloc(
        _dev_ptr(theta, torch.float32, device, "theta"),
        _dev_ptr(vd, torch.float32, device, "vd"),
        _dev_ptr(offsets, torch.int32, device, "offsets"),
        n_clusters, n_points, int(n_hyp), float(tau), int(seed) & 0xFFFFFFFFFFFFFFFF,
        *_output_ptrs(out, device, n_clusters, n_points, n_hyp),
        ctypes.c_void_p(stream.cuda_stream)))
    return {k: v for k, v in out.items() if k != "workspace"}


class PreparedEstimate:
    """rv_estimate_velocity with its tensors checked and their device pointers
    taken once: each call passes only the seed, for callers that estimate frame
    after frame in the same buffers (the tensors' contents may change between
    calls, not their storage).  The tensors may be pinned host tensors, as for
    rv_estimate_velocity.  A call may also estimate a smaller frame held at the
    start of the same buffers (n_points, n_clusters up to the prepared sizes).
    Holds references to every tensor it uses."""

    def __init__(self, theta: torch.Tensor, vd: torch.Tensor, offsets: torch.Tensor, n_hyp: int,
                 tau: float, out: dict, stream: torch.cuda.Stream | None = None):
        self._lib = load_library()
        device = _call_device(theta)
        n_points = int(theta.numel())
        n_clusters = int(offsets.numel()) - 1
        if n_clusters < 0 or int(vd.numel()) != n_points:
            raise ValueError("offsets needs n_clusters + 1 entries; theta and vd must match")
        if stream is None:
            stream = torch.cuda.current_stream(device)
        ws = out["workspace"]
        self._keep = (theta, vd, offsets, dict(out), stream)
        self._ptrs = (
            _dev_ptr(theta, torch.float32, device, "theta", host_ok=True),
            _dev_ptr(vd, torch.float32, device, "vd", host_ok=True),
            _dev_ptr(offsets, torch.int32, device, "offsets", host_ok=True))
        self._sizes = (n_clusters, n_points)
        self._scalars = (int(n_hyp), float(tau))
        self._tail = (
            *_output_ptrs(out, device, n_clusters, n_points, n_hyp, host_ok=True),
            _dev_ptr(ws, torch.uint8, device, "workspace"), int(ws.numel()),
            ctypes.c_void_p(stream.cuda_stream))
        self.out = {k: v for k, v in out.items() if k != "workspace"}

    def __call__(self, seed: int, n_points: int | None = None,
                 n_clusters: int | None = None) -> dict:
        k, n = self._sizes
        if n_clusters is not None or n_points is not None:
            k1 = k if n_clusters is None else int(n_clusters)
            n1 = n if n_points is None else int(n_points)
            if not (0 <= k1 <= k and 0 <= n1 <= n):
                raise ValueError(f"a frame of {k1} clusters and {n1} points does not fit the "
                                 f"prepared {k} and {n}")
            k, n = k1, n1
        _check(self._lib.rv_estimate_velocity(*self._ptrs, k, n, *self._scalars,
                                              int(seed) & 0xFFFFFFFFFFFFFFFF, *self._tail))
        return self.out


def rv_stage_timing(enable: bool) -> None:
    _check(load_library().rv_stage_timing(1 if enable else 0))


def rv_stage_times() -> tuple[list[float], int]:
    """(summed ms per kernel [prep, score, refit], number of timed calls)."""
    ms = (ctypes.c_double * N_STAGES)()
    n = ctypes.c_int64()
    _check(load_library().rv_stage_times(ms, ctypes.byref(n)))
    return list(ms), int(n.value)


def rv_philox4x32_10(ctr: torch.Tensor, key: torch.Tensor,
                     stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """GPU Philox4x32-10 blocks: ctr int32/uint32 [n, 4], key [n, 2] -> [n, 4] (int32 bits)."""
    lib = load_library()
    device = ctr.device
    n = int(ctr.shape[0])
    ctr = ctr.contiguous()
    key = key.contiguous()
    out = torch.empty((n, 4), dtype=torch.int32, device=device)
    if stream is None:
        stream = torch.cuda.current_stream(device)
    _check(lib.rv_philox4x32_10(ctypes.c_void_p(ctr.data_ptr()), ctypes.c_void_p(key.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), n,
                                ctypes.c_void_p(stream.cuda_stream)))
    return out


# ---- many frames ------------------------------------------------------------

def rv_tuning_default() -> RVTuning:
    t = RVTuning()
    load_library().rv_tuning_default(ctypes.byref(t))
    return t


def rv_batch_workspace_bytes(n_frames: int, n_clusters: int, n_points: int, n_hyp: int) -> int:
    return int(load_library().rv_batch_workspace_bytes(int(n_frames), int(n_clusters),
                                                       int(n_points), int(n_hyp)))


def allocate_batch_outputs(n_frames: int, n_clusters: int, n_points: int, n_hyp: int, device, *,
                           want_near: bool = True, want_bits: bool = False,
                           debug: bool = False) -> dict:
    """Outputs and workspace for rv_estimate_velocity_batch / rv_graph_capture_batch."""
    out = allocate_outputs(n_clusters, n_points, n_hyp, device, want_near=want_near,
                           want_bits=want_bits, debug=debug)
    out["workspace"] = torch.empty(
        max(rv_batch_workspace_bytes(n_frames, n_clusters, n_points, n_hyp), 1),
        dtype=torch.uint8, device=torch.device(device))
    return out


def _batch_args(theta, vd, offsets, frame_offsets, seeds, n_hyp, tau, out, tuning):
    device = theta.device
    if device.type != "cuda":
        raise ValueError("theta must be a GPU tensor")
    n_points = int(theta.numel())
    n_clusters = int(offsets.numel()) - 1
    n_frames = int(frame_offsets.numel()) - 1
    if n_clusters < 0 or n_frames < 1:
        raise ValueError("offsets needs n_clusters + 1 entries, frame_offsets n_frames + 1 >= 2")
    if int(vd.numel()) != n_points:
        raise ValueError("theta and vd differ in length")
    if int(seeds.numel()) != n_frames:
        raise ValueError("seeds needs one entry per frame")
    ws = out["workspace"]
    tune = tuning if tuning is not None else rv_tuning_default()
    args = [
        _dev_ptr(theta, torch.float32, device, "theta"),
        _dev_ptr(vd, torch.float32, device, "vd"),
        _dev_ptr(offsets, torch.int32, device, "offsets"),
        _dev_ptr(frame_offsets, torch.int32, device, "frame_offsets"),
        _dev_ptr(seeds, torch.int64, device, "seeds"),
        n_frames, n_clusters, n_points, int(n_hyp), float(tau),
        *_output_ptrs(out, device, n_clusters, n_points, n_hyp),
        ctypes.byref(tune),
        ctypes.c_void_p(ws.data_ptr()), int(ws.numel()),
    ]
    return args, tune


def rv_estimate_velocity_batch(theta, vd, offsets, frame_offsets, seeds, n_hyp: int, tau: float, *,
                               tuning: RVTuning | None = None, want_near: bool = True,
                               want_bits: bool = False, debug: bool = False,
                               out: dict | None = None, stream=None) -> dict:
    """Per-cluster outputs of n_frames frames in one launch sequence.

    ``frame_offsets``: int32 [n_frames + 1] cluster ranges of the frames;
    ``seeds``: int64 [n_frames] (bit patterns of the uint64 seeds), on the GPU.
    Every cluster's outputs equal rv_estimate_velocity on its frame alone.
    """
    lib = load_library()
    n_points = int(theta.numel())
    n_clusters = int(offsets.numel()) - 1
    n_frames = int(frame_offsets.numel()) - 1
    owned = out is None
    if out is None:
        out = allocate_batch_outputs(n_frames, n_clusters, n_points, n_hyp, theta.device,
                                     want_near=want_near, want_bits=want_bits, debug=debug)
    args, _tune = _batch_args(theta, vd, offsets, frame_offsets, seeds, n_hyp, tau, out, tuning)
    if stream is None:
        stream = torch.cuda.current_stream(theta.device)
    _check(lib.rv_estimate_velocity_batch(*args, ctypes.c_void_p(stream.cuda_stream)))
    if owned:
        _used_on(stream, out.values())
    return {k: v for k, v in out.items() if k != "workspace"}


class RVGraph:
    """A captured rv_estimate_velocity_batch launch sequence (HIP graph).

    Keeps references to every tensor it was captured with: their contents may
    change between launches, their storage may not.
    """

    def __init__(self, handle, tensors):
        self._handle = handle
        self._tensors = tensors

    def launch(self, stream=None) -> None:
        if self._handle is None:
            raise RuntimeError("graph destroyed")
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(load_library().rv_graph_launch(self._handle, ctypes.c_void_p(stream.cuda_stream)))

    def destroy(self) -> None:
        if self._handle is not None:
            load_library().rv_graph_destroy(self._handle)
            self._handle = None
            self._tensors = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def rv_graph_capture_batch(theta, vd, offsets, frame_offsets, seeds, n_hyp: int, tau: float,
                           out: dict, *, tuning: RVTuning | None = None) -> RVGraph:
    """Capture one batched estimate into a HIP graph (nothing runs until launch)."""
    lib = load_library()
    args, tune = _batch_args(theta, vd, offsets, frame_offsets, seeds, n_hyp, tau, out, tuning)
    handle = ctypes.c_void_p()
    _check(lib.rv_graph_capture_batch(*args, ctypes.byref(handle)))
    return RVGraph(handle, (theta, vd, offsets, frame_offsets, seeds, out, tune))


# ---- paper-literal variant ----------------------------------------------------

def rv_paper_workspace_bytes(n_clusters: int, n_points: int, n_hyp: int) -> int:
    return int(load_library().rv_paper_workspace_bytes(int(n_clusters), int(n_points), int(n_hyp)))


def allocate_paper_outputs(n_clusters: int, n_points: int, n_hyp: int, device, *,
                           want_bits: bool = False, debug: bool = False) -> dict:
    """Output tensors for rv_estimate_velocity_paper (plus its workspace)."""
    out = allocate_outputs(n_clusters, n_points, n_hyp, device, want_near=False,
                           want_bits=want_bits, debug=debug)
    dev = torch.device(device)
    out["thresh"] = torch.empty(n_clusters, dtype=torch.float64, device=dev)
    out["workspace"] = torch.empty(max(rv_paper_workspace_bytes(n_clusters, n_points, n_hyp), 1),
                                   dtype=torch.uint8, device=dev)
    return out


def rv_estimate_velocity_paper(theta: torch.Tensor, vd: torch.Tensor, offsets: torch.Tensor,
                               n_hyp: int, seed: int, *, want_bits: bool = False,
                               debug: bool = False, out: dict | None = None,
                               stream=None) -> dict:
    """Paper-literal inlier kernel (normalised line fit, MAD threshold, <= test)
    and the least-squares refit; outputs as rv_estimate_velocity plus ``thresh``
    (float64 per cluster).  Outputs and workspace are allocated with torch
    unless ``out`` (from ``allocate_paper_outputs``) is given; the frame-wide
    mask and the debug outputs are written when ``out`` holds them."""
    lib = load_library()
    device = theta.device
    if device.type != "cuda":
        raise ValueError("theta must be a GPU tensor")
    n_points, n_clusters = int(theta.numel()), int(offsets.numel()) - 1
    if n_clusters < 0 or int(vd.numel()) != n_points:
        raise ValueError("offsets needs n_clusters + 1 entries; theta and vd must match")
    owned = out is None
    if owned:
        out = allocate_paper_outputs(n_clusters, n_points, n_hyp, device, want_bits=want_bits,
                                     debug=debug)
    out = dict(out)
    ws = out.pop("workspace")
    if stream is None:
        stream = torch.cuda.current_stream(device)
    _check(lib.rv_estimate_velocity_paper(
        _dev_ptr(theta, torch.float32, device, "theta"), _dev_ptr(vd, torch.float32, device, "vd"),
        _dev_ptr(offsets, torch.int32, device, "offsets"), n_clusters, n_points, int(n_hyp),
        int(seed) & 0xFFFFFFFFFFFFFFFF,
        _dev_ptr(out["vx"], torch.float32, device, "vx", n_clusters),
        _dev_ptr(out["vy"], torch.float32, device, "vy", n_clusters),
        _dev_ptr(out["heading"], torch.float32, device, "heading", n_clusters),
        _dev_ptr(out["n_inliers"], torch.int32, device, "n_inliers", n_clusters),
        _dev_ptr(out["status"], torch.uint8, device, "status", n_clusters),
        _dev_ptr(out["thresh"], torch.float64, device, "thresh", n_clusters),
        _dev_ptr(out.get("inlier_bits"), torch.int32, device, "inlier_bits", (n_points + 31) // 32),
        _dev_ptr(out.get("hyp_counts"), torch.int32, device, "hyp_counts", n_clusters * int(n_hyp)),
        _dev_ptr(out.get("best_hyp"), torch.int32, device, "best_hyp", n_clusters),
        ctypes.c_void_p(ws.data_ptr()), int(ws.numel()), ctypes.c_void_p(stream.cuda_stream)))
    if owned:
        _used_on(stream, list(out.values()) + [ws])
    return out


# ---- frame server -----------------------------------------------------------

def rv_server_config_default() -> RVServerConfig:
    c = RVServerConfig()
    load_library().rv_server_config_default(ctypes.byref(c))
    return c


def rv_server_frame_bytes(cfg: RVServerConfig, n_clusters: int, n_points: int) -> int:
    return int(load_library().rv_server_frame_bytes(ctypes.byref(cfg), int(n_clusters), int(n_points)))


class RVServer:
    """rv_server_t: frames in host memory in, per-cluster results in host memory out.

    Submit copies the frame before returning (``submit_pinned`` queues a frame
    held in pinned host tensors without copying it); ``result`` returns numpy
    arrays.  The arena and the threads live until ``destroy`` (or garbage
    collection).
    """

    def __init__(self, cfg: RVServerConfig | None = None, **overrides):
        lib = load_library()
        self.cfg = cfg if cfg is not None else rv_server_config_default()
        for k, v in overrides.items():
            if k == "tuning":
                self.cfg.tuning = v
            else:
                setattr(self.cfg, k, v)
        handle = ctypes.c_void_p()
        _check(lib.rv_server_create(ctypes.byref(self.cfg), ctypes.byref(handle)))
        self._h = handle
        self._sizes: dict[int, tuple[int, int]] = {}
        self._pinned: dict[int, tuple] = {}  # tensors a queued frame is read from

    def submit(self, theta: np.ndarray, vd: np.ndarray, offsets: np.ndarray, seed: int) -> int:
        """Queue one frame; returns its ticket.  Raises RVError (code RV_ERR_BUSY when full)."""
        theta = np.ascontiguousarray(theta, np.float32)
        vd = np.ascontiguousarray(vd, np.float32)
        offsets = np.ascontiguousarray(offsets, np.int32)
        n_points, n_clusters = int(theta.shape[0]), int(offsets.shape[0]) - 1
        if vd.shape[0] != n_points or n_clusters < 0:
            raise ValueError("theta and vd must have the same length; offsets needs >= 1 entry")
        t = ctypes.c_uint64()
        _check(load_library().rv_server_submit(
            self._h, theta.ctypes.data_as(ctypes.c_void_p), vd.ctypes.data_as(ctypes.c_void_p),
            offsets.ctypes.data_as(ctypes.c_void_p), n_clusters, n_points,
            int(seed) & 0xFFFFFFFFFFFFFFFF, ctypes.byref(t)))
        self._sizes[int(t.value)] = (n_clusters, n_points)
        return int(t.value)

    def submit_pinned(self, theta: torch.Tensor, vd: torch.Tensor, offsets: torch.Tensor,
                      seed: int) -> int:
        """Queue one frame held in host tensors (float32 theta and vd, int32
        offsets), read in place by the server: no copy.  Pinned tensors
        (pin_memory()) keep the server's copies asynchronous; they are not
        checked here, since the pointer query costs more than the copy saves.
        The tensors are referenced until ``result`` takes the ticket; the
        caller leaves their contents unchanged until then."""
        for name, t, dt in (("theta", theta, torch.float32), ("vd", vd, torch.float32),
                            ("offsets", offsets, torch.int32)):
            if t.device.type != "cpu" or not t.is_contiguous() or t.dtype != dt:
                raise ValueError(f"{name} must be a contiguous {dt} host tensor")
        n_points, n_clusters = int(theta.numel()), int(offsets.numel()) - 1
        if int(vd.numel()) != n_points or n_clusters < 0:
            raise ValueError("theta and vd must have the same length; offsets needs >= 1 entry")
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else None  # noqa: E731
        t = ctypes.c_uint64()
        _check(load_library().rv_server_submit_pinned(
            self._h, ptr(theta), ptr(vd), ptr(offsets), n_clusters, n_points,
            int(seed) & 0xFFFFFFFFFFFFFFFF, ctypes.byref(t)))
        self._sizes[int(t.value)] = (n_clusters, n_points)
        self._pinned[int(t.value)] = (theta, vd, offsets)
        return int(t.value)

    def wait(self, ticket: int, timeout_ms: int = -1) -> bool:
        rc = load_library().rv_server_wait(self._h, int(ticket), int(timeout_ms))
        if rc < 0:
            _check(rc)
        return rc == 1

    def result(self, ticket: int) -> dict:
        """Per-cluster results of a finished ticket (waits for it first); with a
        server configured with keep_inlier_bits also the frame's inlier mask
        (``inlier_bits``, int32 words)."""
        self.wait(ticket)
        K, N = self._sizes[int(ticket)]
        out = {"vx": np.empty(K, np.float32), "vy": np.empty(K, np.float32),
               "heading": np.empty(K, np.float32), "n_inliers": np.empty(K, np.int32),
               "status": np.empty(K, np.uint8), "n_near_tau": np.empty(K, np.int32),
               "best_hyp": np.empty(K, np.int32)}
        bits = np.zeros((N + 31) // 32, np.int32) if self.cfg.keep_inlier_bits else None
        times = RVFrameTimes()
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(load_library().rv_server_result(
            self._h, int(ticket), ptr(out["vx"]), ptr(out["vy"]), ptr(out["heading"]),
            ptr(out["n_inliers"]), ptr(out["status"]), ptr(out["n_near_tau"]),
            ptr(out["best_hyp"]), None if bits is None else ptr(bits), ctypes.byref(times)))
        del self._sizes[int(ticket)]
        self._pinned.pop(int(ticket), None)
        if bits is not None:
            out["inlier_bits"] = bits
        out["times"] = {n: int(getattr(times, n)) for n, _ in RVFrameTimes._fields_}
        return out

    def stats(self) -> dict:
        st = RVServerStats()
        _check(load_library().rv_server_stats(self._h, ctypes.byref(st)))
        return st.to_dict()

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().rv_server_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
