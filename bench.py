#!/usr/bin/env python3
"""Benchmark of the per-cluster RANSAC velocity/heading estimator on one MI355X.

A step is one full estimate of one synthetic frame (all three kernels: point
staging, hypotheses and scoring, refit) with the frame already resident in HBM.  Default workload: the dense
frame (4096 clusters, log-uniform sizes in [8, 4096] points, 30 % outliers,
1024 hypotheses per cluster, tau = 0.15 m/s).

Prints one JSON line: throughput in hypothesis-point evaluations per second
(value), clusters/s, p50/p99 frame latency (host pinned memory -> results in
host memory), the roofline of the scoring kernel from HIP events recorded
around it during the timed steps, and the FP64 CPU oracle timed on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "clusters/s + hyp-point evals/s (% FP32 VALU peak); p50/p99 frame latency"
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 x 2 x 2.4 GHz
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
# Algorithmic HBM bytes of the two other stages of the three-kernel path: the
# staging reads theta and v_d and writes float32 (cos, sin), v_d and the low
# parts (8 + 20 B per point); the refit reads v_d, (cos, sin) and the low parts
# (20 B per point) and writes vx, vy, heading, n_inliers, n_near_tau and status
# (21 B per cluster).
PREP_BYTES_PER_POINT = 28
REFIT_BYTES_PER_POINT = 20
REFIT_BYTES_PER_CLUSTER = 21
FLOP_PER_EVAL = 4                # two fused multiply-adds per hypothesis-point residual

WORKLOAD_TEXT = {
    "dense": ("dense frame: 4096 clusters, log-uniform [8, 4096] points (theta U[-60,60] deg, "
              "(vx, vy) U[-30,30]^2 m/s, noise sigma 0.05 m/s), 30% outliers (15% uniform "
              "U[-40,40], 15% micro-Doppler band +/-[0.5,2]|v|), 1024 hypotheses, tau 0.15 m/s, FP32"),
    "small": ("small frame: 64 clusters of U{20..200} points, 20% uniform outliers, "
              "256 hypotheses, tau 0.15 m/s, FP32"),
    "batched": ("batched form: 256 frames of U{100..1500} clusters, log-uniform [8, 2048] points, "
                "20% uniform outliers, 512 hypotheses, tau 0.15 m/s, FP32; one captured HIP graph "
                "(staging, size-class ordering, persistent work-queue scoring, refit) per step"),
    "served": ("served form: 64 simulated radars, each a Poisson(20 frames/s) source; frames of "
               "U{200..1200} clusters, log-uniform [8, 1024] points, 25% uniform outliers, 512 "
               "hypotheses, tau 0.15 m/s, FP32; frame server with a 16 GiB device budget, "
               "continuous batching over launch slots; frames from and results to host memory"),
}
WORKLOAD_TEXT["precision"] = (
    "precision stress: 512 clusters of 65,536 points (theta U[-60,60] deg, (vx, vy) U[-30,30]^2 m/s, "
    "noise sigma 0.05 m/s), 40% micro-Doppler band outliers +/-[0.5,2]|v|, 4096 hypotheses, "
    "tau 0.15 m/s; FP16 residual form (half2 (cos, sin), v_dot2_f32_f16 onto a float32 offset "
    "residual, widened threshold, exact float32 re-count of possible winners), FP64 refit; one "
    "batched-form call per step")
WORKLOAD_TEXT["paper-sweep"] = (
    "paper-literal variant (normalised line fit, MAD threshold, <= test, least-squares refit) "
    "on the shapes of the paper's Tables I and II: {8, 16, 32, 64} clusters x {100, 150} points, "
    "20% uniform outliers, 256 trials per cluster, FP64")
WORKLOAD_TEXT["issue-rates"] = (
    "wave64 issue rates of the scoring loops' instructions (v_fma_f32, compares, v_dot2_f32_f16, "
    "the scalar popcount), of the float32 and FP16 scoring rows, and of the hypothesis "
    "generation's v_mad_u64_u32, v_mul_hi_u32 and v_fma_f64, eight waves per SIMD "
    "(_lib/issue_probe)")
FRAME_WORKLOADS = ("dense", "small")


def kernel_code_sha256(path: str) -> str:
    """sha256 of a kernel source with its // comments and blank lines removed,
    so that a committed profile stays valid across comment-only edits."""
    import hashlib

    lines = []
    with open(path, encoding="utf-8") as f:
        for line in f:
            code = line.split("//", 1)[0].rstrip()
            if code:
                lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def oracle_error_summary(vx, vy, heading, best, o_vx, o_vy, o_hd, o_best):
    """Per-cluster error of float32 results against the FP64 oracle, over the
    clusters where both kept the same hypothesis (same inlier set up to points
    at tau within FP64 rounding).  dv = max(|vx - vx_o|, |vy - vy_o|); each
    result is also checked against its own bound, the float32 rounding of the
    FP64 refit: dv <= 2^-24 max(|vx_o|, |vy_o|) + 1e-12 m/s."""
    import numpy as np

    same = np.asarray(best) == np.asarray(o_best)
    o_vx = np.asarray(o_vx, dtype=np.float64)[same]
    o_vy = np.asarray(o_vy, dtype=np.float64)[same]
    dv = np.maximum(np.abs(np.asarray(vx, dtype=np.float64)[same] - o_vx),
                    np.abs(np.asarray(vy, dtype=np.float64)[same] - o_vy))
    dh = np.abs(np.remainder(np.asarray(heading, dtype=np.float64)[same]
                             - np.asarray(o_hd, dtype=np.float64)[same] + np.pi, 2 * np.pi) - np.pi)
    bound = 2.0 ** -24 * np.maximum(np.abs(o_vx), np.abs(o_vy)) + 1e-12

    def stats(x):
        if x.size == 0:
            return {"max": None, "p50": None, "p99": None}
        return {"max": float(x.max()), "p50": float(np.median(x)), "p99": float(np.quantile(x, 0.99))}

    return {"clusters": int(same.size), "same_hypothesis": int(same.sum()),
            "abs_dv_mps": stats(dv), "abs_dheading_rad": stats(dh),
            "dv_within_float32_rounding": int(np.count_nonzero(dv <= bound)),
            "dv_bound": "2^-24 max(|vx_o|, |vy_o|) + 1e-12 m/s per cluster"}


def warm_up(step, count: int, min_ms: float) -> int:
    """Untimed warm-up: `count` steps, then more until at least min_ms of wall
    time has passed since the first (the GPU's clocks rise over the first tens
    of milliseconds of sustained work: after 10 dense frames the score kernel
    still takes about 10 % longer than after 200).  Synchronises every few
    steps so that the host clock follows the GPU.  step(i) runs warm-up step i;
    returns the number of steps run."""
    import torch

    t0 = time.perf_counter()
    n = 0
    while n < count or (time.perf_counter() - t0) * 1e3 < min_ms:
        step(n)
        n += 1
        if n % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return n


def profiled_traffic(workload: str, kernel: str = "score_kernel"):
    """HBM bytes per scoring launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a copy of known size), or None
    when there is none for this workload or the kernel code changed since."""
    import re

    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    src = os.path.join(ROOT, "paper_2012_12618_amd", "csrc", "rv.hip")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_code_sha256") != kernel_code_sha256(src):
        return None
    return rec["hbm_bytes_per_launch"]


def profiled_valu_issue(workload: str):
    """Vector-instruction issue of score_kernel from the committed SQ counters
    (same kernel source only): instructions per SIMD per cycle at the clock the
    chip held, against 0.25 for back-to-back full-rate wave64 FMAs."""
    import re

    path = os.path.join(ROOT, "profiles", f"score_kernel_{workload}_counters.md")
    src = os.path.join(ROOT, "paper_2012_12618_amd", "csrc", "rv.hip")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    sq = rec.get("sq")
    if sq is None or rec.get("kernel_code_sha256") != kernel_code_sha256(src):
        return None
    simds, xcds = 1024, 8
    cycles = sq["GRBM_GUI_ACTIVE"] / xcds  # GRBM counts per XCD, summed over the 8
    return {"valu_instructions_per_simd_cycle": sq["SQ_INSTS_VALU"] / (simds * cycles),
            "salu_instructions_per_cu_cycle": sq["SQ_INSTS_SALU"] / (simds / 4 * cycles),
            "clock_ghz": cycles / (rec["kernel_us"] * 1e3), "source": os.path.basename(path)}


def host_cpus() -> dict:
    """What the host offers this process: logical CPUs (nproc), the affinity
    mask, the cgroup CPU quota, the thread-count environment and the CPU model."""
    info = {"nproc": os.cpu_count(), "affinity": None, "cgroup_quota_cpus": None,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS") or None, "model": None}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        quota, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if quota != "max":
            info["cgroup_quota_cpus"] = int(quota) / int(period)
    except (OSError, ValueError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


def oracle_threads(args) -> int:
    """Oracle threads: --cpu-threads, else every CPU this process may use (the
    affinity mask, bounded by the cgroup quota and by OMP_NUM_THREADS, which
    the host sets to this job's CPU share)."""
    if args.cpu_threads:
        return args.cpu_threads
    info = host_cpus()
    n = info["affinity"] or info["nproc"] or 1
    if info["cgroup_quota_cpus"]:
        n = min(n, max(1, int(info["cgroup_quota_cpus"])))
    if info["omp_num_threads"] and info["omp_num_threads"].isdigit():
        n = min(n, max(1, int(info["omp_num_threads"])))
    return n


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def calibration_copy(torch, dev, mb: int) -> None:
    """One device-to-device copy of mb MiB (outside any timed region): the
    kernel of known traffic that scales the HBM byte counters."""
    if mb <= 0:
        return
    nbytes = mb << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    print(f"[bench] calibration copy of {nbytes} bytes", file=sys.stderr, flush=True)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def oracle_baseline(frames, n_hyp, tau, seed_of, threads, budget_s=1.5, max_frames=4096):
    """The FP64 oracle on whole frames (fresh seeds) until about budget_s of wall time."""
    import oracle

    done, dt, evals, clusters = 0, 0.0, 0, 0
    while done == 0 or (dt < budget_s and done < max_frames):
        f = frames[done % len(frames)]
        t0 = time.perf_counter()
        oracle.estimate_velocity(f.theta, f.vd, f.offsets, n_hyp, tau, seed_of(done),
                                 want_mask=False, n_threads=threads)
        dt += time.perf_counter() - t0
        evals += sum_evals(f, n_hyp)
        clusters += f.n_clusters
        done += 1
    return done, dt, evals, clusters


def sum_evals(frame, n_hyp):
    from paper_2012_12618_amd import synth

    return synth.evals_per_frame(frame.offsets, n_hyp)


def timed_frames(call, name, n_frames):
    """call(i, seed) for the n_frames timed frames, with Python's cyclic
    garbage collector off meanwhile (a full collection would stall the timing
    thread for milliseconds and count against one frame)."""
    import gc

    from paper_2012_12618_amd import synth

    was = gc.isenabled()
    gc.disable()
    try:
        return [call(i, synth.ransac_seed(name, 10_000 + i)) for i in range(n_frames)]
    finally:
        if was:
            gc.enable()


def latency_run(torch, binding, synth, dev, stream, name, frame, n_hyp, tau, n_frames,
                zero_copy=False, pipelined_parts=()):
    """Host-clock latency of n_frames distinct frames, each from pinned host
    memory through the H2D copies, the estimate and the D2H copies of the
    per-cluster results (synchronised per frame).  Frame i is drawn fresh for
    the small workload (data seed 100000 + i); for the dense one, whose frames
    are 22 MB each, it is base frame i % 8 (the benchmark frame and seven more
    draws) with every azimuth turned by a distinct angle of at most 0.062 rad,
    so that no two timed frames are equal.  Each frame is written into the
    pinned buffer before its clock starts.  Returns (milliseconds per frame,
    recipe text, with zero_copy the milliseconds per frame of the same frames
    estimated straight from and into pinned host memory, else None, and for each
    count P of pipelined_parts the milliseconds per frame of the same frames sent
    and estimated in P parts, a part's estimate overlapping the next part's copy)."""
    import numpy as np

    if n_frames <= 0:
        return [], None, None, {}
    spec = synth.WORKLOADS[name][0]
    if name == "small":
        bases = [synth.make_frame(spec, 100_000 + i) for i in range(n_frames)]
        recipe = f"{n_frames} frames drawn with data seeds 100000.. (all distinct)"

        def frame_at(i):
            f = bases[i]
            return f.theta, f.vd, f.offsets
    else:
        bases = [frame] + [synth.make_frame(spec, 1000 + f) for f in range(7)]
        recipe = ("8 drawn frames (the benchmark frame, data seeds 1000..1006), frame i = base "
                  "i % 8 with every azimuth turned by ((i // 8) - 62) * 1e-3 rad (float32 add)")

        def frame_at(i):
            f = bases[i % len(bases)]
            phi = np.float32(((i // len(bases)) - 62) * 1e-3)
            return f.theta + phi, f.vd, f.offsets
    n_max = max(f.n_points for f in bases)
    k_max = max(f.n_clusters for f in bases)
    h_t = torch.empty(n_max, dtype=torch.float32).pin_memory()
    h_v = torch.empty(n_max, dtype=torch.float32).pin_memory()
    h_o = torch.empty(k_max + 1, dtype=torch.int32).pin_memory()
    d_t = torch.empty(n_max, dtype=torch.float32, device=dev)
    d_v = torch.empty(n_max, dtype=torch.float32, device=dev)
    d_o = torch.empty(k_max + 1, dtype=torch.int32, device=dev)
    out = binding.allocate_outputs(k_max, n_max, n_hyp, dev, want_near=True)
    keys = ("vx", "vy", "heading", "n_inliers", "status")
    res = {k: torch.empty(out[k].shape, dtype=out[k].dtype).pin_memory() for k in keys}

    def one(i, seed):
        th, vd, off = frame_at(i)
        n, k = th.shape[0], off.shape[0] - 1
        h_t[:n].numpy()[:] = th
        h_v[:n].numpy()[:] = vd
        h_o[:k + 1].numpy()[:] = off
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d_t[:n].copy_(h_t[:n], non_blocking=True)
        d_v[:n].copy_(h_v[:n], non_blocking=True)
        d_o[:k + 1].copy_(h_o[:k + 1], non_blocking=True)
        binding.rv_estimate_velocity(d_t[:n], d_v[:n], d_o[:k + 1], n_hyp, tau, seed, out=out,
                                     stream=stream)
        for key in keys:
            res[key][:k].copy_(out[key][:k], non_blocking=True)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3

    for i in range(min(8, n_frames)):  # untimed first use of the buffers
        one(i, synth.ransac_seed(name, 9_000 + i))
    lat = timed_frames(one, name, n_frames)
    pipe = {P: pipelined_latency(torch, binding, dev, stream, frame_at, n_frames, n_hyp, tau, P,
                                 (h_t, h_v, d_t, d_v), res, name, synth)
            for P in pipelined_parts}
    if not zero_copy:
        return lat, recipe, None, pipe

    # The same frames with no copies: inputs and outputs in pinned host memory,
    # read and written by the kernels through their device mapping, one
    # prepared call per frame (the buffers hold the largest frame).
    z_out = binding.allocate_outputs(k_max, n_max, n_hyp, "cpu", want_near=True)
    z_ws = out["workspace"]
    z_out = {key: (v.pin_memory() if key != "workspace" else z_ws) for key, v in z_out.items()}
    prep = binding.PreparedEstimate(h_t, h_v, h_o, n_hyp, tau, z_out, stream=stream)

    def zero(i, seed):
        th, vd, off = frame_at(i)
        n, k = th.shape[0], off.shape[0] - 1
        h_t[:n].numpy()[:] = th
        h_v[:n].numpy()[:] = vd
        h_o[:k + 1].numpy()[:] = off
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prep(seed, n_points=n, n_clusters=k)
        stream.synchronize()
        return (time.perf_counter() - t0) * 1e3

    for i in range(min(8, n_frames)):
        zero(i, synth.ransac_seed(name, 9_000 + i))
    lat_z = timed_frames(zero, name, n_frames)
    return lat, recipe, lat_z, pipe


def pipelined_latency(torch, binding, dev, stream, frame_at, n_frames, n_hyp, tau, n_parts,
                      buffers, res, name, synth):
    """Host-clock latency of the frames of latency_run sent and estimated in
    n_parts parts (shrinking toward the end) by rv_estimate_velocity_pipelined: part
    j's estimate runs on the compute stream while part j + 1 is copied on a copy
    stream, and the per-cluster results are written straight into pinned host
    memory through its device mapping.  The clock covers the call (cutting the
    frame, every enqueue) and the final synchronisation.  Also checks the first
    frame's results against the whole-frame call bit for bit.  Returns
    (milliseconds per frame, whether the results matched)."""
    import numpy as np

    h_t, h_v, d_t, d_v = buffers
    k_max = max(res["vx"].shape[0], 1)
    copy_stream = torch.cuda.Stream(device=dev)
    h_o = torch.empty(k_max + 1, dtype=torch.int32).pin_memory()
    d_o = torch.empty(k_max + 1, dtype=torch.int32, device=dev)
    keys = ("vx", "vy", "heading", "n_inliers", "status")
    z = {k: torch.empty(res[k].shape, dtype=res[k].dtype).pin_memory() for k in keys}
    z["workspace"] = torch.empty(max(binding.rv_workspace_bytes(k_max, h_t.shape[0], n_hyp), 1),
                                 dtype=torch.uint8, device=dev)

    def run(i, seed):
        th, vd, off = frame_at(i)
        n, k = th.shape[0], off.shape[0] - 1
        h_t[:n].numpy()[:] = th
        h_v[:n].numpy()[:] = vd
        h_o[:k + 1].numpy()[:] = off
        part_out = {key: v[:k] for key, v in z.items() if key != "workspace"}
        part_out["workspace"] = z["workspace"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        binding.rv_estimate_velocity_pipelined(h_t[:n], h_v[:n], h_o[:k + 1], n_parts, n_hyp, tau,
                                               seed, device_inputs=(d_t, d_v, d_o), out=part_out,
                                               stream=stream, copy_stream=copy_stream)
        stream.synchronize()
        return (time.perf_counter() - t0) * 1e3

    seed0 = synth.ransac_seed(name, 9_000)
    run(0, seed0)
    th, vd, off = frame_at(0)
    whole = binding.rv_estimate_velocity(torch.from_numpy(th).to(dev), torch.from_numpy(vd).to(dev),
                                         torch.from_numpy(off).to(dev), n_hyp, tau, seed0,
                                         want_near=False, stream=stream)
    stream.synchronize()
    k0 = off.shape[0] - 1
    same = all(np.array_equal(z[key][:k0].numpy().view(np.uint8),
                              whole[key].cpu().numpy().view(np.uint8)) for key in keys)
    for i in range(1, min(8, n_frames)):
        run(i, synth.ransac_seed(name, 9_000 + i))
    lat = timed_frames(run, name, n_frames)
    return lat, same


def batch_bench(args, torch, binding, synth, dev) -> dict:
    """Batched form: every step replays one captured graph over all frames."""
    name = args.workload
    print(f"[bench] generating {name} workload", file=sys.stderr, flush=True)
    batch, n_hyp, tau = synth.make_batch_workload(name, n_frames=args.frames or None)
    fr = batch.frame
    F, K, N = batch.n_frames, fr.n_clusters, fr.n_points
    evals = synth.evals_per_frame(fr.offsets, n_hyp)
    theta = torch.from_numpy(fr.theta).to(dev)
    vd = torch.from_numpy(fr.vd).to(dev)
    offsets = torch.from_numpy(fr.offsets).to(dev)
    fo = torch.from_numpy(batch.frame_offsets).to(dev)
    seeds = torch.from_numpy(batch.seeds.view("int64")).to(dev)
    tuning = None
    if args.tuning:
        from paper_2012_12618_amd import tuner

        tuning = tuner.load(args.tuning, torch.cuda.get_device_name(dev), n_hyp)
    if args.fp16_min_points > 0:
        tuning = tuning or binding.rv_tuning_default()
        tuning.fp16_min_points = args.fp16_min_points
    out = binding.allocate_batch_outputs(F, K, N, n_hyp, dev, want_near=True)
    stream = torch.cuda.current_stream(dev)
    graph = binding.rv_graph_capture_batch(theta, vd, offsets, fo, seeds, n_hyp, tau, out,
                                           tuning=tuning)

    def step():
        seeds.add_(1)  # fresh hypothesis seeds for every frame of every step
        graph.launch(stream)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    warm_steps = warm_up(lambda i: step(), args.warmup, args.min_warmup_ms)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    print(f"[bench] timing {args.steps} graph steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    graph.destroy()

    # Per-kernel durations: the same launch sequence called eagerly with the
    # library's events around each kernel.
    print(f"[bench] kernel timing over {args.steps} eager calls", file=sys.stderr, flush=True)
    binding.rv_stage_times()
    binding.rv_stage_timing(True)
    for _ in range(args.steps):
        seeds.add_(1)
        binding.rv_estimate_velocity_batch(theta, vd, offsets, fo, seeds, n_hyp, tau,
                                           tuning=tuning, out=out, stream=stream)
    torch.cuda.synchronize()
    binding.rv_stage_timing(False)
    stage_ms, n_calls = binding.rv_stage_times()
    stage_avg = [x / max(n_calls, 1) for x in stage_ms]
    score_ms = stage_avg[binding.STAGE_NAMES.index("score")]
    achieved_tflops = FLOP_PER_EVAL * evals / (score_ms / 1e3) / 1e12

    # The plain per-frame form on the same frames, one call per frame.
    print("[bench] per-frame form on the same frames", file=sys.stderr, flush=True)
    per = []
    for f in range(F):
        s = batch.frame_slice(f)
        t_ = (torch.from_numpy(s.theta).to(dev), torch.from_numpy(s.vd).to(dev),
              torch.from_numpy(s.offsets).to(dev))
        per.append((t_, int(batch.seeds[f]), binding.allocate_outputs(s.n_clusters, s.n_points, n_hyp, dev)))

    def per_frame_pass(salt):
        for (t_, v_, o_), seed, o2 in per:
            binding.rv_estimate_velocity(t_, v_, o_, n_hyp, tau, (seed + salt) & (2**64 - 1), out=o2,
                                         stream=stream)

    per_frame_pass(0)
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 5))
    ev0.record(stream)
    for r in range(reps):
        per_frame_pass(r + 1)
    ev1.record(stream)
    torch.cuda.synchronize()
    per_frame_ms = ev0.elapsed_time(ev1) / reps
    del per
    calibration_copy(torch, dev, args.copy_calibration_mb)

    cpu = None
    if not args.no_cpu_baseline:
        threads = oracle_threads(args)
        print(f"[bench] oracle on the host, {threads} threads", file=sys.stderr, flush=True)
        sample = [batch.frame_slice(f) for f in range(min(F, 8))]
        done, dt, ev_done, cl_done = oracle_baseline(
            sample, n_hyp, tau, lambda i: synth.frame_seed(name, 50_000 + i), threads)
        cpu = {"value": ev_done / dt, "unit": "hyp-point evals/s", "cores": threads, "kind": "oracle",
               "sample": (f"{done} whole frame(s) of the batch ({cl_done} clusters, {ev_done} evals), "
                          f"FP64, {dt:.2f} s wall on {threads} threads"),
               "clusters_per_s": cl_done / dt, "host": host_cpus()}

    sec = ms_per_step / 1e3
    line = {
        "metric": METRIC,
        "value": evals / sec,
        "unit": "hyp-point evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_steps_run": warm_steps,
        "min_warmup_ms": args.min_warmup_ms,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16" if tuning is not None and tuning.fp16_min_points > 0 else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[name], "frames": F, "clusters": K, "points": N,
                   "n_hyp": n_hyp, "tau": tau, "evals_per_step": evals,
                   "tuning": tuning.to_dict() if tuning is not None else "default"},
        "clusters_per_s": K / sec,
        "frac_fp32_valu_peak": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
        "per_frame_form": {"ms_per_batch": per_frame_ms, "clusters_per_s": K / (per_frame_ms / 1e3),
                           "evals_per_s": evals / (per_frame_ms / 1e3),
                           "scope": "rv_estimate_velocity once per frame, same frames, one stream"},
        "stage_ms": dict(zip(binding.STAGE_NAMES, stage_avg)),
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "roofline": {"bound": "alu", "kernel": "batch_score_kernel", "achieved": achieved_tflops,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": profiled_traffic(name, "batch_score_kernel"),
                     "algorithmic_flop_per_launch": FLOP_PER_EVAL * evals,
                     "kernel_ms": score_ms},
        "cpu_baseline": cpu,
    }
    return line


def served_bench(args, torch, binding, synth, dev, extra_fp16: int = 0,
                 zero_copy: bool = False) -> dict:
    """Served form: paced arrivals for latency, then the same frames as fast as
    the server takes them for throughput; the per-frame form (one frame per
    launch, one slot) on the same traffic for comparison.  extra_fp16 > 0: the
    served form also runs in the FP16 residual form for clusters of at least
    that many points ("served_fp16_form"), against the same per-frame run.
    zero_copy: the served and per-frame forms also run with every frame held
    in pinned host memory and queued without a copy (RVServer.submit_pinned;
    "served_zero_copy_form", "per_frame_zero_copy_form")."""
    from paper_2012_12618_amd import serve

    name = args.workload
    n_radars, fps = 64, 20.0
    print(f"[bench] generating {n_radars} radar frames", file=sys.stderr, flush=True)
    batch, n_hyp, tau = synth.make_batch_workload(name, n_frames=n_radars)
    frames = [batch.frame_slice(f) for f in range(n_radars)]
    schedule = serve.arrival_schedule(n_radars, fps, args.duration, seed=1)
    warm = serve.arrival_schedule(n_radars, fps, 0.5, seed=2)
    tuning = None
    if args.tuning:
        from paper_2012_12618_amd import tuner

        tuning = tuner.load(args.tuning, torch.cuda.get_device_name(dev), n_hyp)

    def make_server(max_batch, n_streams, fp16_min):
        cfg = binding.rv_server_config_default()
        cfg.n_hyp, cfg.tau = n_hyp, tau
        cfg.hbm_budget_bytes = 16 << 30
        cfg.max_batch_frames, cfg.n_streams = max_batch, n_streams
        if tuning is not None:
            cfg.tuning = tuning
        if fp16_min > 0:  # served forms only; the per-frame form stays FP32
            cfg.tuning.fp16_min_points = fp16_min
        return binding.RVServer(cfg)

    def seed_of(a):
        return synth.frame_seed(name, a.index)

    out = {}
    forms = [("served", 64, 2, args.fp16_min_points, False)]
    if extra_fp16 > 0:
        forms.append(("served_fp16", 64, 2, extra_fp16, False))
    forms.append(("per_frame", 1, 1, 0, False))
    pinned = None
    if zero_copy:
        forms += [("served_zero_copy", 64, 2, args.fp16_min_points, True),
                  ("per_frame_zero_copy", 1, 1, 0, True)]
        pinned = [tuple(torch.from_numpy(a).pin_memory() for a in (f.theta, f.vd, f.offsets))
                  for f in frames]
    for form, max_batch, n_streams, fp16_min, zc in forms:
        server = make_server(max_batch, n_streams, fp16_min)
        pf = pinned if zc else None
        try:
            print(f"[bench] {form}: warmup", file=sys.stderr, flush=True)
            serve.run_traffic(server, frames, warm, seed_of, n_hyp, paced=False,
                              submitters=args.submitters, pinned_frames=pf)
            print(f"[bench] {form}: {len(schedule)} paced arrivals over {args.duration} s",
                  file=sys.stderr, flush=True)
            paced, _ = serve.run_traffic(server, frames, schedule, seed_of, n_hyp, paced=True,
                                         submitters=args.submitters, pinned_frames=pf)
            print(f"[bench] {form}: same arrivals unpaced", file=sys.stderr, flush=True)
            if form == "served":
                binding.rv_stage_times()
                binding.rv_stage_timing(True)
            sat, _ = serve.run_traffic(server, frames, schedule, seed_of, n_hyp, paced=False,
                                       submitters=args.submitters, pinned_frames=pf)
            if form == "served":
                binding.rv_stage_timing(False)
                out["stages"] = binding.rv_stage_times()
        finally:
            server.destroy()
        out[form] = (paced.summary(), sat.summary(), sat)

    paced_s, sat_s, sat = out["served"]
    paced_f, sat_f, _ = out["per_frame"]
    stage_ms, n_calls = out["stages"]
    score_ms_total = stage_ms[binding.STAGE_NAMES.index("score")]
    achieved_tflops = FLOP_PER_EVAL * sat.evals / (score_ms_total / 1e3) / 1e12 if score_ms_total else 0.0

    cpu = None
    if not args.no_cpu_baseline:
        threads = oracle_threads(args)
        print(f"[bench] oracle on the host, {threads} threads", file=sys.stderr, flush=True)
        done, dt, ev_done, cl_done = oracle_baseline(
            frames[:8], n_hyp, tau, lambda i: synth.frame_seed(name, 90_000 + i), threads)
        cpu = {"value": ev_done / dt, "unit": "hyp-point evals/s", "cores": threads, "kind": "oracle",
               "sample": (f"{done} radar frame(s) ({cl_done} clusters, {ev_done} evals), FP64, "
                          f"{dt:.2f} s wall on {threads} threads"),
               "clusters_per_s": cl_done / dt, "host": host_cpus()}

    def brief(paced_sum, sat_sum):
        return {"latency_ms": paced_sum["latency_ms"], "server_latency_ms": paced_sum["server_latency_ms"],
                "offered_frames_per_s": paced_sum["frames_per_s"],
                "mean_batch_frames_paced": paced_sum["mean_batch_frames"],
                "saturated": {k: sat_sum[k] for k in ("frames_per_s", "clusters_per_s", "evals_per_s",
                                                      "mean_batch_frames", "wall_s")}}

    line = {
        "metric": METRIC,
        "value": sat_s["evals_per_s"],
        "unit": "hyp-point evals/s",
        "n_gpus": 1,
        "steps": sat_s["frames"],
        "warmup": len(warm),
        "ms_per_step": sat_s["wall_s"] * 1e3 / max(sat_s["frames"], 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16" if args.fp16_min_points > 0 else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[name], "radars": n_radars, "fps_per_radar": fps,
                   "fp16_min_points": args.fp16_min_points,
                   "duration_s": args.duration, "frames": len(schedule), "n_hyp": n_hyp, "tau": tau,
                   "distinct_frame_contents": n_radars,
                   "value_scope": "frames submitted back to back from host memory, results back "
                                  "in host memory (copies included)",
                   "submitters": args.submitters},
        "clusters_per_s": sat_s["clusters_per_s"],
        "latency_ms": paced_s["latency_ms"],
        "served_form": brief(paced_s, sat_s),
        "per_frame_form": brief(paced_f, sat_f),
        "server": sat_s["server"],
        "frac_fp32_valu_peak": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
        "roofline": {"bound": "alu", "kernel": "batch_score_kernel", "achieved": achieved_tflops,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": None,
                     "algorithmic_flop_per_launch": FLOP_PER_EVAL * sat.evals / max(n_calls, 1),
                     "kernel_ms": score_ms_total / max(n_calls, 1), "launches": n_calls},
        "cpu_baseline": cpu,
    }
    if extra_fp16 > 0:
        paced_h, sat_h, _ = out["served_fp16"]
        line["served_fp16_form"] = dict(brief(paced_h, sat_h), fp16_min_points=extra_fp16)
    if zero_copy:
        scope = ("frames held in pinned host memory, queued without a copy "
                 "(RVServer.submit_pinned); results back in host memory")
        for form in ("served_zero_copy", "per_frame_zero_copy"):
            paced_z, sat_z, _ = out[form]
            line[form + "_form"] = dict(brief(paced_z, sat_z), scope=scope)
    return line


def paper_sweep_bench(args, torch, binding, synth, dev) -> int:
    """Tables I and II of the paper: per shape, GPU time per frame (whole calls
    back to back: the one-launch path), and of the trial stage (normalisation,
    threshold and trials: Table I's kernel) and the refit (Table II's kernel)
    from the library's events on the three-kernel path (the one the frame-wide
    inlier mask takes), over fresh seeds."""
    import numpy as np

    H = 256
    rows = []
    stream = torch.cuda.current_stream(dev)
    for clusters, points in synth.TABLE_SHAPES:
        f = synth.table_frame(clusters, points)
        t = torch.from_numpy(f.theta).to(dev)
        v = torch.from_numpy(f.vd).to(dev)
        o = torch.from_numpy(f.offsets).to(dev)
        # Outputs and workspace allocated once per shape, as a caller that
        # estimates frame after frame would hold them.
        out = binding.allocate_paper_outputs(f.n_clusters, f.n_points, H, dev)
        out_bits = binding.allocate_paper_outputs(f.n_clusters, f.n_points, H, dev, want_bits=True)
        warm_up(lambda i: binding.rv_estimate_velocity_paper(
            t, v, o, H, synth.ransac_seed("paper", i), out=out, stream=stream),
            args.warmup, args.min_warmup_ms)
        # Whole calls first, then the same number of calls with the library's
        # per-kernel events (each event is a queue marker that lengthens a call)
        # on the three-kernel path, whose stages are separate launches.
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for i in range(args.steps):
            binding.rv_estimate_velocity_paper(t, v, o, H, synth.ransac_seed("paper", 1000 + i),
                                               out=out, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        binding.rv_stage_times()
        binding.rv_stage_timing(True)
        for i in range(args.steps):
            binding.rv_estimate_velocity_paper(t, v, o, H, synth.ransac_seed("paper", 2000 + i),
                                               out=out_bits, stream=stream)
        torch.cuda.synchronize()
        binding.rv_stage_timing(False)
        ms, n = binding.rv_stage_times()
        stage = [x / max(n, 1) for x in ms]
        row = {"clusters": clusters, "points": points,
               "gpu_ms_per_frame": ev0.elapsed_time(ev1) / args.steps,
               "gpu_ransac_ms": stage[0] + stage[1], "gpu_lsq_ms": stage[2]}
        if args.host_comparators:
            row.update(host_comparators(f, H))
        rows.append(row)
        print(f"[bench] paper {clusters}x{points}: {row['gpu_ms_per_frame']:.4f} ms/frame",
              file=sys.stderr, flush=True)
    big = rows[-1]
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        f = synth.table_frame(64, 150)
        done, dt = 0, 0.0
        while done == 0 or (dt < 1.5 and done < 4096):
            t0 = time.perf_counter()
            oracle.estimate_velocity_paper(f.theta, f.vd, f.offsets, H, 50_000 + done, want_mask=False)
            dt += time.perf_counter() - t0
            done += 1
        cpu = {"value": done * f.n_clusters / dt, "unit": "clusters/s", "cores": 1, "kind": "oracle",
               "sample": f"{done} frame(s) of 64 clusters x 150 points, H = {H}, FP64, {dt:.2f} s on one thread"}
    line = {
        "metric": METRIC,
        "value": big["clusters"] / (big["gpu_ms_per_frame"] / 1e3),
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "min_warmup_ms": args.min_warmup_ms,
        "ms_per_step": big["gpu_ms_per_frame"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["paper-sweep"], "n_hyp": H,
                   "value_scope": "64 clusters x 150 points, whole estimate per frame"},
        "table": rows,
        "paper_table_ms": {"ransac_gtx1060": {"8x100": 1.64, "8x150": 1.77, "16x100": 1.68,
                                              "16x150": 1.82, "32x100": 1.73, "32x150": 1.89,
                                              "64x100": 1.98, "64x150": 2.23},
                           "lsq_gtx1060": {"8x100": 1.81, "8x150": 1.83, "16x100": 1.81,
                                           "16x150": 1.83, "32x100": 1.81, "32x150": 1.83,
                                           "64x100": 1.81, "64x150": 1.83},
                           "note": "the paper's own timings on its hardware, context only"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


def precision_bench(args, torch, binding, synth, dev, oracle_budget_s: float = 10.0) -> dict:
    """Precision-stress shape: the FP16 residual form against the float32 form
    on the same frame (both through the batched entry point, one frame), every
    output compared bitwise, and the FP64 oracle on sampled clusters."""
    import numpy as np

    import oracle

    print("[bench] generating precision workload", file=sys.stderr, flush=True)
    frame, n_hyp, tau = synth.make_workload("precision")
    K, N = frame.n_clusters, frame.n_points
    evals = synth.evals_per_frame(frame.offsets, n_hyp)
    theta = torch.from_numpy(frame.theta).to(dev)
    vd = torch.from_numpy(frame.vd).to(dev)
    offsets = torch.from_numpy(frame.offsets).to(dev)
    fo = torch.tensor([0, K], dtype=torch.int32, device=dev)
    seeds = torch.tensor([synth.ransac_seed("precision")], dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    fp16_min = args.fp16_min_points or 1024
    forms = {}
    for form, m in (("fp32", 0), ("fp16", fp16_min)):
        tune = binding.rv_tuning_default()
        tune.fp16_min_points = m
        out = binding.allocate_batch_outputs(1, K, N, n_hyp, dev, want_near=True, want_bits=True,
                                             debug=True)

        def call(t=tune, o=out):
            binding.rv_estimate_velocity_batch(theta, vd, offsets, fo, seeds, n_hyp, tau, tuning=t,
                                               out=o, stream=stream)

        print(f"[bench] {form} form: warmup {args.warmup}, {args.steps} steps", file=sys.stderr, flush=True)
        warm_up(lambda i: call(), args.warmup, args.min_warmup_ms)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        binding.rv_stage_times()
        binding.rv_stage_timing(True)
        ev0.record(stream)
        for _ in range(args.steps):
            call()
        ev1.record(stream)
        torch.cuda.synchronize()
        binding.rv_stage_timing(False)
        stage_ms, n_calls = binding.rv_stage_times()
        stage = dict(zip(binding.STAGE_NAMES, [x / max(n_calls, 1) for x in stage_ms]))
        res = {k: v.cpu().numpy() for k, v in out.items() if k != "workspace"}
        forms[form] = {"ms_per_step": ev0.elapsed_time(ev1) / args.steps, "stage_ms": stage, "res": res}
    calibration_copy(torch, dev, args.copy_calibration_mb)
    keys = ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau", "inlier_bits")
    identical = all(np.array_equal(forms["fp16"]["res"][k], forms["fp32"]["res"][k],
                                   equal_nan=k in ("vx", "vy", "heading")) for k in keys)

    # Error of the results against the FP64 oracle on sampled clusters; the
    # same oracle run is the CPU baseline.
    # Error of every result against the FP64 oracle, over clusters taken in
    # rounds of `threads` spread across the frame until about 10 s of oracle
    # wall time (or all of them); the same runs are the CPU baseline.
    threads = oracle_threads(args)
    order = [k for r in range(max(1, K // threads)) for k in range(r, K, max(1, K // threads))]
    ids, dt, rounds = [], 0.0, []
    g = forms["fp16"]["res"]
    o_parts = []
    while len(ids) < K and (dt < oracle_budget_s or not ids):
        chunk = order[len(ids):len(ids) + threads]
        print(f"[bench] oracle on clusters {chunk[0]}.. ({len(ids) + len(chunk)}/{K}), {threads} threads",
              file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        o_parts.append(oracle.estimate_velocity(frame.theta, frame.vd, frame.offsets, n_hyp, tau,
                                                synth.ransac_seed("precision"), cluster_ids=chunk,
                                                want_mask=False, n_threads=threads))
        dt += time.perf_counter() - t0
        ids += chunk
    o_vx = np.concatenate([p.vx for p in o_parts])
    o_vy = np.concatenate([p.vy for p in o_parts])
    o_hd = np.concatenate([p.heading for p in o_parts])
    o_best = np.concatenate([p.best_hyp for p in o_parts])
    idx = np.asarray(ids)
    err = oracle_error_summary(g["vx"][idx], g["vy"][idx], g["heading"][idx], g["best_hyp"][idx],
                               o_vx, o_vy, o_hd, o_best)
    ev_sample = int(sum((int(frame.offsets[k + 1]) - int(frame.offsets[k])) * n_hyp for k in ids))
    cpu = None if args.no_cpu_baseline else {
        "value": ev_sample / dt, "unit": "hyp-point evals/s", "cores": min(threads, len(ids)),
        "kind": "oracle",
        "sample": f"{len(ids)} clusters of 65,536 points x 4096 hypotheses, FP64, {dt:.2f} s wall",
        "host": host_cpus()}

    f16, f32 = forms["fp16"], forms["fp32"]
    recount = fp16_recount_stats(f16["res"]["hyp_counts"], f32["res"]["hyp_counts"],
                                 np.diff(frame.offsets), n_hyp)
    score16 = f16["stage_ms"]["score"]
    achieved = FLOP_PER_EVAL * evals / (score16 / 1e3) / 1e12
    sec = f16["ms_per_step"] / 1e3
    line = {
        "metric": METRIC,
        "value": evals / sec,
        "unit": "hyp-point evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "min_warmup_ms": args.min_warmup_ms,
        "ms_per_step": f16["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["precision"], "clusters": K, "points": N, "n_hyp": n_hyp,
                   "tau": tau, "evals_per_step": evals, "fp16_min_points": fp16_min},
        "clusters_per_s": K / sec,
        "fp32_form": {"ms_per_step": f32["ms_per_step"], "evals_per_s": evals / (f32["ms_per_step"] / 1e3),
                      "stage_ms": f32["stage_ms"]},
        "fp16_over_fp32_time": f16["ms_per_step"] / f32["ms_per_step"],
        "outputs_bitwise_equal_to_fp32_form": identical,
        "fp16_recount": recount,
        "oracle_error": dict(err, scope="FP16-form results (bitwise the float32 form's) against "
                                         "the FP64 oracle, per cluster"),
        "stage_ms": f16["stage_ms"],
        "roofline": {"bound": "alu", "kernel": "batch_score_kernel", "achieved": achieved,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": profiled_traffic("precision", "batch_score_kernel"),
                     "algorithmic_flop_per_launch": FLOP_PER_EVAL * evals, "kernel_ms": score16,
                     "note": "the MI355X vector FP16 and FP32 peaks are the same 157.3 TFLOP/s"},
        "cpu_baseline": cpu,
    }
    return line


def fp16_recount_stats(hi, exact, sizes, n_hyp, block=256):
    """Work of the FP16 form's exact re-count, per scoring block of 256
    hypotheses, from the per-hypothesis counts of the two forms: hi (FP16 form,
    an upper bound of the float32 count) and exact (float32 form).  A block
    counts exactly, in its first pass, the hypothesis with the largest (hi,
    lowest index) among those with a finite widened threshold together with
    those without one ("wide": their FP16 row counted every finite point, seen
    here as hi equal to the cluster size with a smaller exact count); then
    every other hypothesis with hi at least the first one's exact count, 64 per
    pass.  Hypotheses with hi = 0 (invalid, or no point within the widened
    threshold) are never candidates."""
    import numpy as np

    sizes = np.asarray(sizes, np.int64)
    n_clusters = sizes.size
    hi = np.asarray(hi, np.int64).reshape(n_clusters, n_hyp)
    ex = np.asarray(exact, np.int64).reshape(n_clusters, n_hyp)
    rows = np.arange(n_clusters)
    cands, wides, slack = [], [], []
    for b0 in range(0, n_hyp, block):
        h = hi[:, b0:b0 + block]
        e = ex[:, b0:b0 + block]
        wide = (h >= sizes[:, None]) & (e < h)
        finite = (h > 0) & ~wide
        top = np.argmax(np.where(finite, h, -1), axis=1)  # first maximum: the lowest index
        has_top = finite[rows, top]
        t = np.where(has_top, e[rows, top], 0)
        c = finite & (h >= t[:, None])
        c[rows, top] &= ~has_top
        cands.append(c.sum(axis=1))
        wides.append(wide.sum(axis=1))
        slack.append(h - e)
    cands = np.concatenate(cands)
    wides = np.concatenate(wides)
    slack = np.concatenate(slack, axis=1)
    passes = 1 + (cands + 63) // 64
    return {"blocks": int(cands.size),
            "wide_per_block": {"mean": float(wides.mean()), "max": int(wides.max())},
            "candidates_per_block": {"mean": float(cands.mean()), "p50": float(np.median(cands)),
                                     "p99": float(np.quantile(cands, 0.99)), "max": int(cands.max())},
            "exact_passes_per_block": {"mean": float(passes.mean()), "max": int(passes.max())},
            "hi_minus_exact": {"mean": float(slack.mean()), "max": int(slack.max()),
                               "min": int(slack.min())},
            "scope": "per block of 256 hypotheses: hypotheses without a finite FP16 threshold, "
                     "candidates re-counted in float32 after the first exact pass, and exact "
                     "passes over the cluster (the first, then 64 candidates per pass)"}


def host_comparators(f, H):
    """The paper's host comparators on one frame: scikit-learn RANSACRegressor of
    v_d on theta per cluster (max_trials = H) and numpy.linalg.pinv per cluster."""
    import numpy as np

    out = {}
    try:
        from sklearn.linear_model import RANSACRegressor

        t0 = time.perf_counter()
        for k in range(f.n_clusters):
            a, b = f.offsets[k], f.offsets[k + 1]
            RANSACRegressor(max_trials=H, random_state=k).fit(
                f.theta[a:b, None].astype(np.float64), f.vd[a:b].astype(np.float64))
        out["sklearn_ransac_ms"] = (time.perf_counter() - t0) * 1e3
    except ImportError:
        out["sklearn_ransac_ms"] = None
    t0 = time.perf_counter()
    for k in range(f.n_clusters):
        a, b = f.offsets[k], f.offsets[k + 1]
        th = f.theta[a:b].astype(np.float64)
        A = np.stack([np.cos(th), np.sin(th)], axis=1)
        np.linalg.pinv(A) @ f.vd[a:b].astype(np.float64)
    out["numpy_pinv_ms"] = (time.perf_counter() - t0) * 1e3
    return out


def frame_bench(args, torch, binding, synth, dev, name) -> dict:
    """One frame resident in HBM, estimated step after step (dense or small)."""
    import numpy as np

    print(f"[bench] generating {name} workload", file=sys.stderr, flush=True)
    frame, n_hyp, tau = synth.make_workload(name)
    K, N = frame.n_clusters, frame.n_points
    evals = synth.evals_per_frame(frame.offsets, n_hyp)

    theta = torch.from_numpy(frame.theta).to(dev)
    vd = torch.from_numpy(frame.vd).to(dev)
    offsets = torch.from_numpy(frame.offsets).to(dev)
    out = binding.allocate_outputs(K, N, n_hyp, dev, want_near=True)
    stream = torch.cuda.current_stream(dev)
    # Arguments checked and marshalled once; each step passes a fresh seed.
    estimate = binding.PreparedEstimate(theta, vd, offsets, n_hyp, tau, out, stream)

    def step(i):
        estimate(synth.ransac_seed(name, i))

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    warm_steps = warm_up(step, args.warmup, args.min_warmup_ms)

    # Timed region: K steps between two events on the launch stream.  The
    # library's own events around each kernel (per-kernel durations) are
    # recorded on every stage_sample_every-th step of the same region: each
    # event is a marker in the stream's queue, and recorded on every step they
    # would lengthen it.
    binding.rv_stage_times()  # drop anything recorded before
    ev_start = torch.cuda.Event(enable_timing=True)
    ev_end = torch.cuda.Event(enable_timing=True)
    every = max(1, args.stage_sample_every)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ev_start.record(stream)
    for i in range(args.steps):
        sampled = i % every == 0
        if sampled:
            binding.rv_stage_timing(True)
        step(warm_steps + i)
        if sampled:
            binding.rv_stage_timing(False)
    ev_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, n_calls = binding.rv_stage_times()
    ms_per_step = ev_start.elapsed_time(ev_end) / args.steps
    # Spread of single steps: a second pass of K steps with an event between
    # consecutive steps (outside the timed region; those markers lengthen
    # short steps).
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for i in range(args.steps):
        step(warm_steps + args.steps + i)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    step_times = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    sec = ms_per_step / 1e3
    evals_per_s = evals / sec
    clusters_per_s = K / sec
    stage_avg = [x / max(n_calls, 1) for x in stage_ms]
    score_ms = stage_avg[binding.STAGE_NAMES.index("score")]
    achieved_tflops = FLOP_PER_EVAL * evals / (score_ms / 1e3) / 1e12
    # The library's rule for its one-launch path (no inlier mask is requested
    # here): the whole estimate is then one kernel, timed as the scoring stage.
    small_path = n_hyp <= 256 and N <= (1 << 16) and K <= (1 << 16)
    kernel = "small_frame_kernel" if small_path else "score_kernel"

    # Frame latency: pinned host frame -> device -> estimate -> results in host memory.
    print(f"[bench] latency over {args.latency_frames} distinct frames", file=sys.stderr, flush=True)
    # Small frames also straight from and into pinned host memory (no copies);
    # a large frame would send its seed-azimuth reads over PCIe, so it is copied.
    # Large frames are also sent in parts, each part's estimate overlapping the next one's copy.
    lat, lat_recipe, lat_z, lat_p = latency_run(
        torch, binding, synth, dev, stream, name, frame, n_hyp, tau, args.latency_frames,
        zero_copy=small_path, pipelined_parts=() if small_path else (2, 3, 4, 8))

    calibration_copy(torch, dev, args.copy_calibration_mb)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        threads = oracle_threads(args)
        print(f"[bench] oracle on the host, {threads} threads", file=sys.stderr, flush=True)
        # Whole frames with fresh hypothesis seeds until about 1.5 s of wall time.
        frames_done, dt = 0, 0.0
        while frames_done == 0 or (dt < 1.5 and frames_done < 64):
            t0 = time.perf_counter()
            oracle.estimate_velocity(frame.theta, frame.vd, frame.offsets, n_hyp, tau,
                                     synth.ransac_seed(name, 20_000 + frames_done), want_mask=False,
                                     n_threads=threads)
            dt += time.perf_counter() - t0
            frames_done += 1
        cpu = {"value": frames_done * evals / dt, "unit": "hyp-point evals/s", "cores": threads,
               "kind": "oracle",
               "sample": (f"{frames_done} whole {name} frame(s) ({K} clusters, {evals} evals each, "
                          f"fresh seeds), FP64, {dt:.2f} s wall on {threads} threads"),
               "clusters_per_s": frames_done * K / dt, "host": host_cpus()}
        # One thread on every 8th cluster of the frame.
        ids = np.arange(0, K, 8)
        sizes = np.diff(frame.offsets.astype(np.int64))[ids]
        ev1 = int(n_hyp * sizes[sizes >= 2].sum())
        t0 = time.perf_counter()
        oracle.estimate_velocity(frame.theta, frame.vd, frame.offsets, n_hyp, tau,
                                 synth.ransac_seed(name, 30_000), cluster_ids=ids, want_mask=False,
                                 n_threads=1)
        dt1 = time.perf_counter() - t0
        cpu["one_thread"] = {"value": ev1 / dt1, "unit": "hyp-point evals/s",
                             "clusters_per_s": len(ids) / dt1,
                             "sample": f"every 8th cluster ({len(ids)} clusters, {ev1} evals), {dt1:.2f} s"}

    line = {
        "metric": METRIC,
        "value": evals_per_s,
        "unit": "hyp-point evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_steps_run": warm_steps,
        "min_warmup_ms": args.min_warmup_ms,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[name], "clusters": K, "points": N, "n_hyp": n_hyp,
                   "tau": tau, "evals_per_frame": evals},
        "clusters_per_s": clusters_per_s,
        "frac_fp32_valu_peak": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
        "latency_ms": ({"p50": percentile(lat, 50), "p99": percentile(lat, 99), "frames": len(lat),
                        "distinct_frames": len(lat), "frames_recipe": lat_recipe,
                        "scope": "pinned host frame -> H2D -> estimate -> D2H of per-cluster results"}
                       if lat else None),
        "latency_zero_copy_ms": ({"p50": percentile(lat_z, 50), "p99": percentile(lat_z, 99),
                                  "frames": len(lat_z), "frames_recipe": lat_recipe,
                                  "scope": "pinned host frame -> estimate reading the inputs and "
                                           "writing the per-cluster results in pinned host memory "
                                           "through their device mapping (no copies)"}
                                 if lat_z else None),
        "latency_pipelined_ms": ({
            "parts": {str(P): {"p50": percentile(v[0], 50), "p99": percentile(v[0], 99),
                               "bitwise_equal_to_whole_frame": v[1]} for P, v in lat_p.items()},
            "frames": len(lat), "frames_recipe": lat_recipe,
            "scope": "pinned host frame -> rv_estimate_velocity_pipelined: P parts cut at "
                     "cluster boundaries, the H2D copy of part j+1 on a copy stream overlapping "
                     "the estimate of part j -> per-cluster results written into pinned host "
                     "memory through its device mapping"} if lat_p else None),
        "step_ms": {"median": percentile(step_times, 50), "p99": percentile(step_times, 99),
                    "scope": "single steps, a second pass with an event between steps"},
        "stage_ms": dict(zip(binding.STAGE_NAMES, stage_avg)),
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "roofline": {"bound": "alu", "kernel": kernel, "achieved": achieved_tflops,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": profiled_traffic(name) if kernel == "score_kernel" else None,
                     "algorithmic_flop_per_launch": FLOP_PER_EVAL * evals,
                     "kernel_ms": score_ms, "kernel_events_on_steps": n_calls,
                     "valu_issue": profiled_valu_issue(name) if kernel == "score_kernel" else None},
        "stage_roofline": None if small_path else {
            st: {"bound": "hbm", "achieved": b / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBPS,
                 "unit": "GB/s", "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                 "algorithmic_bytes_per_launch": b, "kernel_ms": ms}
            for st, b, ms in (
                ("prep", PREP_BYTES_PER_POINT * N, stage_avg[binding.STAGE_NAMES.index("prep")]),
                ("refit", REFIT_BYTES_PER_POINT * N + REFIT_BYTES_PER_CLUSTER * K,
                 stage_avg[binding.STAGE_NAMES.index("refit")]))},
        "cpu_baseline": cpu,
    }
    return line


def default_extras(args, torch, binding, synth, dev) -> dict:
    """The other workloads' headline figures for the default (dense) line, so
    that one run reports them all: the small frame (the paper's Table I shape:
    per-step time and latency over 1000 distinct frames), the 256-frame batched
    form (one graph replay per step, and the per-frame form on the same
    frames, in the float32 form and in the FP16 residual form), the precision
    stress shape (the FP16 residual form against the float32 form, errors
    against the FP64 oracle on a sample of clusters), and the served form at
    64 radars x 20 frames/s (latency and saturated throughput of the
    served and the per-frame forms; the served form in float32, then in the FP16
    residual form)."""
    import copy

    out = {}
    a = copy.copy(args)
    a.no_cpu_baseline = True
    a.steps = max(20, min(args.steps, 200))
    small = frame_bench(a, torch, binding, synth, dev, "small")
    out["small_frame"] = {
        "workload": WORKLOAD_TEXT["small"], "ms_per_step": small["ms_per_step"],
        "clusters_per_s": small["clusters_per_s"], "evals_per_s": small["value"],
        "latency_ms": small["latency_ms"],
        "latency_zero_copy_ms": small["latency_zero_copy_ms"], "kernel": small["roofline"]["kernel"],
        "kernel_ms": small["roofline"]["kernel_ms"]}
    a = copy.copy(args)
    a.no_cpu_baseline = True
    a.workload = "batched"
    a.steps = max(5, min(args.steps, 20))
    a.warmup = 3
    b = batch_bench(a, torch, binding, synth, dev)
    out["batched"] = {
        "workload": WORKLOAD_TEXT["batched"], "ms_per_step": b["ms_per_step"],
        "clusters_per_s": b["clusters_per_s"], "evals_per_s": b["value"],
        "frames": b["config"]["frames"], "clusters": b["config"]["clusters"],
        "frac_fp32_valu_peak": b["frac_fp32_valu_peak"], "stage_ms": b["stage_ms"],
        "per_frame_form": b["per_frame_form"],
        "batched_over_per_frame_clusters_per_s":
            b["clusters_per_s"] / b["per_frame_form"]["clusters_per_s"]}
    a.fp16_min_points = 1024
    bf = batch_bench(a, torch, binding, synth, dev)
    out["batched_fp16"] = {
        "workload": WORKLOAD_TEXT["batched"] + "; FP16 residual form for clusters of at least "
                    "1024 points (outputs bitwise the float32 form's)",
        "fp16_min_points": 1024, "ms_per_step": bf["ms_per_step"],
        "clusters_per_s": bf["clusters_per_s"], "evals_per_s": bf["value"],
        "stage_ms": bf["stage_ms"], "per_frame_form": bf["per_frame_form"],
        "over_per_frame_clusters_per_s":
            bf["clusters_per_s"] / bf["per_frame_form"]["clusters_per_s"]}
    a = copy.copy(args)
    a.no_cpu_baseline = True
    a.workload = "precision"
    a.steps, a.warmup, a.fp16_min_points = 3, 1, 0
    pr = precision_bench(a, torch, binding, synth, dev, oracle_budget_s=4.0)
    out["precision"] = {k: pr[k] for k in (
        "ms_per_step", "clusters_per_s", "fp32_form", "fp16_over_fp32_time",
        "outputs_bitwise_equal_to_fp32_form", "fp16_recount", "oracle_error", "stage_ms",
        "roofline")}
    out["precision"].update({"workload": WORKLOAD_TEXT["precision"], "evals_per_s": pr["value"],
                             "fp16_min_points": pr["config"]["fp16_min_points"]})
    a = copy.copy(args)
    a.no_cpu_baseline = True
    a.workload = "served"
    a.duration = args.extras_duration
    a.fp16_min_points = 0
    sv = served_bench(a, torch, binding, synth, dev, extra_fp16=256, zero_copy=True)
    pf = sv["per_frame_form"]
    out["served"] = {
        "workload": WORKLOAD_TEXT["served"] + "; the served form in float32 and in the FP16 "
                    "residual form for clusters of at least 256 points (outputs bitwise equal), "
                    "the per-frame form in float32, all on the same arrivals; then the served "
                    "and per-frame forms again with the frames in pinned host memory, queued "
                    "without a copy",
        "duration_s": a.duration, "arrivals": sv["config"]["frames"],
        "served_form": sv["served_form"], "served_fp16_form": sv["served_fp16_form"],
        "per_frame_form": pf,
        "served_zero_copy_form": sv["served_zero_copy_form"],
        "per_frame_zero_copy_form": sv["per_frame_zero_copy_form"],
        "served_over_per_frame_clusters_per_s":
            sv["served_form"]["saturated"]["clusters_per_s"] / pf["saturated"]["clusters_per_s"],
        "p99_served_over_per_frame":
            sv["served_form"]["latency_ms"]["p99"] / pf["latency_ms"]["p99"],
        "served_fp16_over_per_frame_clusters_per_s":
            sv["served_fp16_form"]["saturated"]["clusters_per_s"] / pf["saturated"]["clusters_per_s"],
        "p99_served_fp16_over_per_frame":
            sv["served_fp16_form"]["latency_ms"]["p99"] / pf["latency_ms"]["p99"],
        "p99_served_over_per_frame_zero_copy":
            sv["served_zero_copy_form"]["latency_ms"]["p99"]
            / sv["per_frame_zero_copy_form"]["latency_ms"]["p99"]}
    return out


def issue_rates_bench() -> int:
    """Runs the issue-rate probe built beside the library and prints its JSON."""
    import subprocess

    probe = os.path.join(ROOT, "paper_2012_12618_amd", "_lib", "issue_probe")
    if not os.path.exists(probe):
        print(f"bench.py: {probe} is missing (run __graft_entry__.build())", file=sys.stderr)
        return 1
    res = subprocess.run([probe], capture_output=True, text=True, timeout=120)
    if res.returncode != 0:
        print(res.stderr, file=sys.stderr)
        return res.returncode
    rec = json.loads(res.stdout)
    rec.update({"metric": "wave64 instruction issue rates", "workload": WORKLOAD_TEXT["issue-rates"]})
    print(json.dumps(rec), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--min-warmup-ms", type=float, default=100.0,
                    help="after the warm-up steps, more untimed steps until this much time has passed")
    ap.add_argument("--workload", default="dense", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--latency-frames", type=int, default=1000,
                    help="frames timed from pinned host memory to results in host memory")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads (0: every CPU this process may use, see oracle_threads)")
    ap.add_argument("--frames", type=int, default=0,
                    help="batched workload: number of frames (0: the workload's 256)")
    ap.add_argument("--submitters", type=int, default=4,
                    help="served workload: threads submitting frames (radars dealt round-robin)")
    ap.add_argument("--duration", type=float, default=5.0,
                    help="served workload: seconds of simulated arrivals in the timed run")
    ap.add_argument("--zero-copy-submit", action="store_true",
                    help="served workload: also run the served and per-frame forms with the "
                         "frames in pinned host memory, queued without a copy")
    ap.add_argument("--host-comparators", action="store_true",
                    help="paper-sweep: also time scikit-learn RANSACRegressor and numpy pinv per "
                         "cluster on the host (the paper's Table I/II comparators; context only)")
    ap.add_argument("--tuning", default="",
                    help="batched workload: JSON tuning table written by paper_2012_12618_amd.tuner "
                         "(default: the library's default setting)")
    ap.add_argument("--stage-sample-every", type=int, default=10,
                    help="frame workloads: record the library's per-kernel events on every n-th "
                         "timed step (1: every step)")
    ap.add_argument("--fp16-min-points", type=int, default=0,
                    help="batched and precision workloads: clusters of at least this many points "
                         "take the FP16 residual form (precision default: 1024; batched default: "
                         "none)")
    ap.add_argument("--no-extras", action="store_true",
                    help="dense workload: skip the small, batched and served figures that the "
                         "default line carries")
    ap.add_argument("--extras-duration", type=float, default=3.0,
                    help="seconds of simulated arrivals for the served figures of the default line")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (outside the timed "
                         "region), the reference kernel for scaling HBM byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this estimator runs on one GPU (asked for --gpus {args.gpus}); clusters are "
              "independent, so a multi-GPU deployment shards frames or clusters without any "
              "collective and its throughput is the sum of single-GPU runs.", file=sys.stderr)
        return 2
    if os.environ.get("WORLD_SIZE", "1") not in ("", "1"):
        print("bench.py: run on a single rank", file=sys.stderr)
        return 2

    if args.workload == "issue-rates":
        return issue_rates_bench()

    import numpy as np
    import torch

    from paper_2012_12618_amd import binding, synth

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    binding.load_library()
    dev = torch.device("cuda:0")
    name = args.workload
    if name == "served":
        print(json.dumps(served_bench(args, torch, binding, synth, dev,
                                      zero_copy=args.zero_copy_submit)), flush=True)
        return 0
    if name == "paper-sweep":
        return paper_sweep_bench(args, torch, binding, synth, dev)
    if name == "precision":
        line = precision_bench(args, torch, binding, synth, dev)
        print(json.dumps(line), flush=True)
        return 0 if line["outputs_bitwise_equal_to_fp32_form"] else 1
    if name not in FRAME_WORKLOADS:
        line = batch_bench(args, torch, binding, synth, dev)
    else:
        line = frame_bench(args, torch, binding, synth, dev, name)
        if name == "dense" and not args.no_extras:
            line.update(default_extras(args, torch, binding, synth, dev))
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
