"""Autotuner for the batched form.

Two launch parameters of ``rv_estimate_velocity_batch`` change only its speed,
never a result bit:

* ``rows_max[b]``: register rows of 64 points a wave holds per pass over a
  cluster of size bucket b (bucket 0: n < 64; bucket b >= 1: 32*2^b <= n <
  64*2^b; the last bucket: everything larger).  More rows mean fewer passes,
  so fewer re-reads of the hypotheses from LDS; fewer rows mean less work
  wasted in the last, partial pass of a cluster.
* ``blocks_per_cu``: workgroups of the persistent scoring grid per compute
  unit (0: as many as fit).
* ``lanes_max_points``: the orientation of the scoring loop by cluster size.
  Clusters of at most this many points score with lanes = hypotheses (each
  lane counts its own inliers over the cluster's points, read from LDS as
  broadcasts: 64 hypotheses per wave instruction whatever the cluster size);
  larger ones with lanes = points (each wave instruction tests one
  hypothesis against 64 points, and the last row of a cluster leaves lanes
  idle).  This is the hypotheses-per-wave knob: 64 hypotheses per
  instruction below the threshold, one above.

The tuner times whole batched calls on the caller's own inputs (coordinate
descent: one bucket at a time, then the grid), keeps the fastest setting per
coordinate, then times the winner and the default alternately and keeps the
winner only when it is faster by more than ``min_gain`` (timings drift by a
few per cent over a run).  The table can be saved as JSON keyed by device name
and n_hyp.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import binding

ROW_CANDIDATES = (4, 8, 12, 16)
GRID_CANDIDATES = (0, 1, 2, 4)
LANES_CANDIDATES = (0, 32, 64, 96, 128, 192, 256)


def size_bucket(n: int) -> int:
    """Bucket of a cluster of n points (the kernel's own rule)."""
    b = 0
    while b < binding.RV_TUNE_BUCKETS - 1 and n >= (64 << b):
        b += 1
    return b


def buckets_in_use(offsets_host) -> list[int]:
    """Buckets where rows_max can matter: clusters longer than the smallest candidate tile."""
    import numpy as np

    sizes = np.diff(np.asarray(offsets_host, dtype=np.int64))
    used = set()
    for n in np.unique(sizes):
        if n > 64 * min(ROW_CANDIDATES):
            used.add(size_bucket(int(n)))
    return sorted(used)


def _time_call(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return statistics.median(times)


def autotune(theta, vd, offsets, frame_offsets, seeds, n_hyp: int, tau: float, *,
             offsets_host=None, reps: int = 3, rows=ROW_CANDIDATES, grids=GRID_CANDIDATES,
             lanes=LANES_CANDIDATES, min_gain: float = 0.01,
             log=None) -> tuple[binding.RVTuning, dict]:
    """Pick lanes_max_points, rows_max per bucket and blocks_per_cu for this
    batch; returns (tuning, report)."""
    n_frames = int(frame_offsets.numel()) - 1
    out = binding.allocate_batch_outputs(n_frames, int(offsets.numel()) - 1, int(theta.numel()),
                                         n_hyp, theta.device)
    if offsets_host is None:
        offsets_host = offsets.cpu().numpy()
    best = binding.rv_tuning_default()

    def run(t):
        binding.rv_estimate_velocity_batch(theta, vd, offsets, frame_offsets, seeds, n_hyp, tau,
                                           tuning=t, out=out)

    # Warm-up of at least 200 ms: the chip's clock rises over the first tens of
    # milliseconds of sustained work, which would favour whatever is timed later.
    import time

    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.2:
        run(best)
        torch.cuda.synchronize()
    best_ms = _time_call(lambda: run(best), reps)
    trials = [{"tuning": best.to_dict(), "ms": best_ms}]
    for m in lanes:
        if m == best.lanes_max_points:
            continue
        cand = binding.RVTuning.from_dict(best.to_dict())
        cand.lanes_max_points = m
        ms = _time_call(lambda: run(cand), reps)
        trials.append({"tuning": cand.to_dict(), "ms": ms})
        if log:
            log(f"lanes_max_points {m}: {ms:.3f} ms (best {best_ms:.3f})")
        if ms < best_ms:
            best, best_ms = cand, ms
    for b in buckets_in_use(offsets_host):
        for r in rows:
            if r == best.rows_max[b]:
                continue
            cand = binding.RVTuning.from_dict(best.to_dict())
            cand.rows_max[b] = r
            ms = _time_call(lambda: run(cand), reps)
            trials.append({"tuning": cand.to_dict(), "ms": ms})
            if log:
                log(f"bucket {b} rows {r}: {ms:.3f} ms (best {best_ms:.3f})")
            if ms < best_ms:
                best, best_ms = cand, ms
    for gsz in grids:
        if gsz == best.blocks_per_cu:
            continue
        cand = binding.RVTuning.from_dict(best.to_dict())
        cand.blocks_per_cu = gsz
        ms = _time_call(lambda: run(cand), reps)
        trials.append({"tuning": cand.to_dict(), "ms": ms})
        if log:
            log(f"blocks_per_cu {gsz}: {ms:.3f} ms (best {best_ms:.3f})")
        if ms < best_ms:
            best, best_ms = cand, ms
    # Drift check: the winner and the default, timed alternately; the winner is
    # kept only if it is faster by more than min_gain.
    default = binding.rv_tuning_default()
    a_ms, d_ms = [], []
    for _ in range(3):
        a_ms.append(_time_call(lambda: run(best), reps))
        d_ms.append(_time_call(lambda: run(default), reps))
    a, d = statistics.median(a_ms), statistics.median(d_ms)
    kept = a < d * (1.0 - min_gain)
    if log:
        log(f"winner {a:.3f} ms vs default {d:.3f} ms: {'kept' if kept else 'default kept'}")
    if not kept:
        best, a = default, d
    return best, {"best": best.to_dict(), "best_ms": a, "default_ms": d, "trials": trials}


def table_key(device_name: str, n_hyp: int) -> str:
    return f"{device_name}|H={int(n_hyp)}"


def save(path: str, device_name: str, n_hyp: int, tuning: binding.RVTuning) -> None:
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    table[table_key(device_name, n_hyp)] = tuning.to_dict()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load(path: str, device_name: str, n_hyp: int) -> binding.RVTuning | None:
    """The saved tuning for this device and n_hyp, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    d = table.get(table_key(device_name, n_hyp))
    return None if d is None else binding.RVTuning.from_dict(d)


def main(argv=None) -> int:
    """Tune on one of the synthetic batched workloads and print the report as
    JSON: ``python -m paper_2012_12618_amd.tuner --workload batched [--frames N]
    [--out table.json]``."""
    import argparse

    from . import synth

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--workload", default="batched", choices=("batched", "served"))
    ap.add_argument("--frames", type=int, default=0, help="frames (0: the workload's own count)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default="", help="JSON table to add the winner to")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("tuner: no GPU visible")
        return 1
    batch, n_hyp, tau = synth.make_batch_workload(args.workload, n_frames=args.frames or None)
    fr = batch.frame
    dev = torch.device("cuda:0")
    t = torch.from_numpy(fr.theta).to(dev)
    v = torch.from_numpy(fr.vd).to(dev)
    off = torch.from_numpy(fr.offsets).to(dev)
    fo = torch.from_numpy(batch.frame_offsets).to(dev)
    seeds = torch.from_numpy(batch.seeds.view("int64")).to(dev)
    best, report = autotune(t, v, off, fo, seeds, n_hyp, tau, offsets_host=fr.offsets,
                            reps=args.reps, log=lambda m: print(f"[tuner] {m}", flush=True))
    if args.out:
        save(args.out, torch.cuda.get_device_name(dev), n_hyp, best)
    report.update({"workload": args.workload, "frames": batch.n_frames, "n_hyp": n_hyp,
                   "device": torch.cuda.get_device_name(dev)})
    print(json.dumps(report))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
