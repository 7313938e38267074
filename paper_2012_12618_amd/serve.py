"""Served form: simulated radars sending frames to the frame server.

``RVServer`` (the C server of include/rv.h) does the serving: the request
queue, admission by the device-memory budget, continuous batching over launch
slots and the copies.  This module only drives it the way a deployment would:
``arrival_schedule`` draws when each radar's frames arrive, ``run_traffic``
submits them at those times from one thread while another collects results,
and the report gives p50/p99 frame latency and throughput.

Arrivals: every radar sends frames as a Poisson process of rate ``fps``
(exponential gaps with mean 1/fps), starting at a uniform phase in [0, 1/fps).
"""
from __future__ import annotations

import dataclasses
import gc
import threading
import time

import numpy as np

from . import binding


@dataclasses.dataclass
class Arrival:
    t: float        # seconds after the start of the run
    radar: int
    index: int      # arrival index over all radars, in time order


def arrival_schedule(n_radars: int, fps: float, duration_s: float, seed: int) -> list[Arrival]:
    """Arrivals of n_radars Poisson(fps) sources over [0, duration_s), in time order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    events = []
    for r in range(n_radars):
        t = rng.uniform(0.0, 1.0 / fps)
        while t < duration_s:
            events.append((t, r))
            t += rng.exponential(1.0 / fps)
    events.sort()
    return [Arrival(t=t, radar=r, index=i) for i, (t, r) in enumerate(events)]


def percentile(xs, q: float) -> float:
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    a = np.sort(np.asarray(xs, dtype=np.float64))
    if a.size == 0:
        return float("nan")
    k = int(np.ceil(q / 100.0 * a.size)) - 1
    return float(a[min(max(k, 0), a.size - 1)])


@dataclasses.dataclass
class TrafficReport:
    frames: int
    clusters: int
    evals: int
    wall_s: float                 # first submit to last result
    latency_ms: list[float]       # per frame: arrival -> results in host memory
    server_latency_ms: list[float]  # per frame: submitted -> results in host memory (server clock)
    batch_frames: list[int]
    busy_retries: int
    late_submits: int             # submits that started more than 1 ms after their arrival time
    stats: dict

    def summary(self) -> dict:
        return {
            "frames": self.frames, "clusters": self.clusters, "wall_s": self.wall_s,
            "frames_per_s": self.frames / self.wall_s, "clusters_per_s": self.clusters / self.wall_s,
            "evals_per_s": self.evals / self.wall_s,
            "latency_ms": {"p50": percentile(self.latency_ms, 50),
                           "p99": percentile(self.latency_ms, 99),
                           "max": max(self.latency_ms)},
            "server_latency_ms": {"p50": percentile(self.server_latency_ms, 50),
                                  "p99": percentile(self.server_latency_ms, 99),
                                  "max": max(self.server_latency_ms)},
            "mean_batch_frames": float(np.mean(self.batch_frames)),
            "busy_retries": self.busy_retries, "late_submits": self.late_submits,
            "server": self.stats,
        }


def run_traffic(server: binding.RVServer, frames, schedule: list[Arrival], seed_of,
                n_hyp: int, *, paced: bool = True, keep_results: bool = False, submitters: int = 1,
                pinned_frames=None):
    """Submit frames[a.radar] at each arrival's time (or as fast as the server
    takes them when paced is False) and collect every result.

    ``submitters`` threads share the radars (radar r goes to thread r mod
    submitters), each submitting its radars' arrivals in time order, as one
    feeder per group of sensors would.  A frame's latency is the time from its
    arrival to the return of its submit (the copy into pinned memory, plus any
    lateness of the submitting thread) plus the server's time from that copy to
    results in host memory.  seed_of(arrival) gives the frame's hypothesis seed.
    With ``pinned_frames`` (per frame, (theta, vd, offsets) pinned host tensors
    of the same values) the frames are queued without a copy
    (RVServer.submit_pinned), as from a sensor driver that fills pinned buffers.
    Returns (report, results) where results maps arrival index -> result dict
    when keep_results.
    """
    evals_of = [int(n_hyp * np.diff(f.offsets.astype(np.int64))[np.diff(f.offsets) >= 2].sum())
                for f in frames]
    tickets: list[tuple[int, Arrival, float]] = []
    cond = threading.Condition()
    running = [submitters]
    results = {}
    lat, slat, bsz = [], [], []
    counters = {"busy": 0, "late": 0}
    errors = []

    def submitter(t0, mine):
        for a in mine:
            if paced:
                delay = t0 + a.t - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                elif delay < -1e-3:
                    counters["late"] += 1
            f = frames[a.radar]
            start = time.perf_counter()
            while True:
                try:
                    if pinned_frames is None:
                        tk = server.submit(f.theta, f.vd, f.offsets, seed_of(a))
                    else:
                        tk = server.submit_pinned(*pinned_frames[a.radar], seed_of(a))
                    break
                except binding.RVError as e:
                    if e.code != binding.RV_ERR_BUSY:
                        errors.append(e)
                        break
                    counters["busy"] += 1
                    time.sleep(50e-6)
            if errors:
                break
            arrival = (t0 + a.t) if paced else start
            with cond:
                tickets.append((tk, a, time.perf_counter() - arrival))
                cond.notify()
        with cond:
            running[0] -= 1
            cond.notify()

    # Python's cyclic garbage collector stays off while the traffic runs: a full
    # collection holds every thread of the process (the submitters included)
    # for tens of milliseconds, which would count against the frame in flight.
    gc_was_enabled = gc.isenabled()
    gc.disable()
    try:
        t0 = time.perf_counter() + 0.01
        parts = [[a for a in schedule if a.radar % submitters == i] for i in range(submitters)]
        threads = [threading.Thread(target=submitter, args=(t0, part), daemon=True)
                   for part in parts]
        for th in threads:
            th.start()
        got = 0
        t_last = t0
        while True:
            with cond:
                while got >= len(tickets) and running[0] > 0:
                    cond.wait()
                if got >= len(tickets):
                    break
                tk, a, pre = tickets[got]
            r = server.result(tk)
            t_last = time.perf_counter()
            tm = r["times"]
            server_ms = (tm["done_ns"] - tm["submitted_ns"]) * 1e-6
            lat.append(pre * 1e3 + server_ms)
            slat.append(server_ms)
            bsz.append(tm["batch_frames"])
            if keep_results:
                results[a.index] = r
            got += 1
        for th in threads:
            th.join()
    finally:
        if gc_was_enabled:
            gc.enable()
    if errors:
        raise errors[0]
    clusters = sum(frames[a.radar].n_clusters for a in schedule)
    evals = sum(evals_of[a.radar] for a in schedule)
    rep = TrafficReport(frames=len(schedule), clusters=clusters, evals=evals,
                        wall_s=max(t_last - t0, 1e-9), latency_ms=lat, server_latency_ms=slat,
                        batch_frames=bsz, busy_retries=counters["busy"],
                        late_submits=counters["late"], stats=server.stats())
    return rep, results
