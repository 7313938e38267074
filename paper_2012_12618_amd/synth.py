"""Seeded synthetic radar frames shaped like clustered automotive point clouds.

This module is the only code shared by the estimator's tests, the oracle's tests
and the benchmark.  It draws inputs; it holds none of the estimator's arithmetic
(no hypothesis draws, no residual tests, no fits).

Generative model (the paper's rigid-body velocity profile, Sec. 3.2, Eq. 6):
every point j of cluster i moves with the cluster's velocity (vx_i, vy_i), so its
radial Doppler velocity is vx_i*cos(theta_ij) + vy_i*sin(theta_ij).  The paper's
captured 78.6 GHz traffic data is not available; these frames stand in for it.

Recipe, per frame (numpy ``Generator(PCG64(seed))``, draws in this order):

1. cluster sizes n_i: ``uniform`` -> integers in [a, b]; ``loguniform`` ->
   floor(exp(U[ln a, ln(b + 1)))), clipped to [a, b];
2. true velocities (vx_i, vy_i) ~ U[-v_max, v_max]^2 (v_max = 30 m/s);
3. azimuth theta ~ U[-60 deg, 60 deg] per point, converted to radians in float64
   and rounded once to float32 (the stored value);
4. noise-free radial velocity from the stored float32 azimuth, plus N(0, sigma^2)
   noise, sigma = 0.05 m/s (sigma is the standard deviation);
5. outliers: exactly round(p_u * n_i) uniform outliers, v_d ~ U[-40, 40], and
   round(p_b * n_i) micro-Doppler band outliers, v_d = v_true(theta) +/- u*|v|
   with u ~ U[0.5, 2] and an equiprobable sign, at uniformly random positions
   inside the cluster;
6. v_d is computed in float64 and rounded once to float32.

Optional ``theta_spread_deg`` replaces step 3 with a narrow azimuth window of that
width around a random centre in [-60, 60] deg (ill-conditioned clusters).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

V_MAX = 30.0          # |vx|, |vy| bound of the true velocity, m/s
THETA_MAX_DEG = 60.0  # azimuth field of view, +/- degrees
UNIFORM_OUTLIER_SPAN = 40.0  # uniform outliers: v_d ~ U[-40, 40] m/s


@dataclasses.dataclass(frozen=True)
class FrameSpec:
    """Shape of one synthetic frame."""

    n_clusters: int
    size_kind: str            # "uniform" | "loguniform" | "fixed"
    size_lo: int
    size_hi: int
    p_uniform: float = 0.20   # fraction of uniform outliers per cluster
    p_band: float = 0.0       # fraction of micro-Doppler band outliers per cluster
    sigma: float = 0.05       # inlier noise standard deviation, m/s
    theta_spread_deg: float | None = None


@dataclasses.dataclass
class Frame:
    """One frame in CSR form: points of cluster k are [offsets[k], offsets[k+1])."""

    theta: np.ndarray      # float32 [N], azimuth in radians
    vd: np.ndarray         # float32 [N], radial Doppler velocity, m/s
    offsets: np.ndarray    # int32 [K+1]
    truth_vx: np.ndarray   # float64 [K]
    truth_vy: np.ndarray   # float64 [K]
    kind: np.ndarray       # int8 [N]: 0 inlier, 1 uniform outlier, 2 band outlier

    @property
    def n_clusters(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_points(self) -> int:
        return int(self.theta.shape[0])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))


# Workload shapes.  Each entry: (frame spec, hypotheses per cluster, tau in m/s).
# "small": 64 clusters of U{20..200} points, 20 % uniform outliers, 256 hypotheses.
# "dense": 4096 clusters, log-uniform sizes in [8, 4096], 30 % outliers split evenly
#          between uniform and micro-Doppler band outliers, 1024 hypotheses.
# "precision": 512 clusters of 65,536 points, 40 % micro-Doppler band outliers,
#          4096 hypotheses (the precision-stress shape of the FP16 residual form).
WORKLOADS = {
    "small": (FrameSpec(64, "uniform", 20, 200, p_uniform=0.20), 256, 0.15),
    "dense": (FrameSpec(4096, "loguniform", 8, 4096, p_uniform=0.15, p_band=0.15), 1024, 0.15),
    "precision": (FrameSpec(512, "fixed", 65536, 65536, p_uniform=0.0, p_band=0.40), 4096, 0.15),
}
# Data seed of each workload and the per-frame hypothesis seed convention:
# hypothesis seed = (workload number << 32) | frame index.
WORKLOAD_NUMBER = {"small": 1, "dense": 2, "batched": 3, "served": 4, "paper": 5, "precision": 6}


@dataclasses.dataclass(frozen=True)
class BatchSpec:
    """Many frames: cluster counts uniform in [clusters_lo, clusters_hi] per frame."""

    n_frames: int
    clusters_lo: int
    clusters_hi: int
    frame: FrameSpec          # its n_clusters is replaced per frame


# "batched": 256 frames of U{100..1500} clusters, log-uniform [8, 2048] points,
#            20 % uniform outliers, 512 hypotheses.
# "served":  frames of U{200..1200} clusters, log-uniform [8, 1024] points, 25 %
#            uniform outliers, 512 hypotheses (the frames of the request loop).
BATCH_WORKLOADS = {
    "batched": (BatchSpec(256, 100, 1500, FrameSpec(0, "loguniform", 8, 2048, p_uniform=0.20)), 512, 0.15),
    "served": (BatchSpec(64, 200, 1200, FrameSpec(0, "loguniform", 8, 1024, p_uniform=0.25)), 512, 0.15),
}


def ransac_seed(workload: str, frame_index: int = 0) -> int:
    return (WORKLOAD_NUMBER[workload] << 32) | (frame_index & 0xFFFFFFFF)


def _sizes(rng: np.random.Generator, spec: FrameSpec) -> np.ndarray:
    k = spec.n_clusters
    if spec.size_kind == "uniform":
        return rng.integers(spec.size_lo, spec.size_hi + 1, size=k).astype(np.int64)
    if spec.size_kind == "loguniform":
        x = rng.uniform(math.log(spec.size_lo), math.log(spec.size_hi + 1), size=k)
        return np.clip(np.floor(np.exp(x)), spec.size_lo, spec.size_hi).astype(np.int64)
    if spec.size_kind == "fixed":
        return np.full(k, spec.size_lo, dtype=np.int64)
    raise ValueError(f"unknown size kind {spec.size_kind!r}")


def make_frame(spec: FrameSpec, seed: int) -> Frame:
    """Draw one frame (see the module docstring for the recipe)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = _sizes(rng, spec)
    k = spec.n_clusters
    n = int(sizes.sum())
    offsets = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    if offsets[-1] > np.iinfo(np.int32).max:
        raise ValueError("frame too large for int32 offsets")
    cid = np.repeat(np.arange(k), sizes)

    tvx = rng.uniform(-V_MAX, V_MAX, size=k)
    tvy = rng.uniform(-V_MAX, V_MAX, size=k)

    if spec.theta_spread_deg is None:
        theta_deg = rng.uniform(-THETA_MAX_DEG, THETA_MAX_DEG, size=n)
    else:
        half = 0.5 * spec.theta_spread_deg
        centre = rng.uniform(-THETA_MAX_DEG + half, THETA_MAX_DEG - half, size=k)
        theta_deg = centre[cid] + rng.uniform(-half, half, size=n)
    theta = np.deg2rad(theta_deg).astype(np.float32)
    th64 = theta.astype(np.float64)

    v_true = tvx[cid] * np.cos(th64) + tvy[cid] * np.sin(th64)
    vd = v_true + rng.normal(0.0, spec.sigma, size=n)

    # Exact outlier counts per cluster at uniformly random positions: rank the
    # points of each cluster by a random key; the lowest ranks become outliers.
    n_u = np.rint(spec.p_uniform * sizes).astype(np.int64)
    n_b = np.rint(spec.p_band * sizes).astype(np.int64)
    key = rng.random(size=n)
    order = np.lexsort((key, cid))
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n) - offsets[cid[order]]
    kind = np.zeros(n, dtype=np.int8)
    kind[rank < n_u[cid]] = 1
    kind[(rank >= n_u[cid]) & (rank < (n_u + n_b)[cid])] = 2

    u_out = rng.uniform(-UNIFORM_OUTLIER_SPAN, UNIFORM_OUTLIER_SPAN, size=n)
    speed = np.hypot(tvx, tvy)[cid]
    band = v_true + rng.choice([-1.0, 1.0], size=n) * rng.uniform(0.5, 2.0, size=n) * speed
    vd = np.where(kind == 1, u_out, vd)
    vd = np.where(kind == 2, band, vd)

    return Frame(
        theta=theta,
        vd=vd.astype(np.float32),
        offsets=offsets.astype(np.int32),
        truth_vx=tvx,
        truth_vy=tvy,
        kind=kind,
    )


def make_workload(name: str, seed: int | None = None) -> tuple[Frame, int, float]:
    """Frame, hypotheses per cluster and tau of a named workload."""
    spec, n_hyp, tau = WORKLOADS[name]
    return make_frame(spec, WORKLOAD_NUMBER[name] if seed is None else seed), n_hyp, tau


def concat_frames(frames: list[Frame]) -> Frame:
    """Concatenate frames into one CSR frame (cluster order preserved)."""
    offs = [np.zeros(1, dtype=np.int64)]
    base = 0
    for f in frames:
        offs.append(f.offsets[1:].astype(np.int64) + base)
        base += f.n_points
    return Frame(
        theta=np.concatenate([f.theta for f in frames]),
        vd=np.concatenate([f.vd for f in frames]),
        offsets=np.concatenate(offs).astype(np.int32),
        truth_vx=np.concatenate([f.truth_vx for f in frames]),
        truth_vy=np.concatenate([f.truth_vy for f in frames]),
        kind=np.concatenate([f.kind for f in frames]),
    )


def evals_per_frame(offsets: np.ndarray, n_hyp: int) -> int:
    """Nominal hypothesis-point evaluations: sum of n_hyp * n_i over clusters with n_i >= 2."""
    sizes = np.diff(np.asarray(offsets, dtype=np.int64))
    return int(n_hyp * sizes[sizes >= 2].sum())


@dataclasses.dataclass
class Batch:
    """Frames concatenated into one CSR, with each frame's cluster range and seed."""

    frame: Frame                 # all frames' clusters, in frame order
    frame_offsets: np.ndarray    # int32 [F+1]: frame f owns clusters [fo[f], fo[f+1])
    seeds: np.ndarray            # uint64 [F]: hypothesis seed of each frame

    @property
    def n_frames(self) -> int:
        return int(self.frame_offsets.shape[0] - 1)

    def frame_slice(self, f: int) -> Frame:
        """Frame f alone (its clusters re-based to start at point 0)."""
        c0, c1 = int(self.frame_offsets[f]), int(self.frame_offsets[f + 1])
        p0, p1 = int(self.frame.offsets[c0]), int(self.frame.offsets[c1])
        return Frame(theta=self.frame.theta[p0:p1], vd=self.frame.vd[p0:p1],
                     offsets=(self.frame.offsets[c0:c1 + 1] - p0).astype(np.int32),
                     truth_vx=self.frame.truth_vx[c0:c1], truth_vy=self.frame.truth_vy[c0:c1],
                     kind=self.frame.kind[p0:p1])


def frame_seed(workload: str, frame_index: int) -> int:
    return ransac_seed(workload, frame_index)


def make_batch(spec: BatchSpec, seed: int, workload: str = "batched", n_frames: int | None = None) -> Batch:
    """Frames f = 0..F-1: cluster count drawn from PCG64(seed), frame data from
    make_frame with data seed (seed << 20) + f, hypothesis seed frame_seed(workload, f)."""
    F = spec.n_frames if n_frames is None else n_frames
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = rng.integers(spec.clusters_lo, spec.clusters_hi + 1, size=F)
    frames = [make_frame(dataclasses.replace(spec.frame, n_clusters=int(c)), (seed << 20) + f)
              for f, c in enumerate(counts)]
    fo = np.zeros(F + 1, dtype=np.int64)
    np.cumsum(counts, out=fo[1:])
    seeds = np.array([frame_seed(workload, f) for f in range(F)], dtype=np.uint64)
    return Batch(frame=concat_frames(frames), frame_offsets=fo.astype(np.int32), seeds=seeds)


def make_batch_workload(name: str, n_frames: int | None = None) -> tuple[Batch, int, float]:
    spec, n_hyp, tau = BATCH_WORKLOADS[name]
    return make_batch(spec, WORKLOAD_NUMBER[name], workload=name, n_frames=n_frames), n_hyp, tau


# The paper's timing tables (Table I: RANSAC, Table II: least squares) sweep
# {8, 16, 32, 64} clusters x {100, 150} points per cluster.
TABLE_SHAPES = [(c, p) for c in (8, 16, 32, 64) for p in (100, 150)]


def table_frame(n_clusters: int, points: int, seed: int | None = None) -> Frame:
    """A frame of the Table I/II shape: fixed cluster size, 20 % uniform outliers."""
    spec = FrameSpec(n_clusters=n_clusters, size_kind="fixed", size_lo=points, size_hi=points,
                     p_uniform=0.20)
    return make_frame(spec, (5 << 20) + n_clusters * 1000 + points if seed is None else seed)
