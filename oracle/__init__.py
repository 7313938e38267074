"""FP64 CPU oracle of the per-cluster velocity and heading estimator.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only code allowed to import this package.  The
estimator's product path never does, and this package imports nothing from it.

The arithmetic lives in ``rv_oracle.c`` (plain C, FP64, compiled with
``-ffp-contract=off``); this module only marshals numpy arrays.  Each step
cites the paper passage it follows in the C source: Sec. 3.1 / Alg. 1 for the
RANSAC trials, Sec. 3.2 / Eq. 7 / Alg. 2 for the least-squares refit and Eq. 8
for the heading.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rv_oracle.c")
_SRC_PAPER = os.path.join(_HERE, "rv_oracle_paper.c")
# RV_ORACLE_LIB names another build of the same sources (the sanitizer check
# in check_sanitizers.sh loads an ASan/UBSan build this way).
_LIB = os.environ.get("RV_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

# Per-cluster status codes (same meaning as the estimator's).
CLUSTER_OK = 0
CLUSTER_TOO_FEW_POINTS = 1
CLUSTER_ALL_DEGENERATE = 2
CLUSTER_SINGULAR_REFIT = 3
CLUSTER_BAD_OFFSETS = 4

NEAR_TAU_WINDOW = 1e-5          # m/s, half-width of the "near tau" flag
FP32_BAND_REL = 1.5 * 2.0**-24  # relative band covering a float32 residual evaluation


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no FP contraction, no fast-math)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_PAPER))
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= newest:
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = [
        "gcc", "-O3", "-march=x86-64-v3", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
        "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, _SRC_PAPER, "-lm", "-lpthread",
    ]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, u64, f32, f64 = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                               ctypes.c_float, ctypes.c_double)
    lib.oracle_estimate_velocity.restype = ctypes.c_int
    lib.oracle_estimate_velocity.argtypes = [
        P, P, P, i64, i64, i32, f32, u64, P, i64, f64, f64, f64,
        P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, ctypes.c_int,
    ]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_philox4x32_10.argtypes = [P, P, P]
    lib.oracle_map_pair.restype = None
    lib.oracle_map_pair.argtypes = [ctypes.c_uint32, ctypes.c_uint32, i64, P, P]
    lib.oracle_draw_pair.restype = None
    lib.oracle_draw_pair.argtypes = [u64, ctypes.c_uint32, ctypes.c_uint32, i64, P, P]
    lib.oracle_fit_hypothesis.restype = ctypes.c_int
    lib.oracle_fit_hypothesis.argtypes = [P, P, P, i64, i64, f32, u64, i64, i64, f64,
                                          P, P, P, P, P, P, P, P]
    lib.oracle_refit_mask.restype = ctypes.c_int
    lib.oracle_refit_mask.argtypes = [P, P, P, i64, P, P, P, P, P]
    lib.oracle_all_pairs_best.restype = i32
    lib.oracle_all_pairs_best.argtypes = [P, P, i32, f32, P, P]
    lib.oracle_estimate_velocity_paper.restype = ctypes.c_int
    lib.oracle_estimate_velocity_paper.argtypes = [P, P, P, i64, i64, i32, u64,
                                                   P, P, P, P, P, P, P, P, P, P]
    lib.oracle_median.restype = f64
    lib.oracle_median.argtypes = [P, i64]
    lib.oracle_paper_line_distance.restype = f64
    lib.oracle_paper_line_distance.argtypes = [f64] * 6
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block: ctr (4 x u32), key (2 x u32) -> 4 x u32."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def map_pair(u0: int, u1: int, n: int) -> tuple[int, int]:
    lib = _load()
    i = ctypes.c_int64()
    j = ctypes.c_int64()
    lib.oracle_map_pair(u0 & 0xFFFFFFFF, u1 & 0xFFFFFFFF, n, ctypes.byref(i), ctypes.byref(j))
    return i.value, j.value


def draw_pair(seed: int, h: int, k: int, n: int) -> tuple[int, int]:
    lib = _load()
    i = ctypes.c_int64()
    j = ctypes.c_int64()
    lib.oracle_draw_pair(seed & 0xFFFFFFFFFFFFFFFF, h, k, n, ctypes.byref(i), ctypes.byref(j))
    return i.value, j.value


@dataclass
class OracleResult:
    vx: np.ndarray          # float64 [R]
    vy: np.ndarray          # float64 [R]
    heading: np.ndarray     # float64 [R]
    n_inliers: np.ndarray   # int32 [R]
    status: np.ndarray      # uint8 [R]
    n_near_tau: np.ndarray  # int32 [R]
    best_hyp: np.ndarray    # int32 [R]
    inlier_mask: np.ndarray | None = None   # uint8 [N]
    hyp_valid: np.ndarray | None = None     # uint8 [R, H]
    hyp_i: np.ndarray | None = None         # int32 [R, H]
    hyp_j: np.ndarray | None = None
    hyp_vx: np.ndarray | None = None        # float64 [R, H]
    hyp_vy: np.ndarray | None = None
    hyp_count: np.ndarray | None = None     # int32 [R, H]
    hyp_count_lo: np.ndarray | None = None
    hyp_count_hi: np.ndarray | None = None


def estimate_velocity(theta, vd, offsets, n_hyp: int, tau: float, seed: int, *,
                      cluster_ids=None, debug: bool = False, want_mask: bool = True,
                      near_window: float = NEAR_TAU_WINDOW, band_abs: float = NEAR_TAU_WINDOW,
                      band_rel: float = FP32_BAND_REL, n_threads: int | None = None) -> OracleResult:
    """Run the oracle over a CSR frame held in host (numpy) memory.

    With ``cluster_ids`` only those clusters are computed (their hypothesis
    streams still use their index in the frame); results follow the list order.
    ``debug`` adds the per-hypothesis arrays, with count_lo / count_hi bands of
    half-width max(band_abs, band_rel * magnitude) (see ``rv_oracle.c``).
    """
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float32)
    v = np.ascontiguousarray(vd, dtype=np.float32)
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    n_clusters = off.shape[0] - 1
    n_points = th.shape[0]
    if v.shape[0] != n_points:
        raise ValueError("theta and vd differ in length")
    ids = None if cluster_ids is None else np.ascontiguousarray(cluster_ids, dtype=np.int64)
    R = n_clusters if ids is None else ids.shape[0]
    H = int(n_hyp)
    out = OracleResult(
        vx=np.empty(R), vy=np.empty(R), heading=np.empty(R),
        n_inliers=np.empty(R, dtype=np.int32), status=np.empty(R, dtype=np.uint8),
        n_near_tau=np.empty(R, dtype=np.int32), best_hyp=np.empty(R, dtype=np.int32),
    )
    if want_mask:
        out.inlier_mask = np.zeros(n_points, dtype=np.uint8)
    if debug:
        out.hyp_valid = np.empty((R, H), dtype=np.uint8)
        out.hyp_i = np.empty((R, H), dtype=np.int32)
        out.hyp_j = np.empty((R, H), dtype=np.int32)
        out.hyp_vx = np.empty((R, H))
        out.hyp_vy = np.empty((R, H))
        out.hyp_count = np.empty((R, H), dtype=np.int32)
        out.hyp_count_lo = np.empty((R, H), dtype=np.int32)
        out.hyp_count_hi = np.empty((R, H), dtype=np.int32)
    if n_threads is None:
        n_threads = min(os.cpu_count() or 1, 16)
    rc = lib.oracle_estimate_velocity(
        _ptr(th), _ptr(v), _ptr(off), n_clusters, n_points, H, float(tau),
        int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(ids), 0 if ids is None else R,
        near_window, band_abs, band_rel,
        _ptr(out.vx), _ptr(out.vy), _ptr(out.heading), _ptr(out.n_inliers), _ptr(out.status),
        _ptr(out.n_near_tau), _ptr(out.best_hyp), _ptr(out.inlier_mask),
        _ptr(out.hyp_valid), _ptr(out.hyp_i), _ptr(out.hyp_j), _ptr(out.hyp_vx), _ptr(out.hyp_vy),
        _ptr(out.hyp_count), _ptr(out.hyp_count_lo), _ptr(out.hyp_count_hi),
        int(n_threads),
    )
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


@dataclass
class HypothesisFit:
    vx: float
    vy: float
    heading: float
    n_inliers: int
    n_near_tau: int
    status: int
    mask: np.ndarray       # uint8 [n_k], inlier set of the cluster's points
    near_mask: np.ndarray  # uint8 [n_k], points within near_window of tau


def fit_hypothesis(theta, vd, offsets, tau: float, seed: int, k: int, h: int, *,
                   near_window: float = NEAR_TAU_WINDOW) -> HypothesisFit | None:
    """Refit of cluster k on the inliers of its hypothesis h (None if h is degenerate)."""
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float32)
    v = np.ascontiguousarray(vd, dtype=np.float32)
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    n = int(off[k + 1]) - int(off[k])
    mask = np.zeros(max(n, 1), dtype=np.uint8)
    near = np.zeros(max(n, 1), dtype=np.uint8)
    vx, vy, hd = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n_in, n_near = ctypes.c_int32(), ctypes.c_int32()
    st = ctypes.c_uint8()
    rc = lib.oracle_fit_hypothesis(
        _ptr(th), _ptr(v), _ptr(off), off.shape[0] - 1, th.shape[0], float(tau),
        int(seed) & 0xFFFFFFFFFFFFFFFF, int(k), int(h), near_window,
        ctypes.byref(vx), ctypes.byref(vy), ctypes.byref(hd), ctypes.byref(n_in),
        ctypes.byref(n_near), ctypes.byref(st), _ptr(mask), _ptr(near))
    if rc == -2:
        return None
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return HypothesisFit(vx.value, vy.value, hd.value, n_in.value, n_near.value, st.value,
                         mask[:n], near[:n])


@dataclass
class MaskFit:
    vx: float
    vy: float
    heading: float
    n_inliers: int
    status: int


def refit_on_mask(theta, vd, mask) -> MaskFit:
    """Least-squares refit and heading of ONE cluster (its theta, vd) on a given
    inlier set ``mask`` (bool or uint8 per point; non-finite points skipped),
    Sec. 3.2 Eq. 7 and Eq. 8, summed in point order like the oracle's own refit."""
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float32)
    v = np.ascontiguousarray(vd, dtype=np.float32)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    n = th.shape[0]
    if v.shape[0] != n or m.shape[0] != n:
        raise ValueError("theta, vd and mask differ in length")
    vx, vy, hd = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n_in, st = ctypes.c_int32(), ctypes.c_uint8()
    rc = lib.oracle_refit_mask(_ptr(th), _ptr(v), _ptr(m), n, ctypes.byref(vx), ctypes.byref(vy),
                               ctypes.byref(hd), ctypes.byref(n_in), ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return MaskFit(vx.value, vy.value, hd.value, n_in.value, st.value)


def all_pairs_best(theta, vd, tau: float):
    """Exhaustive search over all valid pairs of ONE cluster.

    Returns (best count or -1, n x n best-pair mask, n x n pair counts (-1 = invalid)).
    """
    lib = _load()
    th = np.ascontiguousarray(theta, dtype=np.float32)
    v = np.ascontiguousarray(vd, dtype=np.float32)
    n = th.shape[0]
    mask = np.zeros((n, n), dtype=np.uint8)
    counts = np.full((n, n), -1, dtype=np.int32)
    best = lib.oracle_all_pairs_best(_ptr(th), _ptr(v), n, float(tau), _ptr(mask), _ptr(counts))
    return int(best), mask.astype(bool), counts


# ---- paper-literal variant (Sec. 3.1 Alg. 1 with Eq. 5's threshold) ----------

@dataclass
class PaperResult:
    vx: np.ndarray          # float64 [K]
    vy: np.ndarray
    heading: np.ndarray
    thresh: np.ndarray      # float64 [K]: MAD of the normalised Doppler values
    n_inliers: np.ndarray   # int32 [K]
    status: np.ndarray      # uint8 [K]
    best_hyp: np.ndarray    # int32 [K]
    inlier_mask: np.ndarray | None  # uint8 [N]
    hyp_valid: np.ndarray | None    # uint8 [K, H]
    hyp_count: np.ndarray | None    # int32 [K, H]


def estimate_velocity_paper(theta, vd, offsets, n_hyp: int, seed: int, *, want_mask: bool = True,
                            debug: bool = False) -> PaperResult:
    """The paper-literal estimate (rv_oracle_paper.c): min-max normalisation,
    MAD threshold, line through two seeds, perpendicular distance <= thresh,
    most inliers, least-squares refit, atan2."""
    lib = _load()
    theta = np.ascontiguousarray(theta, np.float32)
    vd = np.ascontiguousarray(vd, np.float32)
    offsets = np.ascontiguousarray(offsets, np.int32)
    K, N = len(offsets) - 1, len(theta)
    out = dict(vx=np.empty(K), vy=np.empty(K), heading=np.empty(K), thresh=np.empty(K),
               n_inliers=np.empty(K, np.int32), status=np.empty(K, np.uint8),
               best_hyp=np.empty(K, np.int32))
    mask = np.empty(max(N, 1), np.uint8) if want_mask else None
    hv = np.empty((max(K, 1), n_hyp), np.uint8) if debug else None
    hc = np.empty((max(K, 1), n_hyp), np.int32) if debug else None
    rc = lib.oracle_estimate_velocity_paper(
        _ptr(theta), _ptr(vd), _ptr(offsets), K, N, int(n_hyp), int(seed) & 0xFFFFFFFFFFFFFFFF,
        _ptr(out["vx"]), _ptr(out["vy"]), _ptr(out["heading"]), _ptr(out["thresh"]),
        _ptr(out["n_inliers"]), _ptr(out["status"]), _ptr(out["best_hyp"]),
        _ptr(mask) if mask is not None else None, _ptr(hv) if hv is not None else None,
        _ptr(hc) if hc is not None else None)
    if rc != 0:
        raise ValueError("oracle_estimate_velocity_paper: bad arguments")
    return PaperResult(**out, inlier_mask=None if mask is None else mask[:N],
                       hyp_valid=None if hv is None else hv[:K],
                       hyp_count=None if hc is None else hc[:K])


def median(values) -> float:
    """The oracle's median (mean of the two middle values for an even count)."""
    a = np.array(values, dtype=np.float64)
    return float(_load().oracle_median(_ptr(a), a.size))


def paper_line_distance(x1, y1, x2, y2, px, py) -> float:
    """Alg. 1's distance of (px, py) to the line through (x1, y1), (x2, y2)."""
    return float(_load().oracle_paper_line_distance(x1, y1, x2, y2, px, py))
