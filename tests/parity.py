"""GPU-versus-oracle acceptance protocol (helper module for the GPU tests and the
smoke check; not collected by pytest).

The estimator scores hypotheses in float32 while the oracle works in FP64, so
the inlier count of a hypothesis may differ where a residual lies within the
float32 rounding error of tau.  The protocol:

1. status bytes equal;
2. per hypothesis: the GPU count lies in the oracle's [count_lo, count_hi] band
   (the band covers the float32 error bound of each residual, and at least
   1e-5 m/s); an invalid hypothesis counts 0;
3. selection: when no candidate for the maximum has an ambiguous count the GPU
   keeps the oracle's hypothesis; otherwise it keeps a candidate (count_hi at
   least the largest count_lo), reported as an ambiguous selection;
4. the refit is compared with the oracle's refit of the hypothesis the GPU
   kept: inlier masks equal except at points flagged within 1e-5 m/s of tau;
   with equal masks n_inliers and n_near_tau are equal and vx, vy agree with
   the oracle's refit within 1e-4 m/s; where the masks differ, vx, vy and the
   heading are compared with the oracle's FP64 least-squares refit on the
   GPU's own mask (Sec. 3.2, Eq. 7); the heading agrees within 2e-4/|v| + 1e-6
   rad when |v| >= 0.01 m/s.

Statistics: besides the counts above, how many hypothesis counts differ from
the FP64 count (``hyp_count_differs``) and how many of those lie outside the
absolute 1e-5 m/s band and pass only through the band's relative term
(``hyp_rel_band_only``), so that widening beyond the stated window is never
silent.
"""
from __future__ import annotations

import math
import sys

import numpy as np

V_TOL = 1e-4


def v_tolerance(ref_vx: float, ref_vy: float) -> float:
    """Bound on |GPU - oracle| for vx and vy: 1e-4 m/s plus the float32
    rounding of the outputs (half a unit in the last place, at most
    2^-24 max(|vx|, |vy|)), which alone exceeds 1e-4 m/s above about 1680 m/s
    (refits through a few nearly collinear points)."""
    return V_TOL + 2.0 ** -24 * max(abs(ref_vx), abs(ref_vy))


def unpack_bits(words: np.ndarray, n_points: int) -> np.ndarray:
    """int32/uint32 words (bit p%32 of word p/32 = point p) -> bool [n_points]."""
    w = np.ascontiguousarray(words).view(np.uint32)
    return np.unpackbits(w.view(np.uint8), bitorder="little")[:n_points].astype(bool)


def run_gpu(theta, vd, offsets, n_hyp, tau, seed, *, debug=True, bits=True, device="cuda:0",
            label=""):
    """Run the HIP estimator on numpy inputs; returns numpy outputs."""
    import torch

    from paper_2012_12618_amd import binding

    print(f"[gpu] rv_estimate_velocity {label} K={len(offsets) - 1} N={len(theta)} "
          f"H={n_hyp} tau={tau} seed={seed:#x}", flush=True)
    t = torch.from_numpy(np.ascontiguousarray(theta, np.float32)).to(device)
    v = torch.from_numpy(np.ascontiguousarray(vd, np.float32)).to(device)
    o = torch.from_numpy(np.ascontiguousarray(offsets, np.int32)).to(device)
    res = binding.rv_estimate_velocity(t, v, o, n_hyp, tau, seed, want_near=True,
                                       want_bits=bits, debug=debug)
    torch.cuda.synchronize()
    out = {k: x.cpu().numpy() for k, x in res.items()}
    if bits:
        out["mask"] = unpack_bits(out["inlier_bits"], len(theta))
    return out


def check(theta, vd, offsets, n_hyp, tau, seed, g: dict, o, *, check_hyp=True,
          cluster_ids=None) -> dict:
    """Apply the protocol to GPU outputs ``g`` and oracle result ``o`` (debug run).

    With ``cluster_ids``, ``o`` holds only those clusters (oracle run with the
    same list) while ``g`` holds the whole frame; only the listed clusters are
    checked."""
    import oracle

    offsets = np.asarray(offsets, dtype=np.int64)
    K_all = len(offsets) - 1
    ids = np.arange(K_all) if cluster_ids is None else np.asarray(cluster_ids, dtype=np.int64)
    K = len(ids)
    stats = {"clusters": K, "ambiguous_selection": 0, "mask_diff_points": 0,
             "refit_on_gpu_mask": 0, "max_dv": 0.0, "max_dheading": 0.0, "hyp_checked": 0,
             "hyp_count_differs": 0, "hyp_rel_band_only": 0}
    if cluster_ids is not None:
        g = dict(g)
        for key in ("vx", "vy", "heading", "n_inliers", "status", "n_near_tau", "best_hyp"):
            if key in g:
                g[key] = g[key][ids]
        if "hyp_counts" in g:
            g["hyp_counts"] = g["hyp_counts"].reshape(K_all, n_hyp)[ids]
    assert np.array_equal(g["status"], o.status), (
        f"status differs at clusters {ids[np.flatnonzero(g['status'] != o.status)][:10]}")
    if K == 0:
        return stats

    H = n_hyp
    if check_hyp:
        gc = g["hyp_counts"].reshape(K, H)
        valid = o.hyp_valid.astype(bool)
        out_of_band = valid & ((gc < o.hyp_count_lo) | (gc > o.hyp_count_hi))
        if out_of_band.any():
            k, h = np.argwhere(out_of_band)[0]
            raise AssertionError(
                f"{out_of_band.sum()} hypothesis counts outside the band; first k={k} h={h}: "
                f"gpu={gc[k, h]} band=[{o.hyp_count_lo[k, h]}, {o.hyp_count_hi[k, h]}] "
                f"oracle={o.hyp_count[k, h]} vx={o.hyp_vx[k, h]} vy={o.hyp_vy[k, h]}")
        assert np.all(gc[~valid] == 0), "an invalid hypothesis has a nonzero count"
        stats["hyp_checked"] = int(valid.sum())
        differs = valid & (gc != o.hyp_count)
        stats["hyp_count_differs"] = int(differs.sum())
        rows = np.flatnonzero(differs.any(axis=1))
        if rows.size:
            # the same clusters with the absolute half-width only
            a = oracle.estimate_velocity(theta, vd, np.asarray(offsets, np.int32), n_hyp, tau, seed,
                                         cluster_ids=ids[rows], debug=True, want_mask=False,
                                         band_rel=0.0)
            d = differs[rows]
            outside = d & ((gc[rows] < a.hyp_count_lo) | (gc[rows] > a.hyp_count_hi))
            stats["hyp_rel_band_only"] = int(outside.sum())

    gmask = g.get("mask")
    for i in range(K):
        k = int(ids[i])
        st = int(o.status[i])
        if st in (oracle.CLUSTER_TOO_FEW_POINTS, oracle.CLUSTER_BAD_OFFSETS,
                  oracle.CLUSTER_ALL_DEGENERATE):
            assert g["n_inliers"][i] == 0
            assert math.isnan(g["vx"][i]) and math.isnan(g["vy"][i]) and math.isnan(g["heading"][i])
            assert g["best_hyp"][i] == -1
            continue
        lo, hi = int(offsets[k]), int(offsets[k + 1])
        hg, ho = int(g["best_hyp"][i]), int(o.best_hyp[i])
        if hg == ho:
            ref_vx, ref_vy, ref_hd = o.vx[i], o.vy[i], o.heading[i]
            ref_n, ref_near = int(o.n_inliers[i]), int(o.n_near_tau[i])
            ref_mask = o.inlier_mask[lo:hi].astype(bool) if o.inlier_mask is not None else None
            ref_nearmask = None
            ref_status = st
        else:
            # decided from the oracle's bands alone (no GPU counts needed)
            assert o.hyp_valid is not None, (
                f"cluster {k}: gpu kept h={hg}, oracle h={ho}, and the oracle ran without bands")
            valid = o.hyp_valid[i].astype(bool)
            clo, chi = o.hyp_count_lo[i], o.hyp_count_hi[i]
            m_lo = clo[valid].max()
            cand = valid & (chi >= m_lo)
            assert (clo[cand] != chi[cand]).any(), (
                f"cluster {k}: selection differs (gpu {hg}, oracle {ho}) without ambiguity")
            assert cand[hg], f"cluster {k}: gpu kept h={hg} which cannot be a maximum"
            stats["ambiguous_selection"] += 1
            f = oracle.fit_hypothesis(theta, vd, offsets.astype(np.int32), tau, seed, k, hg)
            assert f is not None
            ref_vx, ref_vy, ref_hd = f.vx, f.vy, f.heading
            ref_n, ref_near = f.n_inliers, f.n_near_tau
            ref_mask, ref_nearmask, ref_status = f.mask.astype(bool), f.near_mask.astype(bool), f.status
        assert int(g["status"][i]) == ref_status
        masks_equal = True
        if gmask is not None and ref_mask is not None:
            diff = np.flatnonzero(gmask[lo:hi] != ref_mask)
            if diff.size:
                if ref_nearmask is None:
                    f = oracle.fit_hypothesis(theta, vd, offsets.astype(np.int32), tau, seed, k, hg)
                    ref_nearmask = f.near_mask.astype(bool)
                assert ref_nearmask[diff].all(), (
                    f"cluster {k}: inlier masks differ at points not near tau: {diff[:10]}")
                stats["mask_diff_points"] += int(diff.size)
                masks_equal = False
        if masks_equal:
            assert int(g["n_inliers"][i]) == ref_n, f"cluster {k}: n_inliers {g['n_inliers'][i]} vs {ref_n}"
            if "n_near_tau" in g:
                assert int(g["n_near_tau"][i]) == ref_near
        else:
            # Sec. 3.2, Eq. 7 on the GPU's own inlier set, in FP64
            gm = gmask[lo:hi]
            assert int(g["n_inliers"][i]) == int(gm.sum()), f"cluster {k}: n_inliers vs its mask"
            mf = oracle.refit_on_mask(theta[lo:hi], vd[lo:hi], gm)
            ref_vx, ref_vy, ref_hd, ref_status = mf.vx, mf.vy, mf.heading, mf.status
            assert int(g["status"][i]) == ref_status, f"cluster {k}: status on the GPU's mask"
            stats["refit_on_gpu_mask"] += 1
        if ref_status != oracle.CLUSTER_OK:
            continue
        dv = max(abs(float(g["vx"][i]) - ref_vx), abs(float(g["vy"][i]) - ref_vy))
        stats["max_dv"] = max(stats["max_dv"], dv)
        assert dv <= v_tolerance(ref_vx, ref_vy), f"cluster {k}: |dv| = {dv}"
        speed = math.hypot(ref_vx, ref_vy)
        if speed >= 0.01:
            dh = abs(math.remainder(float(g["heading"][i]) - ref_hd, 2 * math.pi))
            stats["max_dheading"] = max(stats["max_dheading"], dh)
            assert dh <= 2e-4 / speed + 1e-6, f"cluster {k}: heading off by {dh}"
    return stats


def report(name: str, stats: dict) -> None:
    print(f"[parity] {name}: {stats}", file=sys.stderr, flush=True)
