"""CPU: the error band of the FP16 residual form of the scoring.

The FP16 form counts a point for hypothesis h = (hx, hy) when |D| < tau_h.
D is the dot product of the point's FP16 (cos, sin), rounded toward zero, with
the FP16 offset -(h - r), rounded to nearest, added in float32 to the point's
float32 residual w against the workgroup's reference velocity r.  The widened
threshold is tau_h = tau + 2^-8 A + 2^-18 (tau + M + 1) + 2 t, with
A = |hx - rx| + |hy - ry|, M = |hx| + |hy| + |rx| + |ry| and t the magnitude of
the offset components below 2^-14 (the smallest normal FP16 value), which are
sent as 0.  The form selects exactly the float32 form's hypothesis only if
every point whose float32 residual fma(-hy, s, fma(-hx, c, v)) is below tau
also passes |D| < tau_h.

These tests model that arithmetic in numpy: float32 FMAs (exact products in
float64, one rounding), FP16 conversions, the dot product's additions in
several orders and roundings, FP16 subnormals kept or flushed.  They check the
bound on inputs built to stress it: inliers within 10^-7 tau of the threshold,
offsets from 0 to 2^14, velocities to 10^4 m/s, tau from 10^-3 to 3 m/s,
azimuths near 0 and near +-pi/2, and that the error stays below half the
band, the bound the band doubles.  Two tests weaken the band (a smaller offset
term; no subnormal term with subnormal offsets flushed) and the check finds
the violations.
"""
import numpy as np
import pytest

F32 = np.float32
F16 = np.float16
TWO_M14 = F32(2.0 ** -14)
MAX_OFFSET = F32(16384.0)


def fma32(a, b, c):
    """float32 fma: the product is exact in float64, the sum rounds once (to
    float64, then float32; a double rounding at most moves a result by one
    float32 ulp, far inside the band's factor of two)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def to_f16_rtz(x):
    h = x.astype(F16)
    over = np.abs(h.astype(F32)) > np.abs(x)
    h[over] = np.nextafter(h[over], F16(0))
    return h


def flush16(h):
    h = h.copy()
    h[np.abs(h.astype(F32)) < TWO_M14] = F16(0)
    return h


def rtz32(x64):
    y = x64.astype(F32)
    over = np.abs(y.astype(np.float64)) > np.abs(x64)
    y[over] = np.nextafter(y[over], F32(0))
    return y


def widened(hx, hy, rx, ry, tau, subnormal_term=True):
    """(FP16 -(h - r), tau_h, converted?) of each hypothesis, in float32 steps."""
    dx = hx - rx
    dy = hy - ry
    a = np.abs(dx) + np.abs(dy)
    m = np.abs(hx) + np.abs(hy) + np.abs(rx) + np.abs(ry)
    tiny = np.zeros_like(a)
    if subnormal_term:
        sx = np.abs(dx) < TWO_M14
        sy = np.abs(dy) < TWO_M14
        tiny = np.where(sx, np.abs(dx), F32(0)) + np.where(sy, np.abs(dy), F32(0))
        dx = np.where(sx, F32(0), dx)
        dy = np.where(sy, F32(0), dy)
    band = a * F32(2.0 ** -8) + (tau + m + F32(1)) * F32(2.0 ** -18) + F32(2) * tiny
    return (-dx).astype(F16), (-dy).astype(F16), tau + band, a < MAX_OFFSET


def dot_variants(ch, sh, ndx, ndy, w):
    p1 = ch.astype(np.float64) * ndx.astype(np.float64)  # exact: 11 x 11 bits
    p2 = sh.astype(np.float64) * ndy.astype(np.float64)
    w64 = w.astype(np.float64)
    yield "one rounding", (p1 + p2 + w64).astype(F32)
    yield "products first", ((p1 + p2).astype(F32).astype(np.float64) + w64).astype(F32)
    yield "chained", ((w64 + p1).astype(F32).astype(np.float64) + p2).astype(F32)
    yield "toward zero", rtz32(p1 + p2 + w64)


def adversarial(rng, scale, tau, nh=1500, npts=96):
    """Hypotheses around a reference, and for each hypothesis points that are
    its inliers, most of them within a hair of the threshold."""
    r = (scale * rng.uniform(-1, 1, (nh, 2))).astype(F32)
    far = np.abs(r[:, 0]) + np.abs(r[:, 1]) >= MAX_OFFSET  # the kernel's reference rule
    r[far] = 0
    mag = 10.0 ** rng.uniform(-10, np.log10(16000.0), nh)
    mag[rng.random(nh) < 0.05] = 0.0
    phi = rng.uniform(-np.pi, np.pi, nh)
    off = np.stack([mag * np.cos(phi), mag * np.sin(phi)], 1)
    axis = rng.random(nh)
    off[axis < 0.1, 1] = 0.0  # one component exactly zero
    off[(axis >= 0.1) & (axis < 0.2), 0] *= 1e-9  # one component tiny
    h = (r.astype(np.float64) + off).astype(F32)

    kind = rng.random((nh, npts))
    theta = rng.uniform(-np.pi / 2 + 1e-3, np.pi / 2 - 1e-3, (nh, npts))
    edge = np.pi / 2 - 10.0 ** rng.uniform(-7, -2, (nh, npts))
    theta = np.where(kind < 0.15, np.sign(theta) * edge, theta)
    near0 = np.sign(theta) * 10.0 ** rng.uniform(-8, -2, (nh, npts))
    theta = np.where((kind >= 0.15) & (kind < 0.3), near0, theta)
    c = np.cos(theta).astype(F32)
    s = np.sin(theta).astype(F32)

    u = rng.uniform(-1, 1, (nh, npts))
    hair = np.sign(u) * (1.0 - 10.0 ** rng.uniform(-7, -1, (nh, npts)))
    u = np.where(rng.random((nh, npts)) < 0.6, hair, u)
    v = (h[:, :1].astype(np.float64) * c + h[:, 1:].astype(np.float64) * s
         + float(tau) * u).astype(F32)
    return h, r, c, s, v


def violations(h, r, c, s, v, tau, flush, subnormal_term=True):
    hx, hy = h[:, :1], h[:, 1:]
    rx, ry = r[:, :1], r[:, 1:]
    e32 = fma32(-hy, s, fma32(-hx, c, v))
    inlier = np.abs(e32) < tau
    ndx, ndy, th, conv = widened(hx, hy, rx, ry, tau, subnormal_term)
    w = fma32(-ry, s, fma32(-rx, c, v))
    ch, sh = to_f16_rtz(c), to_f16_rtz(s)
    if flush:
        ch, sh, ndx, ndy = flush16(ch), flush16(sh), flush16(ndx), flush16(ndy)
    out = {}
    worst = 0.0  # largest |D - float32 residual| / (tau_h - tau) over the inliers
    band = np.broadcast_to((th.astype(np.float64) - float(tau)), inlier.shape)
    for name, d in dot_variants(ch, sh, ndx, ndy, w):
        out[name] = int(np.count_nonzero(inlier & conv & ~(np.abs(d) < th)))
        err = np.abs(d.astype(np.float64) - e32.astype(np.float64))
        sel = inlier & conv
        if np.any(sel):
            worst = max(worst, float(np.max(err[sel] / band[sel])))
    return out, int(np.count_nonzero(inlier & conv)), worst


@pytest.mark.parametrize("scale", [0.0, 1.0, 40.0, 1000.0, 12000.0])
@pytest.mark.parametrize("tau", [1e-3, 0.15, 3.0])
@pytest.mark.parametrize("flush", [False, True])
def test_fp16_band_bounds_every_float32_inlier(scale, tau, flush):
    rng = np.random.default_rng(int(scale * 7 + tau * 1000) + (1 << 20) * flush)
    tau = F32(tau)
    h, r, c, s, v = adversarial(rng, scale, tau)
    bad, checked, worst = violations(h, r, c, s, v, tau, flush)
    assert checked > 50_000  # the cases are mostly near-threshold inliers
    assert all(n == 0 for n in bad.values()), bad
    # The derivation bounds the error by half the band (the band takes twice
    # the bound); with subnormals kept that half holds as stated.
    if not flush:
        assert worst < 0.5, worst


def test_a_weaker_offset_term_is_caught():
    # The check has teeth: with 2^-12 A in place of 2^-8 A the FP16 counts
    # are no longer upper bounds on these inputs.
    rng = np.random.default_rng(3)
    tau = F32(0.15)
    h, r, c, s, v = adversarial(rng, 40.0, tau)
    real = widened

    def weaker(hx, hy, rx, ry, tau, subnormal_term=True):
        ndx, ndy, th, conv = real(hx, hy, rx, ry, tau, subnormal_term)
        a = np.abs(hx - rx) + np.abs(hy - ry)
        return ndx, ndy, th - a * F32(2.0 ** -8) + a * F32(2.0 ** -12), conv

    globals()["widened"] = weaker
    try:
        bad, _, _ = violations(h, r, c, s, v, tau, flush=False)
    finally:
        globals()["widened"] = real
    assert min(bad.values()) > 0


def test_offsets_below_fp16_normal_range_need_their_term():
    # A near-static hypothesis 3e-5 m/s from the reference (an FP16 subnormal
    # offset), tau = 1e-3 and inliers just inside tau: if the dot product
    # flushed the offset and the band had no term for it, such inliers would
    # fall outside tau_h.
    rng = np.random.default_rng(5)
    n = 4096
    tau = F32(1e-3)
    h = np.array([[3e-5, -2e-5]], dtype=F32)
    r = np.zeros((1, 2), dtype=F32)
    theta = rng.uniform(-1.2, 1.2, (1, n))
    c = np.cos(theta).astype(F32)
    s = np.sin(theta).astype(F32)
    u = np.sign(rng.uniform(-1, 1, (1, n))) * (1 - 10.0 ** rng.uniform(-6, -3, (1, n)))
    v = (h[:, :1].astype(np.float64) * c + h[:, 1:].astype(np.float64) * s
         + float(tau) * u).astype(F32)
    bad_old, checked, _ = violations(h, r, c, s, v, tau, flush=True, subnormal_term=False)
    assert checked > 3000 and min(bad_old.values()) > 0
    bad_new, _, _ = violations(h, r, c, s, v, tau, flush=True, subnormal_term=True)
    assert all(n == 0 for n in bad_new.values()), bad_new
