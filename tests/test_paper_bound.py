"""CPU: the division-free form of Alg. 1's inlier test in the paper-literal
trial kernel.

For one line with distance denominator d >= 1, the kernel replaces the test
RN(|num| / d) <= th (RN: the correctly rounded FP64 quotient) by
|num| <= bound, where bound is the largest double x >= 0 with RN(x / d) <= th,
found by bisection over the bit patterns of the eight doubles around
RN(th * d).  The two tests agree for every num because RN(x / d) never
decreases as x grows.  Python floats are IEEE doubles with correctly rounded
division, so the search is modelled here with the kernel's steps and checked
against the literal test at the bound, next to it and at random values, over
slopes from 0 to 10^8 and thresholds from 10^-80 to 1.  Two weakened searches
(the product RN(th * d) taken as the bound; the bound one double too high)
disagree with the literal test, so the check has teeth.
"""
import math
import random
import struct

import pytest


def bits(x):
    return struct.unpack("<q", struct.pack("<d", x))[0]


def from_bits(b):
    return struct.unpack("<d", struct.pack("<q", b))[0]


def pass_bound(d, th, half_width=4):
    """The kernel's search; None where it falls back to the literal test."""
    if not (1.0 <= d < math.inf) or not (0.0 < th < math.inf):
        return None
    x0 = th * d
    if not (2.0 ** -1000 < x0 < 2.0 ** 1000):
        return None
    lo = bits(x0) - half_width
    hi = lo + 2 * half_width
    if not (from_bits(lo) / d <= th) or from_bits(hi) / d <= th:
        return None
    while hi - lo > 1:
        mid = lo + (hi - lo) // 2
        if from_bits(mid) / d <= th:
            lo = mid
        else:
            hi = mid
    return from_bits(lo)


def cases(seed, n):
    rng = random.Random(seed)
    for _ in range(n):
        m = rng.choice([0.0, 1e-9, 0.3, 3.0, 1e4, 1e8]) * rng.uniform(-1, 1)
        d = math.sqrt(m * m + 1.0)
        th = rng.choice([rng.uniform(0, 1), 10 ** rng.uniform(-80, 0), 0.5, 0.25, 1.0])
        yield rng, d, th


def disagreements(bound_of, seed=1, n=20000):
    bad = checked = 0
    for rng, d, th in cases(seed, n):
        bd = bound_of(d, th)
        if bd is None:
            continue
        b = bits(bd)
        probes = [from_bits(b + k) for k in range(-3, 4)] + [rng.uniform(0, 2 * bd) for _ in range(3)]
        for x in probes:
            for num in (x, -x):
                checked += 1
                bad += (abs(num / d) <= th) != (abs(num) <= bd)
    return bad, checked


def test_bound_agrees_with_the_literal_test():
    bad, checked = disagreements(pass_bound)
    assert checked > 300_000 and bad == 0


def test_no_fallback_on_the_paper_workloads_range():
    # Normalised coordinates give thresholds in (0, 1] and d = sqrt(m^2 + 1).
    assert all(pass_bound(d, th) is not None for _, d, th in cases(2, 20000))


@pytest.mark.parametrize("d,th", [(1.0, 0.0), (math.inf, 0.3), (math.nan, 0.3), (2.0, math.nan),
                                  (1.5, 2.0 ** -1070)])
def test_degenerate_inputs_take_the_literal_test(d, th):
    assert pass_bound(d, th) is None


def test_weakened_searches_are_caught():
    bad_product, _ = disagreements(lambda d, th: None if pass_bound(d, th) is None else th * d)
    assert bad_product > 0

    def one_above(d, th):
        bd = pass_bound(d, th)
        return None if bd is None else from_bits(bits(bd) + 1)

    bad_above, _ = disagreements(one_above)
    assert bad_above > 0
