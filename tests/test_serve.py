"""Served-form driver logic (CPU): arrival schedule and percentiles."""
import numpy as np

from paper_2012_12618_amd import serve


def test_arrivals_are_poisson_per_radar():
    s = serve.arrival_schedule(64, 20.0, 20.0, seed=7)
    ts = np.array([a.t for a in s])
    assert np.all(np.diff(ts) >= 0) and ts.min() >= 0 and ts.max() < 20.0
    assert [a.index for a in s] == list(range(len(s)))
    # 64 radars x 20 frames/s x 20 s = 25600 expected, Poisson sd 160
    assert abs(len(s) - 25600) < 5 * 160
    gaps = np.concatenate([np.diff([a.t for a in s if a.radar == r]) for r in range(64)])
    # exponential gaps: mean 1/20 s, coefficient of variation 1
    assert abs(gaps.mean() - 0.05) < 0.002
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05
    assert serve.arrival_schedule(64, 20.0, 20.0, seed=7)[100] == s[100]


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert serve.percentile(xs, 50) == 50 and serve.percentile(xs, 99) == 99
    assert serve.percentile(xs, 100) == 100 and serve.percentile([3.0], 99) == 3.0
    assert np.isnan(serve.percentile([], 50))
