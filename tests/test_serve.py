"""The request loop's host-side pieces (no GPU): admission rule and the
arrival process."""
import numpy as np

from paper_1402_2518_amd import serve


def test_admission_rule():
    # a free slot and room in the budget
    assert serve.admissible(10, 0, 100, 0, 4)
    assert serve.admissible(10, 90, 100, 3, 4)
    assert not serve.admissible(11, 90, 100, 3, 4)
    assert not serve.admissible(1, 0, 100, 4, 4)
    # larger than the whole budget: admitted only when nothing else runs
    assert serve.admissible(500, 0, 100, 0, 4)
    assert not serve.admissible(500, 10, 100, 1, 4)


def test_poisson_arrivals():
    rng = np.random.default_rng(3)
    t = serve.poisson_arrivals(50.0, 200.0, rng)
    assert (np.diff(t) > 0).all() and t.min() >= 0 and t.max() < 200
    assert abs(len(t) / 200.0 - 50.0) < 2.0  # rate
    gaps = np.diff(t)
    assert abs(gaps.mean() - 0.02) < 0.001 and abs(gaps.std() / gaps.mean() - 1) < 0.05  # exponential gaps
