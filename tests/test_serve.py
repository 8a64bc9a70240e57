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


def test_pick_passes_a_blocked_head_for_a_bounded_time():
    R = serve.Request
    big = R(0, "a", None, None, arrival=0.0)
    small = R(1, "a", None, None, arrival=0.1)
    big.footprint, small.footprint = 80, 10
    w = [big, small]
    # the head does not fit next to 50 running bytes; the smaller one does
    assert serve.pick(w, 50, 100, 1, 4, now=0.2, max_pass_s=0.5) == 1
    # the head has waited past the bound: nothing passes it
    assert serve.pick(w, 50, 100, 1, 4, now=0.6, max_pass_s=0.5) is None
    # the head fits: it goes first
    assert serve.pick(w, 10, 100, 1, 4, now=0.2, max_pass_s=0.5) == 0
    # no free slot
    assert serve.pick(w, 0, 100, 4, 4, now=0.2, max_pass_s=0.5) is None
    # nothing running: the head is admitted whatever its size
    big.footprint = 500
    assert serve.pick(w, 0, 100, 0, 4, now=0.2, max_pass_s=0.5) == 0
    assert serve.pick([], 0, 100, 0, 4, now=0.0, max_pass_s=0.5) is None


def test_footprint_counts_the_device_copy_of_a_host_cube():
    class Lib:
        N, L = 10, 100

        def workspace_bytes(self, P, precision, cov):
            return 1000

    dev = serve.footprint(Lib(), 50, "fp64", "full")
    host = serve.footprint(Lib(), 50, "fp64", "full", host_input=True)
    assert dev == 50 * (8 * 10 + 8 * 100 + 1 + 4 + 8) + 1000
    assert host - dev == 50 * (4 * 100 + 4)
