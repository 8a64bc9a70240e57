"""Pins of the oracle's detection post-processing: the RMS and 1-sigma maps,
the thresholds of eq. 8, the detection rules of Sec. 4 and the second pass
of the conclusion.  Each is checked against something other than itself:
the objective the unmixing reports, closed forms, hand-computed values, and
reductions of the second pass to the first."""
import numpy as np
import pytest

import oracle
import pins
from paper_1402_2518_amd import synth


def _cube(N=10, L=80, P=60, seed=3, noise=0.01):
    rng = np.random.default_rng(seed)
    S = synth.mineral_spectra(N, L, rng).astype(np.float32)
    A = rng.dirichlet(np.ones(N), P)
    X = (A @ S.astype(float) + noise * rng.standard_normal((P, L))).astype(np.float32)
    s = rng.uniform(0.5, 2.0, P).astype(np.float32)
    return S, X, s


def test_rms_matches_the_reported_objective():
    # F s^2 = |residual'|^2 from c - 2 b.a + a.G a; the map sums the residual itself
    S, X, s = _cube()
    r = oracle.unmix(S, X, s, cov=False)
    rms = oracle.rms_map(S, X, r["a"])
    assert np.abs(rms ** 2 * S.shape[1] / (r["F"] * s.astype(float) ** 2) - 1).max() <= 1e-8


def test_rms_with_noise_covariance_is_unwhitened():
    # with a noise covariance the map stays in reflectance units: it equals
    # the expanded form y.y - 2 a.(S y) + a.(S S^T) a of the plain residual,
    # and does not change when C is scaled (the coefficients do not)
    rng = np.random.default_rng(8)
    S, X, s = _cube(N=6, L=40, P=30, seed=8)
    Q = rng.standard_normal((40, 40))
    C = Q @ Q.T / 40 + np.diag(rng.uniform(0.5, 2.0, 40))
    r = oracle.unmix(S, X, s, C=C, cov=False)
    rms = oracle.rms_map(S, X, r["a"])
    Sd, Xd, a = S.astype(float), X.astype(float), r["a"]
    sq = (Xd * Xd).sum(1) - 2 * ((Xd @ Sd.T) * a).sum(1) + ((a @ (Sd @ Sd.T)) * a).sum(1)
    assert np.abs(rms ** 2 * 40 / sq - 1).max() <= 1e-8
    r2 = oracle.unmix(S, X, s, C=7.0 * C, cov=False)
    assert np.abs(oracle.rms_map(S, X, r2["a"]) / rms - 1).max() <= 1e-9
    # and differs from the whitened residual norm (F s^2) when C != I
    assert np.abs(rms ** 2 * 40 / (r["F"] * s.astype(float) ** 2) - 1).max() > 1e-3


def test_rms_of_an_exact_mixture_is_zero():
    rng = np.random.default_rng(1)
    S = pins.disjoint_library(4, 40, rng)
    a = np.array([[0.25, 0.5, 0.125, 0.125]])
    X = (a @ S.astype(float)).astype(np.float32)
    r = oracle.unmix(S, X, None, cov=False)
    assert oracle.rms_map(S, X, r["a"])[0] <= 1e-12


def test_sigma1_closed_form_on_an_equal_orthogonal_library():
    # G = c I and every coefficient free: Cov = (s^2 / c)(I - 1 1^T / N)
    rng = np.random.default_rng(2)
    N, L = 5, 50
    S = pins.disjoint_library(N, L, rng, equal=True)
    c = float((S[0].astype(float) ** 2).sum())
    X = (np.full((1, N), 1.0 / N) @ S.astype(float)).astype(np.float32)
    s = np.array([0.3], np.float32)
    r = oracle.unmix(S, X, s)
    want = float(s[0]) * np.sqrt((1 - 1.0 / N) / c)
    assert np.abs(oracle.sigma1_map(r["cov"])[0] - want).max() <= 1e-10 * want


def test_threshold_hand_computed():
    # endmember 0: present [0.2, 0.4] (mean 0.3, std 0.1), absent [0, 0.02]
    # (mean 0.01, std 0.01): (0.3 - 0.2 + 0.01 + 0.06) / 2 = 0.085.
    # endmember 1 is never absent: no threshold.
    A = np.array([[0.2, 0.5], [0.4, 0.1], [0.0, 0.3], [0.02, 0.2]])
    present = np.array([[1, 1], [1, 1], [0, 1], [0, 1]], bool)
    t = oracle.thresholds(A, present)
    assert abs(t[0] - 0.085) <= 1e-15 and np.isnan(t[1])


def test_threshold_separates_well_separated_classes():
    # present coefficients ~0.3 +- 0.01, absent ~0.001 +- 0.001: the threshold
    # lies between the two populations
    rng = np.random.default_rng(4)
    P = 2000
    present = rng.random((P, 3)) < 0.3
    A = np.where(present, 0.3 + 0.01 * rng.standard_normal((P, 3)), np.abs(0.001 * rng.standard_normal((P, 3))))
    t = oracle.thresholds(A, present)
    assert (t > 0.005).all() and (t < 0.25).all()
    assert ((A > t) == present).mean() > 0.99


def test_detection_rules_truth_table():
    A = np.array([[0.30, 0.30, 0.30, 0.05]])
    s1 = np.array([[0.01, 0.50, 0.01, 0.01]])
    thr = np.array([0.1, 0.1, 0.1, 0.1])
    d = oracle.detect(A, s1, np.array([0.001]), thr, rms_max=0.01)
    assert d.tolist() == [[True, False, True, False]]  # error above coefficient; below threshold
    assert not oracle.detect(A, s1, np.array([0.02]), thr, rms_max=0.01).any()  # fit worse than the noise


def test_second_pass_keeping_everything_is_the_first_pass():
    S, X, s = _cube(N=6, L=50, P=20, seed=6)
    full = oracle.unmix(S, X, s)
    sp = oracle.second_pass(S, X, s, np.ones((20, 6), bool))
    assert np.abs(sp["a"] - full["a"]).max() <= 1e-12
    assert np.abs(sp["cov"] - full["cov"]).max() <= 1e-12 * np.abs(full["cov"]).max()


def test_second_pass_on_the_optimal_free_set_changes_nothing():
    # restricting a convex problem to the support of its certified minimiser
    # leaves the minimiser where it is
    S, X, s = _cube(N=8, L=60, P=25, seed=9)
    full = oracle.unmix(S, X, s)
    ok = full["status"] == 0
    keep = full["a"] > full["lam"]
    sp = oracle.second_pass(S[:], X[ok], s[ok], keep[ok])
    assert np.abs(sp["a"] - full["a"][ok]).max() <= 1e-10


@pytest.mark.parametrize("constraint", [oracle.STO, oracle.POS])
def test_second_pass_single_and_pair(constraint):
    rng = np.random.default_rng(12)
    S, X, s = _cube(N=5, L=40, P=6, seed=12)
    keep = np.zeros((6, 5), bool)
    keep[:3, 2] = True                    # one spectrum
    keep[3:, 0] = keep[3:, 4] = True      # two spectra
    sp = oracle.second_pass(S, X, s, keep, constraint=constraint)
    Sd, Xd = S.astype(float), X.astype(float)
    for p in range(3):
        if constraint == oracle.STO:
            assert sp["a"][p, 2] == pytest.approx(1.0, abs=1e-14)
        else:  # clipped least squares on one spectrum
            want = max(0.0, float(Xd[p] @ Sd[2]) / float(Sd[2] @ Sd[2]))
            assert sp["a"][p, 2] == pytest.approx(want, rel=1e-10)
        assert np.abs(np.delete(sp["a"][p], 2)).max() == 0.0
        if constraint == oracle.STO:  # a single free coefficient under the sum row has no variance
            assert np.abs(sp["cov"][p]).max() <= 1e-12
    if constraint == oracle.STO:
        for p in range(3, 6):
            want = pins.two_endmembers(Sd[0], Sd[4], Xd[p])
            assert np.abs(sp["a"][p, [0, 4]] - want).max() <= 1e-10
    assert np.isnan(oracle.second_pass(S, X[:1], s[:1], np.zeros((1, 5), bool))["a"]).all()
