"""Pins of the oracle's other constraint options (sum-lower-than-one and
positivity only): library NNLS, enumeration of free sets, the convexity rule
linking the three problems, natural residuals and covariance closed forms.
CPU only."""
import numpy as np
import pytest
from scipy.optimize import nnls

import oracle
import pins
from paper_1402_2518_amd import synth


def _mixtures(N, L, P, seed, noise=0.01, scale=(0.6, 1.4)):
    """Mixtures whose sum of coefficients is spread around one, so that the
    sum constraint binds for some pixels and not for others."""
    rng = np.random.default_rng(seed)
    S = rng.uniform(0.05, 1.0, (N, L)).astype(np.float32)
    A = rng.dirichlet(np.ones(N), P) * rng.uniform(*scale, (P, 1))
    X = (A @ S + noise * rng.standard_normal((P, L))).astype(np.float32)
    return S, X


@pytest.mark.parametrize("N,L", [(3, 20), (6, 40), (8, 64)])
def test_pos_matches_brute_force_and_nnls(oracle_lib, N, L):
    S, X = _mixtures(N, L, 150, seed=N)
    r = oracle_lib.unmix(S, X, None, cov=False, constraint=oracle.POS)
    assert (r["status"] & ~np.uint8(oracle.DEGENERATE) == 0).all(), r["status"]
    G, B = pins.gram(S), pins.proj(S, X)
    assert np.abs(r["a"] - pins.brute_force_pos(G, B)).max() <= 1e-9
    for p in range(0, 150, 10):  # the library NNLS on the least-squares form
        a_n, _ = nnls(S.astype(np.float64).T, X[p].astype(np.float64))
        assert np.abs(r["a"][p] - a_n).max() <= 1e-8
    assert np.abs(r["nu"]).max() == 0.0
    assert pins.natural_residual_set(G, B, r["a"], "pos").max() <= 1e-10


@pytest.mark.parametrize("N,L", [(3, 20), (6, 40), (8, 64)])
def test_slo_is_pos_or_sto(oracle_lib, N, L):
    """Convexity: the sum-lower-than-one minimiser is the positivity-only one
    when that sums to at most one, and the sum-to-one one otherwise."""
    S, X = _mixtures(N, L, 150, seed=10 + N)
    G, B = pins.gram(S), pins.proj(S, X)
    r = oracle_lib.unmix(S, X, None, cov=False, constraint=oracle.SLO)
    assert (r["status"] & ~np.uint8(oracle.DEGENERATE) == 0).all(), r["status"]
    a_pos = pins.brute_force_pos(G, B)
    a_sto, _ = pins.brute_force(G, B)
    below = a_pos.sum(1) <= 1.0
    assert 10 <= below.sum() <= 140, below.sum()  # both regimes present
    want = np.where(below[:, None], a_pos, a_sto)
    assert np.abs(r["a"] - want).max() <= 1e-9
    assert (r["a"].sum(1) <= 1.0 + 1e-12).all()
    assert pins.natural_residual_set(G, B, r["a"], "slo").max() <= 1e-10
    # the sum multiplier is zero off the bound and nonnegative on it
    assert np.abs(r["nu"][below]).max() <= 1e-12
    assert (r["nu"][~below] >= -1e-12).all()


def test_sto_unchanged_by_option(oracle_lib):
    S, X = _mixtures(6, 40, 100, seed=3)
    r0 = oracle_lib.unmix(S, X, None)
    r1 = oracle_lib.unmix(S, X, None, constraint=oracle.STO)
    assert np.array_equal(r0["a"], r1["a"]) and np.array_equal(r0["cov"], r1["cov"])


@pytest.mark.parametrize("constraint", ["pos", "slo"])
def test_covariance_on_an_orthogonal_library(oracle_lib, constraint):
    """G = c I: positivity only gives a = max(b / c, 0) and, on the free set,
    Cov = (s^2 / c) I; sum-lower-than-one adds the sum row only where the
    bound is active, where Cov = (s^2 / c)(I - 1 1^T / |F|)."""
    N, L = 12, 96
    rng = np.random.default_rng(21)
    S = pins.disjoint_library(N, L, rng, equal=True)
    X = (rng.uniform(0, 1, (40, L)) * rng.uniform(0.02, 0.6, (40, 1))).astype(np.float32)
    s = rng.uniform(0.5, 2.0, 40).astype(np.float32)
    cons = oracle.POS if constraint == "pos" else oracle.SLO
    r = oracle_lib.unmix(S, X, s, constraint=cons)
    G, B = pins.gram(S), pins.proj(S, X)
    c = G[0, 0]
    a_pos = np.maximum(B / c, 0.0)
    if constraint == "pos":
        want, bound = a_pos, np.zeros(40, bool)
    else:
        bound = a_pos.sum(1) > 1.0
        want = np.where(bound[:, None], pins.simplex_project(B / c), a_pos)
        assert 5 <= bound.sum() <= 35
    assert np.abs(r["a"] - want).max() <= 1e-12
    for p in range(40):
        F = want[p] > 0
        k = F.sum()
        C = np.zeros((N, N))
        blk = np.eye(k) - (np.ones((k, k)) / k if bound[p] else 0.0)
        C[np.ix_(F, F)] = float(s[p]) ** 2 / c * blk
        assert np.abs(r["cov"][p] - C).max() <= 1e-12 * max(1.0, np.abs(C).max())


def test_uncertified_covariance_uses_the_slack_corner(oracle_lib):
    """Three iterations, sum-lower-than-one: Cov = (s^2/gamma)(H^-1 - u u^T /
    (1^T u + s/nu)) at the last iterate; pinned by inverting the bordered
    matrix [[H, 1], [1^T, -s/nu]] with NumPy."""
    S, X = _mixtures(5, 30, 20, seed=8)
    r = oracle_lib.unmix(S, X, None, constraint=oracle.SLO, maxit=3)
    assert (r["status"] == oracle.MAXIT).all()
    G = pins.gram(S)
    gam = G.diagonal().max()
    for p in range(20):
        a, lam, nu = r["a"][p], r["lam"][p], r["nu"][p]
        slack = 1.0 - a.sum()
        H = G / gam + np.diag(lam / a)
        K = np.block([[H, np.ones((5, 1))], [np.ones((1, 5)), np.array([[-slack / nu]])]])
        want = np.linalg.inv(K)[:5, :5] / gam
        assert np.abs(r["cov"][p] - want).max() <= 1e-9 * np.abs(want).max()


def test_orbital_workload_constraint_options(oracle_lib):
    """On the orbital mixtures (sums of one by construction) the three
    options agree where the sum constraint is not binding."""
    w = synth.WORKLOADS["orbital"]
    S = synth.make_library(w)
    X, s = synth.make_cube(w, S, 0, 300)
    rs = {c: oracle_lib.unmix(S, X, s, cov=False, constraint=c) for c in (oracle.STO, oracle.SLO, oracle.POS)}
    G, B = pins.gram(S), pins.proj(S, X)
    for c, name in ((oracle.SLO, "slo"), (oracle.POS, "pos")):
        ok = rs[c]["status"] == 0
        assert ok.mean() > 0.9
        assert pins.natural_residual_set(G, B[ok], rs[c]["a"][ok], name).max() <= 1e-9
    free_sum = rs[oracle.POS]["a"].sum(1)
    same = (free_sum <= 1.0) & (rs[oracle.POS]["status"] == 0) & (rs[oracle.SLO]["status"] == 0)
    assert np.abs(rs[oracle.SLO]["a"][same] - rs[oracle.POS]["a"][same]).max() <= 1e-9
