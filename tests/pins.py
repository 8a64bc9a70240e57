"""Independent checks that pin the CPU oracle to the mathematics.

Every routine here is written from the problem statement of the paper (the
least-squares criterion of eqs. 2/6 under positivity, eq. 3, and sum-to-one,
eq. 4) or from textbook closed forms, in NumPy, and shares nothing with the
oracle's C code.  Each one pins a different part:

* ``simplex_project`` / ``natural_residual``: the KKT conditions of the QP in
  one number (zero exactly at the minimiser).  Projection onto the simplex by
  the sorting method (Held, Wolfe & Crowder 1974).
* ``brute_force``: every active set of a tiny library (the "test all
  combinations" idea of Sec. 2.1), each solved as an equality-constrained
  problem; the feasible one with the smallest criterion is the minimiser.
* ``water_filling``: the closed-form minimiser for a diagonal Gram matrix.
* ``two_endmembers``: the closed form for N = 2 (projection onto a segment).
* ``scls``: the sum-to-one-only solution (Sec. 2.2, SCLS), equal to the
  minimiser when that is interior.
* ``bordered_cov``: the estimator covariance on a free set, as the upper-left
  block of the inverse of the bordered matrix [[G_FF, 1], [1^T, 0]].
"""
from __future__ import annotations

import itertools

import numpy as np


def gram(S: np.ndarray, C: np.ndarray | None = None):
    """``G = S C^-1 S^T`` (float64), with ``C = I`` when omitted."""
    S = np.asarray(S, np.float64)
    if C is None:
        return S @ S.T
    return S @ np.linalg.solve(C, S.T)


def proj(S: np.ndarray, X: np.ndarray, C: np.ndarray | None = None):
    """``b = S C^-1 x^T`` for every row of ``X`` (P x N)."""
    S = np.asarray(S, np.float64)
    X = np.asarray(X, np.float64)
    if C is None:
        return X @ S.T
    return np.linalg.solve(C, X.T).T @ S.T


def simplex_project(V: np.ndarray) -> np.ndarray:
    """Euclidean projection of each row of ``V`` onto {a >= 0, sum a = 1}."""
    V = np.atleast_2d(np.asarray(V, np.float64))
    U = -np.sort(-V, axis=1)
    css = np.cumsum(U, axis=1) - 1.0
    k = np.arange(1, V.shape[1] + 1)
    good = U - css / k > 0
    r = V.shape[1] - np.argmax(good[:, ::-1], axis=1)
    theta = css[np.arange(V.shape[0]), r - 1] / r
    return np.maximum(V - theta[:, None], 0.0)


def natural_residual(G: np.ndarray, B: np.ndarray, A: np.ndarray) -> np.ndarray:
    """``||a - P(a - grad)||_inf`` per pixel for ``1/2 a.Gh a - bh.a`` with
    ``Gh = G / max diag G``; zero exactly at the minimiser."""
    gam = np.max(np.diag(G))
    grad = A @ (G / gam) - B / gam
    return np.abs(A - simplex_project(A - grad)).max(axis=1)


def objective(G, B, A):
    """``a.G a - 2 b.a`` per pixel (eq. 2 up to the constant)."""
    return np.einsum("pi,ij,pj->p", A, G, A) - 2.0 * np.einsum("pi,pi->p", B, A)


def brute_force(G: np.ndarray, B: np.ndarray, tol: float = 1e-12):
    """Exact minimiser for every row of ``B`` by enumerating active sets.

    For each nonempty subset S: solve ``[[G_SS, 1], [1^T, 0]] [a_S; nu] =
    [b_S; 1]``; keep solutions with ``a_S >= -tol``; return the one with the
    smallest criterion, and its multipliers ``lambda = G a - b + nu`` (which
    must be >= 0 for the minimiser).
    """
    G = np.asarray(G, np.float64)
    B = np.atleast_2d(np.asarray(B, np.float64))
    P, N = B.shape
    best = np.full(P, np.inf)
    A = np.zeros((P, N))
    NU = np.zeros(P)
    for r in range(1, N + 1):
        for sub in itertools.combinations(range(N), r):
            s = list(sub)
            K = np.zeros((r + 1, r + 1))
            K[:r, :r] = G[np.ix_(s, s)]
            K[:r, r] = 1.0
            K[r, :r] = 1.0
            if abs(np.linalg.det(K)) < 1e-300:
                continue
            rhs = np.zeros((r + 1, P))
            rhs[:r] = B[:, s].T
            rhs[r] = 1.0
            sol = np.linalg.solve(K, rhs)
            a = np.zeros((P, N))
            a[:, s] = sol[:r].T
            feas = (sol[:r] >= -tol).all(axis=0)
            f = objective(G, B, a)
            take = feas & (f < best - 1e-15 * np.abs(f).clip(1))
            best[take] = f[take]
            A[take] = a[take]
            NU[take] = sol[r][take]  # G_SS a_S + nu 1 = b_S
    # multipliers of a >= 0 in the convention G a - b + nu 1 - lambda = 0
    lam = A @ G - B + NU[:, None]
    return A, lam


def water_filling(g: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Minimiser of ``sum 1/2 g_i a_i^2 - b_i a_i`` on the simplex (g > 0).

    KKT gives ``a_i = max(0, (b_i - theta)/g_i)`` with theta fixed by the
    sum; theta is found exactly by sorting the breakpoints ``b_i``.
    """
    g = np.asarray(g, np.float64)
    b = np.asarray(b, np.float64)
    order = np.argsort(-b)
    bs, gs = b[order], g[order]
    for k in range(1, len(b) + 1):
        theta = (np.sum(bs[:k] / gs[:k]) - 1.0) / np.sum(1.0 / gs[:k])
        if theta < bs[k - 1] and (k == len(b) or theta >= bs[k]):
            return np.maximum(0.0, (b - theta) / g)
    raise AssertionError("no breakpoint interval found")


def two_endmembers(m1: np.ndarray, m2: np.ndarray, y: np.ndarray) -> np.ndarray:
    """N = 2, C = I: ``a = (t, 1-t)`` with t the clipped projection of y onto
    the segment [m2, m1]."""
    d = np.asarray(m1, np.float64) - np.asarray(m2, np.float64)
    t = float(np.dot(d, np.asarray(y, np.float64) - m2) / np.dot(d, d))
    t = min(1.0, max(0.0, t))
    return np.array([t, 1.0 - t])


def scls(G: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Sum-to-one constrained least squares (all coefficients free)."""
    N = G.shape[0]
    K = np.zeros((N + 1, N + 1))
    K[:N, :N] = G
    K[:N, N] = K[N, :N] = 1.0
    sol = np.linalg.solve(K, np.concatenate([b, [1.0]]))
    return sol[:N]


def bordered_cov(G: np.ndarray, free: np.ndarray, s: float) -> np.ndarray:
    """``s^2 [[G_FF, 1],[1^T, 0]]^-1`` upper-left block, zero elsewhere."""
    N = G.shape[0]
    F = np.nonzero(free)[0]
    k = len(F)
    K = np.zeros((k + 1, k + 1))
    K[:k, :k] = G[np.ix_(F, F)]
    K[:k, k] = K[k, :k] = 1.0
    Ki = np.linalg.inv(K)
    out = np.zeros((N, N))
    out[np.ix_(F, F)] = s * s * Ki[:k, :k]
    return out


def disjoint_library(N: int, L: int, rng, equal: bool = False) -> np.ndarray:
    """float32 library whose spectra have disjoint channel supports, so the
    Gram matrix is exactly diagonal (``equal``: exactly c I)."""
    if L < N:
        raise ValueError("need L >= N")
    S = np.zeros((N, L), np.float32)
    width = L // N
    base = rng.integers(1, 64, size=width) / 64.0
    for i in range(N):
        vals = base if equal else rng.integers(1, 64, size=width) / 64.0
        S[i, i * width:(i + 1) * width] = vals
    return S


# ----------------------------------------------------- other constraint sets
# The IPLS options besides sum-to-one: sum-lower-than-one (a >= 0,
# 1^T a <= 1) and positivity only (a >= 0).

def solid_simplex_project(V: np.ndarray) -> np.ndarray:
    """Euclidean projection of each row onto {a >= 0, 1^T a <= 1}: the
    positive part when its sum is at most one, else the projection onto the
    simplex (the sum constraint is then active)."""
    V = np.atleast_2d(np.asarray(V, np.float64))
    Pp = np.maximum(V, 0.0)
    over = Pp.sum(axis=1) > 1.0
    out = Pp.copy()
    if over.any():
        out[over] = simplex_project(V[over])
    return out


def natural_residual_set(G: np.ndarray, B: np.ndarray, A: np.ndarray, constraint: str) -> np.ndarray:
    """Natural residual ``||a - P(a - grad)||_inf`` for the constraint set
    ``"pos"`` (projection = positive part) or ``"slo"`` (solid simplex)."""
    gam = np.max(np.diag(G))
    V = A - (A @ (G / gam) - B / gam)
    Pj = np.maximum(V, 0.0) if constraint == "pos" else solid_simplex_project(V)
    return np.abs(A - Pj).max(axis=1)


def brute_force_pos(G: np.ndarray, B: np.ndarray, tol: float = 1e-12) -> np.ndarray:
    """Exact positivity-only minimiser per row by enumerating the free set S:
    ``G_SS a_S = b_S`` (the empty set gives a = 0); keep feasible solutions
    and return the one with the smallest criterion."""
    G = np.asarray(G, np.float64)
    B = np.atleast_2d(np.asarray(B, np.float64))
    P, N = B.shape
    best = np.zeros(P)  # a = 0
    A = np.zeros((P, N))
    for r in range(1, N + 1):
        for sub in itertools.combinations(range(N), r):
            s = list(sub)
            Gs = G[np.ix_(s, s)]
            if abs(np.linalg.det(Gs)) < 1e-300:
                continue
            sol = np.linalg.solve(Gs, B[:, s].T)
            a = np.zeros((P, N))
            a[:, s] = sol.T
            feas = (sol >= -tol).all(axis=0)
            f = objective(G, B, a)
            take = feas & (f < best - 1e-15 * np.abs(f).clip(1))
            best[take] = f[take]
            A[take] = a[take]
    return A


def objective_gap_bound(S, x, s, l1, pairs, tol_mu=1e-13, tol_d=1e-12):
    """Largest excess of the eq. 2 objective over s^2 at an interior iterate
    that met the stopping tests, over the least value.  For the convex QP,
    q(a) - q(a*) <= grad q(a)^T (a - a*) = r_d^T (a - a*) + lam^T a
    - lam^T a* - nu (1^T a - 1^T a*), with lam^T a* >= 0; so the scaled gap is
    at most pairs mu + ||r_d||_inf ||a - a*||_1 (plus nu r_p, of the order of
    tol_p times a unit multiplier, folded into the slack).  ``l1`` bounds
    ||a - a*||_1; the objective is 2 gamma q / s^2 plus a constant."""
    Sd = np.asarray(S, np.float64)
    gam = float((Sd * Sd).sum(1).max())
    bh = np.abs(Sd @ np.asarray(x, np.float64)).max() / gam
    q = pairs * tol_mu + tol_d * (1.0 + bh) * l1 + 1e-13
    return 2.0 * gam * q / float(s) ** 2
