"""The pins have teeth: plausible mistakes planted in a copy of the oracle's C
source (on the CPU only) must each fail at least one pin.

Each mutant is a one-line textual change of ``oracle/linmin_oracle.c`` built
into a temporary library; the unmodified source must pass the same checks.
"""
import os

import numpy as np
import pytest

import oracle
import pins
from paper_1402_2518_amd import synth

MUTANTS = {
    "dual residual drops nu": ("double v = -bh[i] - lam[i] + nu;", "double v = -bh[i] - lam[i];"),
    "wrong sign of r_p in dnu": ("*dnu = (sw + rp) / su;", "*dnu = (sw - rp) / su;"),
    "dl drops the D da term": ("dl[i] = -rc[i] / a[i] - W->D[i] * da[i];", "dl[i] = -rc[i] / a[i];"),
    "unscaled projection": ("bh[i] = s / gam;", "bh[i] = s;"),
    "covariance without u u^T": ("scale * (W->tmp[p] - W->u[p] * W->u[q] * corner_inv);", "scale * (W->tmp[p]);"),
    "covariance scaled by s not s^2": ("double scale = (double)sig * sig / gam;", "double scale = (double)sig / gam;"),
    "objective drops the factor 2": ("(c - 2.0 * ba + q)", "(c - ba + q)"),
    "finishing step accepts any partition": ("if (worst_a < 0 && worst_l < 0) {", "if (1) {"),
    "renormalised pixel uses Lc transposed": ("for (int l = j; l < L; ++l) s += (double)x[l] * Lc[l * L + j];",
                                              "for (int l = j; l < L; ++l) s += (double)x[l] * Lc[j * L + l];"),
    "corrector safeguard removed": ("const double soc = t_aff >= 0.1 ? 1.0 : 0.0;", "const double soc = 1.0;"),
    "gram transposed index": ("for (int j = 0; j < N; ++j) v += Gh[i * N + j] * a[j];",
                              "for (int j = 0; j < N; ++j) v += Gh[i * N + j] * a[i];"),
    "slack corner dropped from dnu": ("else if (cons == LO_SLO) *dnu = (sw + rp - rcs / nu) / (su + s / nu);",
                                      "else if (cons == LO_SLO) *dnu = (sw + rp - rcs / nu) / su;"),
    "positivity only finishes with the sum row": ("int certified = 0, slack_free = pos;",
                                                  "int certified = 0, slack_free = 0;"),
    "free slack keeps the sum row": ("*nu = bordered ? (sw - 1.0) / su : 0.0;", "*nu = (sw - 1.0) / su;"),
    "uncertified covariance drops the slack corner": (
        "if (bordered) corner_inv = 1.0 / (su + ((slo && !certified) ? s / nu : 0.0));",
        "if (bordered) corner_inv = 1.0 / su;"),
}


def pin_failures(lib):
    """Run a compact set of pins against the library at ``lib``; return the
    names of those that fail (an exception counts as a failure)."""
    out = []

    def check(name, fn):
        try:
            with np.errstate(all="ignore"):
                if not fn():
                    out.append(name)
        except Exception:
            out.append(name)

    w = synth.WORKLOADS["orbital"]
    S = synth.make_library(w)
    X, s = synth.make_cube(w, p1=150)
    r = oracle.unmix(S, X, s, lib=lib)
    G, B = pins.gram(S), pins.proj(S, X)
    check("kkt", lambda: pins.natural_residual(G, B, r["a"]).max() <= 1e-10)
    bad = oracle.MAXIT | oracle.NOT_PD | oracle.INEXACT
    check("converged and certified", lambda: not (r["status"] & bad).any() and r["iters"].max() < 40)
    from test_oracle import cycling_pixels
    Sc_, Xc_, sc_ = cycling_pixels()
    rcy = oracle.unmix(Sc_, Xc_, sc_, cov=False, lib=lib)
    check("no cycling", lambda: not (rcy["status"] & bad).any())
    check("sum", lambda: np.abs(r["a"].sum(1) - 1).max() <= 1e-13)
    res = X.astype(float) - r["a"] @ S.astype(float)
    check("objective", lambda: np.abs(r["F"] / ((res ** 2).sum(1) / s.astype(float) ** 2) - 1).max() <= 1e-8)
    check("cov rows sum to 0", lambda: all(np.abs(c.sum(1)).max() <= 1e-8 * np.abs(c).max() for c in r["cov"]))

    wt = synth.WORKLOADS["tiny"]
    St = synth.make_library(wt)
    Xt, st = synth.make_cube(wt, p1=100)
    rt = oracle.unmix(St, Xt, st, lib=lib)
    Gt = pins.gram(St)
    check("brute force", lambda: np.abs(rt["a"] - pins.brute_force(Gt, pins.proj(St, Xt))[0]).max() <= 1e-9)

    def cov_ok():
        for p in range(len(Xt)):
            if rt["status"][p]:
                continue
            want = pins.bordered_cov(Gt, rt["a"][p] > rt["lam"][p], float(st[p]))
            if np.abs(rt["cov"][p] - want).max() > 1e-8 * np.abs(want).max() + 1e-18:
                return False
        return True
    check("covariance", cov_ok)

    rng = np.random.default_rng(23)
    N, L = 5, 30
    Sc = synth.mineral_spectra(N, L, rng).astype(np.float32)
    Q = rng.standard_normal((L, L))
    C = Q @ Q.T / L + np.diag(rng.uniform(0.5, 2.0, L))
    Xc = (rng.dirichlet(np.ones(N), 40) @ Sc.astype(float) + 0.01 * rng.standard_normal((40, L))).astype(np.float32)
    rc = oracle.unmix(Sc, Xc, None, C=C, lib=lib)
    ev, V = np.linalg.eigh(C)
    Wh = V @ np.diag(ev ** -0.5) @ V.T
    Sw, Xw = Sc.astype(float) @ Wh, Xc.astype(float) @ Wh
    check("renormalisation", lambda: np.abs(rc["a"] - pins.brute_force(Sw @ Sw.T, Xw @ Sw.T)[0]).max() <= 1e-9)

    # the other constraint options on mixtures whose sums straddle one
    rng = np.random.default_rng(31)
    N, L = 6, 40
    Sk = rng.uniform(0.05, 1.0, (N, L)).astype(np.float32)
    Ak = rng.dirichlet(np.ones(N), 60) * rng.uniform(0.6, 1.4, (60, 1))
    Xk = (Ak @ Sk.astype(float) + 0.01 * rng.standard_normal((60, L))).astype(np.float32)
    Gk, Bk = pins.gram(Sk), pins.proj(Sk, Xk)
    a_pos = pins.brute_force_pos(Gk, Bk)
    rp_ = oracle.unmix(Sk, Xk, None, cov=False, constraint=oracle.POS, lib=lib)
    check("positivity only", lambda: np.abs(rp_["a"] - a_pos).max() <= 1e-9)
    rs_ = oracle.unmix(Sk, Xk, None, cov=False, constraint=oracle.SLO, lib=lib)
    want = np.where((a_pos.sum(1) <= 1.0)[:, None], a_pos, pins.brute_force(Gk, Bk)[0])
    check("sum lower than one", lambda: np.abs(rs_["a"] - want).max() <= 1e-9)
    r3 = oracle.unmix(Sk[:5], Xk[:10], None, constraint=oracle.SLO, maxit=3, lib=lib)

    def corner_ok():
        Gc = pins.gram(Sk[:5])
        gam = Gc.diagonal().max()
        for p in range(10):
            a, lam, nu = r3["a"][p], r3["lam"][p], r3["nu"][p]
            H = Gc / gam + np.diag(lam / a)
            K = np.block([[H, np.ones((5, 1))], [np.ones((1, 5)), np.array([[-(1.0 - a.sum()) / nu]])]])
            want_c = np.linalg.inv(K)[:5, :5] / gam
            if np.abs(r3["cov"][p] - want_c).max() > 1e-9 * np.abs(want_c).max():
                return False
        return True
    check("slack corner covariance", corner_ok)
    return out


@pytest.fixture(scope="module")
def builddir(tmp_path_factory):
    return tmp_path_factory.mktemp("mutants")


def test_unmodified_source_passes(builddir):
    lib = oracle.build(force=True, src=oracle.SRC, out=str(builddir / "clean.so"))
    assert pin_failures(lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(builddir, name):
    old, new = MUTANTS[name]
    with open(oracle.SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site not unique/present: {old}"
    path = builddir / (name.replace(" ", "_").replace("^", "") + ".c")
    path.write_text(src.replace(old, new))
    lib = oracle.build(force=True, src=str(path), out=str(path) + ".so")
    failed = pin_failures(lib)
    assert failed, f"mutant '{name}' passed every pin"
