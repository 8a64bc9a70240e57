"""The additional spectra of Sec. 2.5 (named in the table after the
references): pins of the oracle's builder, the C-ABI builder against it,
and the oracle on the rank-deficient libraries these spectra make.

The pins are properties the paper's description fixes without restating the
formulas: the four span level and slope only (rank 2), the twelve add one
cosine/sine pair per period (rank 6), a quarter-cycle curve has no extremum
inside the domain and a half-cycle one exactly one, each +/- pair cancels,
and the position along the domain does not depend on the wavelength units.
"""
import numpy as np
import pytest
from scipy.optimize import nnls

import oracle
import pins
from paper_1402_2518_amd import linmin, synth


@pytest.mark.parametrize("L", [2, 65, 240])
def test_four_extras_span_level_and_slope(L):
    E = oracle.extra_spectra(L, 4)
    assert E.shape == (4, L)
    assert np.linalg.matrix_rank(E) == 2
    flat1, flat0, up, down = E
    assert (flat1 == 1.0).all() and np.allclose(flat0, 1e-4 * flat1, rtol=0, atol=1e-18)
    assert np.abs(up + down - flat1).max() <= 1e-15  # the two slopes sum to the unit level
    assert up[0] == 0.0 and up[-1] == 1.0 and down[0] == 1.0 and down[-1] == 0.0
    if L > 2:
        assert np.abs(np.diff(up, 2)).max() <= 1e-15  # linear in the channel on an even grid
    assert (np.diff(up) > 0).all() and (np.diff(down) < 0).all()


@pytest.mark.parametrize("L", [65, 241])
def test_twelve_extras_periods_and_signs(L):
    E = oracle.extra_spectra(L, 12)
    assert E.shape == (12, L)
    assert np.array_equal(E[:4], oracle.extra_spectra(L, 4))
    assert np.linalg.matrix_rank(E) == 6
    for k, cycles in ((0, 0.25), (1, 0.5)):
        c, s, nc, ns = E[4 + 4 * k: 8 + 4 * k]
        assert np.abs(c + nc).max() == 0 and np.abs(s + ns).max() == 0
        assert np.abs(c * c + s * s - 1).max() <= 1e-15
        assert abs(c[0] - 1) <= 1e-15 and abs(s[0]) <= 1e-15
        if cycles == 0.25:
            # a quarter cycle: cosine falls 1 -> 0 and sine rises 0 -> 1, both monotone
            assert abs(c[-1]) <= 1e-15 and abs(s[-1] - 1) <= 1e-15
            assert (np.diff(c) < 0).all() and (np.diff(s) > 0).all()
        else:
            # half a cycle: cosine runs 1 -> -1 with one zero crossing, sine
            # returns to zero with its single maximum in the middle
            assert abs(c[-1] + 1) <= 1e-15 and abs(s[-1]) <= 1e-15
            assert (np.diff(c) < 0).all() and (np.diff(np.sign(c)) != 0).sum() in (1, 2)
            assert int(np.argmax(s)) == (L - 1) // 2 and abs(s.max() - 1) <= 1e-3


def test_wavelength_grid():
    rng = np.random.default_rng(4)
    wl = np.cumsum(rng.uniform(0.5, 3.0, 120)) + 900.0
    E = oracle.extra_spectra(120, 12, wl)
    # the position along the domain is affine-invariant in the wavelengths
    assert np.abs(E - oracle.extra_spectra(120, 12, 1e-3 * wl - 7.0)).max() <= 1e-12
    # an even grid reproduces the channel-index form
    assert np.abs(oracle.extra_spectra(120, 12, np.linspace(1.0, 2.5, 120)) -
                  oracle.extra_spectra(120, 12)).max() <= 1e-12
    # on an uneven grid the slopes are linear in the wavelength, not in the
    # channel index
    rate = np.diff(E[2]) / np.diff(wl)
    assert np.abs(rate / rate.mean() - 1).max() <= 1e-10
    assert np.abs(np.diff(E[2], 2)).max() > 1e-4


def _ulps(a, b):
    a = np.ascontiguousarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.ascontiguousarray(b, np.float32).view(np.int32).astype(np.int64)
    return int(np.abs(a - b).max())


@pytest.mark.parametrize("L,n", [(2, 4), (64, 4), (240, 12), (438, 12)])
def test_c_abi_builder_matches_oracle(L, n):
    assert _ulps(linmin.extra_spectra(L, n), oracle.extra_spectra(L, n)) <= 1


def test_c_abi_builder_on_a_wavelength_grid():
    rng = np.random.default_rng(9)
    wl = np.cumsum(rng.uniform(0.5, 3.0, 240)) + 400.0
    assert _ulps(linmin.extra_spectra(240, 12, wl), oracle.extra_spectra(240, 12, wl)) <= 1


def test_c_abi_builder_rejects_bad_arguments():
    for L, n in ((1, 4), (64, 5), (64, 0)):
        with pytest.raises(linmin.LinminError) as e:
            linmin.extra_spectra(L, n)
        assert e.value.code == linmin.EINVAL
    wl = np.linspace(1.0, 2.0, 16)
    wl[7] = wl[6]
    with pytest.raises(linmin.LinminError):
        linmin.extra_spectra(16, 4, wl)
    wl[7] = np.nan
    with pytest.raises(linmin.LinminError):
        linmin.extra_spectra(16, 4, wl)


def _nnls_objective(S, x, s, cons):
    """Least objective of eq. 2 (over s^2) under the constraint option, by
    NNLS: positivity exactly; the sum row as an equation weighted 1e5."""
    Sd = S.astype(float)
    ap, _ = nnls(Sd.T, x, maxiter=5000)
    if cons == oracle.POS or (cons == oracle.SLO and ap.sum() <= 1.0):
        a = ap
    else:
        W = 1e5
        a, _ = nnls(np.vstack([Sd.T, W * np.ones((1, len(S)))]), np.concatenate([x, [W]]), maxiter=5000)
    return float(((x - a @ Sd) ** 2).sum()) / float(s) ** 2, a


@pytest.mark.parametrize("n", [4, 12])
@pytest.mark.parametrize("cons", [oracle.STO, oracle.SLO, oracle.POS])
def test_oracle_on_the_paper_extra_library(n, cons):
    """The minimiser may be non-unique on these libraries but the least
    objective is not.  Certified pixels reach it to rounding; the others are
    interior iterates that met the stopping tests, whose excess is bounded
    by the complementarity gap and the dual residual."""
    w = synth.WORKLOADS["orbital"]
    M = synth.mineral_spectra(32, w.L, np.random.default_rng(5))
    S = np.concatenate([M, oracle.extra_spectra(w.L, n)]).astype(np.float32)
    X, s = synth.make_cube(w, p1=24)
    r = oracle.unmix(S, X, s, constraint=cons, cov=False)
    pairs = len(S) + (1 if cons == oracle.SLO else 0)
    for p in range(len(X)):
        F, a_ref = _nnls_objective(S, X[p].astype(float), s[p], cons)
        gap = r["F"][p] - F
        slack = 1e-8 * F  # rounding, and the weighted sum row of the reference
        if r["status"][p] & oracle.INEXACT:
            bound = pins.objective_gap_bound(S, X[p], s[p], r["a"][p].sum() + a_ref.sum(), pairs)
            assert -slack <= gap <= bound + slack
        else:
            assert abs(gap) <= slack
