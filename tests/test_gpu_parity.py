"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Element-by-element comparisons on seeded inputs that span several workgroups
and a ragged tail, plus the edge cases of the method.  Tolerances (derived in
the design doc): coefficients 1e-6 absolute for FP64 and 1e-3 for the mixed form
(its FP64 finishing step brings it to the FP64 level in practice); covariance
1e-6 relative to its largest entry on certified non-degenerate pixels;
objective 1e-9 relative (FP64) / 1e-4 relative (mixed).
"""
import os
import sys

import numpy as np
import pytest

import oracle
import pins
from paper_1402_2518_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1402_2518_amd import linmin
    linmin.load()
    return torch.device("cuda:0")


def _gpu(S, X, s, dev, C=None, precision="fp64", cov="full", **opts):
    from paper_1402_2518_amd import linmin
    lib = linmin.Library(S, C)
    Xt = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(dev)
    st = None if s is None else torch.from_numpy(np.ascontiguousarray(s, np.float32)).to(dev)
    out = lib.unmix(Xt, st, precision=precision, cov=cov, **opts)
    torch.cuda.synchronize()
    res = {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}
    res["gamma"] = lib.gamma
    res["sigma"] = np.ones(len(X)) if s is None else np.asarray(s, np.float64)
    lib.close()
    return res


def _certificate(S, X, C, constraint, A):
    """KKT natural residual of coefficients A (rows of X): zero exactly at
    the minimiser of the problem, computed by the independent pins."""
    G, B = pins.gram(S, C), pins.proj(S, X, C)
    if constraint == "sto":
        return pins.natural_residual(G, B, A)
    return pins.natural_residual_set(G, B, A, constraint)


def _compare(g, r, S, X, C=None, constraint="sto", a_tol=1e-6, cov_tol=1e-6, f_tol=1e-9, check_cov=True):
    """Element-by-element comparison of a GPU result with the oracle's.

    Statuses must agree exactly (the DEGENERATE bit aside: it is a threshold
    tie-break between two valid readings).  The one exception is a pixel
    that one side certified while the other ended on an uncertified interior
    iterate (INEXACT): both iterates met the same stopping tests, and on an
    ill-conditioned free set the finishing step may certify one and not the
    other.  Such a pixel passes only with a proof: the certified side's
    coefficients have a KKT natural residual of at most 1e-10 (they are the
    minimiser), and the uncertified side's objective exceeds the certified
    one by no more than the bound on an interior iterate that met the
    stopping tests (complementarity gap plus dual residual times the
    distance to the minimiser); the coefficient tolerance applies to the
    pixels whose statuses agree."""
    assert np.isfinite(g["a"]).all()
    ok = (g["status"] == 0) & (r["status"] == 0)
    assert ok.mean() > 0.95, np.bincount(g["status"])
    mask = ~np.uint8(oracle.DEGENERATE)
    gs, rs = g["status"] & mask, r["status"] & mask
    same = gs == rs
    one_certified = ((gs == 0) & (rs == oracle.INEXACT)) | ((gs == oracle.INEXACT) & (rs == 0))
    # coefficients where the statuses agree; a pixel certified on one side
    # only is judged by the proof below (its uncertified side is an interior
    # iterate, which may lie farther from the minimiser than the tolerance
    # along a nearly flat direction of the objective)
    da = np.abs(g["a"] - r["a"])[same].max() if same.any() else 0.0
    assert da <= a_tol, f"max |a_gpu - a_oracle| = {da}"
    diff = np.flatnonzero(~same)
    info = [(int(i), int(g["status"][i]), int(r["status"][i]), int(g["iters"][i]), int(r["iters"][i]),
             float(np.abs(g["a"][i] - r["a"][i]).max())) for i in diff[:8]]
    assert (same | one_certified).all(), info
    if len(diff):
        assert C is None, ("status mismatch with a noise covariance", info)
        gcert = gs[diff] == 0
        Acert = np.where(gcert[:, None], g["a"][diff], r["a"][diff])
        Aunc = np.where(gcert[:, None], r["a"][diff], g["a"][diff])
        kkt = _certificate(S, X[diff], C, constraint, Acert)
        assert kkt.max() <= 1e-10, ("certified side is not the minimiser", info, kkt)
        Fc = np.where(gcert, g["objective"][diff], r["F"][diff])
        Fu = np.where(gcert, r["F"][diff], g["objective"][diff])
        pairs = S.shape[0] + (1 if constraint == "slo" else 0)
        for j, i in enumerate(diff):
            l1 = float(np.abs(Aunc[j] - Acert[j]).sum())
            bound = pins.objective_gap_bound(S, X[i], g["sigma"][i], l1, pairs)
            assert Fc[j] <= Fu[j] * (1 + f_tol), (info, Fc[j], Fu[j])
            assert Fu[j] - Fc[j] <= bound + f_tol * abs(Fc[j]), (info, Fu[j] - Fc[j], bound)
        _say(f"[gpu]   certified on one side only: {len(diff)} of {len(gs)} pixels "
             f"(GPU certified {int(gcert.sum())}), each with a KKT certificate")
    dF = np.abs(g["objective"][same] / r["F"][same] - 1).max()
    assert dF <= f_tol, f"objective rel err {dF}"
    if check_cov and g["cov"] is not None:
        cg, cr = g["cov"][ok], r["cov"][ok]
        # relative to the pixel's largest entry, floored at the natural scale
        # s^2 / gamma (a single free coefficient has an all-zero covariance)
        nat = g["sigma"][ok] ** 2 / g["gamma"]
        scale = np.maximum(np.abs(cr).reshape(len(cr), -1).max(1), nat)[:, None, None]
        dc = (np.abs(cg - cr) / scale).max() if len(cg) else 0.0
        assert dc <= cov_tol, f"cov rel err {dc}"
    return da


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tiny_workload_parity(dev, precision):
    _say(f"[gpu] tiny workload 1000 px N=8 {precision}")
    w = synth.WORKLOADS["tiny"]
    S = synth.make_library(w)
    X, s = synth.make_cube(w)
    g = _gpu(S, X, s, dev, precision=precision)
    r = oracle.unmix(S, X, s)
    _compare(g, r, S, X, a_tol=1e-6 if precision == "fp64" else 1e-3,
             f_tol=1e-9 if precision == "fp64" else 1e-4)
    # and against enumeration of every active set
    a_bf, _ = pins.brute_force(pins.gram(S), pins.proj(S, X))
    assert np.abs(g["a"] - a_bf).max() <= 1e-6


@pytest.mark.parametrize("name,n", [("orbital", 3001), ("precision", 403)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_workload_samples_parity(dev, name, n, precision):
    _say(f"[gpu] {name} first {n} px {precision}")
    w = synth.WORKLOADS[name]
    S = synth.make_library(w)
    X, s = synth.make_cube(w, p1=n)
    g = _gpu(S, X, s, dev, precision=precision)
    r = oracle.unmix(S, X, s)
    _compare(g, r, S, X, a_tol=1e-6 if precision == "fp64" else 1e-3,
             f_tol=1e-9 if precision == "fp64" else 1e-4)
    _say(f"[gpu]   iters gpu mean {g['iters'].mean():.2f} oracle {r['iters'].mean():.2f}")


@pytest.mark.parametrize("N", [1, 2, 5, 16, 24, 31, 40, 48, 57, 64, 80, 96, 100, 128])
def test_library_sizes(dev, N):
    _say(f"[gpu] library size N={N}")
    w = synth.custom_workload(N, max(N, 96) if N <= 64 else (128 if N <= 96 else 160), 517, seed=N, n_extra=min(4, N - 1) if N > 1 else 0,
                              k_max=max(1, min(4, N - 4)) if N > 4 else 1)
    S = synth.make_library(w)
    X, s = synth.make_cube(w)
    for precision in ("fp64", "mixed"):
        g = _gpu(S, X, s, dev, precision=precision)
        r = oracle.unmix(S, X, s)
        _compare(g, r, S, X, a_tol=1e-6 if precision == "fp64" else 1e-3,
                 f_tol=1e-9 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("N", [8, 21, 36, 45, 64, 90, 128])
def test_fp32_stage_kernel_families(dev, N):
    """The mixed form's FP32 stage on each kernel family compiled for the
    size (the 4x4x1 matrix-core tiles, sixteen pixels per wavefront up to
    N = 36 and column-cyclic above, and the lane groups): both hand an
    iterate to the same FP64 stage, so both must meet the oracle."""
    from paper_1402_2518_amd import linmin
    _say(f"[gpu] FP32 stage kernel families N={N}")
    w = synth.custom_workload(N, max(96, N + 8), 1203 if N <= 64 else 397, seed=700 + N, n_extra=4, k_max=4)
    S = synth.make_library(w)
    X, s = synth.make_cube(w)
    r = oracle.unmix(S, X, s)
    before = linmin.get_kernel_lanes(N, linmin.STAGE_FP32)
    try:
        for fam in ("tile32", "group"):
            linmin.set_kernel(N, linmin.STAGE_FP32, fam)
            assert linmin.get_kernel(N, linmin.STAGE_FP32) == linmin.KERNELS[fam]
            g = _gpu(S, X, s, dev, precision="mixed")
            _compare(g, r, S, X, a_tol=1e-3, f_tol=1e-4)
            _say(f"[gpu]   {fam}: iters {g['iters'].mean():.2f}")
    finally:
        linmin.set_kernel(N, linmin.STAGE_FP32, *before)


@pytest.mark.parametrize("N", [50, 64])
def test_fp64_kernel_families(dev, N):
    """The FP64 path on each matrix-core layout compiled for the size (the
    four-pixel tiles and the row-cyclic tiles of a pixel over two blocks), in
    both precisions (the FP64 kernel is also the mixed form's second stage
    and its retry): each must meet the oracle."""
    from paper_1402_2518_amd import linmin
    _say(f"[gpu] FP64 kernel families N={N}")
    w = synth.custom_workload(N, 2 * N, 611, seed=900 + N, n_extra=4, k_max=4)
    S = synth.make_library(w)
    X, s = synth.make_cube(w)
    r = oracle.unmix(S, X, s)
    before = linmin.get_kernel_lanes(N, linmin.STAGE_FP64)
    try:
        for fam in ("rowcyclic", "tile"):
            linmin.set_kernel(N, linmin.STAGE_FP64, fam)
            for precision in ("fp64", "mixed"):
                g = _gpu(S, X, s, dev, precision=precision)
                _compare(g, r, S, X, a_tol=1e-6 if precision == "fp64" else 1e-3,
                         f_tol=1e-9 if precision == "fp64" else 1e-4)
                _say(f"[gpu]   {fam} {precision}: iters {g['iters'].mean():.2f}")
    finally:
        linmin.set_kernel(N, linmin.STAGE_FP64, *before)


def test_mixed_retry_reproduces_fp64(dev):
    """The mixed form solves again in FP64 every pixel whose finishing step
    did not certify after the hand-over, so a pixel that the mixed form
    reports uncertified carries exactly the FP64 path's outputs (same
    kernel, same inputs), bit for bit; on this sum-lower-than-one mixture at
    N = 64, with the hand-over at 1e-8, pixels that the FP64 path cannot
    certify are left uncertified by the mixed form's FP64 steps as well.
    Every other pixel meets the oracle within the mixed tolerances."""
    _say("[gpu] mixed-form retry pass, N = 64 sum-lower-than-one")
    S, X, s = _straddling(64, 128, 403, seed=164)
    g64 = _gpu(S, X, s, dev, precision="fp64", constraint="slo")
    gmx = _gpu(S, X, s, dev, precision="mixed", constraint="slo", mu_switch=1e-8)
    unc = (gmx["status"] & (oracle.INEXACT | oracle.MAXIT | oracle.NOT_PD)) != 0
    assert unc.any()
    for key in ("a", "status", "iters", "objective"):
        assert np.array_equal(np.nan_to_num(gmx[key][unc], nan=3.5), np.nan_to_num(g64[key][unc], nan=3.5)), key
    r = oracle.unmix(S, X, s, constraint=oracle.SLO)
    _compare(gmx, r, S, X, constraint="slo", a_tol=1e-3, f_tol=1e-4)
    _say(f"[gpu]   {int(unc.sum())} uncertified pixels equal to the FP64 path")


def test_cycling_pixels_converge(dev):
    _say("[gpu] orbital pixels that make plain Mehrotra cycle")
    from test_oracle import cycling_pixels
    S, X, s = cycling_pixels()
    for precision in ("fp64", "mixed"):
        g = _gpu(S, X, s, dev, precision=precision)
        r = oracle.unmix(S, X, s)
        assert (g["status"] & ~np.uint8(oracle.DEGENERATE) == 0).all(), g["status"]
        assert np.abs(g["a"] - r["a"]).max() <= 1e-6


def test_ragged_and_empty(dev):
    _say("[gpu] ragged pixel counts and P=0")
    w = synth.WORKLOADS["orbital"]
    S = synth.make_library(w)
    X, s = synth.make_cube(w, p1=40)
    r = oracle.unmix(S, X, s)
    for P in (1, 2, 15, 17, 33):
        g = _gpu(S, X[:P], s[:P], dev)
        assert np.abs(g["a"] - r["a"][:P]).max() <= 1e-6
    g = _gpu(S, X[:0], s[:0], dev)
    assert g["a"].shape == (0, S.shape[0])


def test_edge_pixels_are_isolated(dev):
    _say("[gpu] NaN/Inf spectra and bad sigma")
    w = synth.WORKLOADS["orbital"]
    S = synth.make_library(w)
    X, s = synth.make_cube(w, p1=64)
    X = X.copy()
    s = s.copy()
    X[3, 7] = np.nan
    X[20, 0] = np.inf
    s[5] = 0.0
    s[6] = -1.0
    s[7] = np.nan
    g = _gpu(S, X, s, dev)
    r = oracle.unmix(S, X, s)
    assert g["status"][3] & oracle.NONFINITE and g["status"][20] & oracle.NONFINITE
    assert np.isnan(g["a"][3]).all() and np.isnan(g["cov"][20]).all()
    for i in (5, 6, 7):
        assert g["status"][i] & oracle.BAD_SIGMA
        assert np.isnan(g["objective"][i]) and np.isnan(g["cov"][i]).all()
    good = [i for i in range(64) if i not in (3, 20)]
    assert np.abs(g["a"][good] - r["a"][good]).max() <= 1e-6
    # neighbours are bit-identical to a run without the bad pixels
    clean = np.delete(np.arange(64), [3, 20])
    g2 = _gpu(S, X[clean], s[clean], dev)
    assert np.array_equal(g2["a"], g["a"][clean])


def test_closed_forms_on_gpu(dev):
    _say("[gpu] identity Gram, N=2 segment, N=1")
    rng = np.random.default_rng(7)
    S = pins.disjoint_library(36, 240, rng, equal=True)
    X = (rng.uniform(0, 1, (300, 240)) * 0.5).astype(np.float32)
    g = _gpu(S, X, None, dev)
    c = pins.gram(S)[0, 0]
    assert np.abs(g["a"] - pins.simplex_project(pins.proj(S, X) / c)).max() <= 1e-10
    S2 = rng.uniform(0.1, 0.6, (2, 50)).astype(np.float32)
    X2 = rng.uniform(0.0, 0.7, (100, 50)).astype(np.float32)
    g2 = _gpu(S2, X2, None, dev)
    want = np.array([pins.two_endmembers(S2[0].astype(float), S2[1].astype(float), x.astype(float)) for x in X2])
    assert np.abs(g2["a"] - want).max() <= 1e-9
    S1 = S2[:1]
    g1 = _gpu(S1, X2, np.full(100, 0.01, np.float32), dev)
    assert np.all(g1["a"] == 1.0) and np.all(g1["cov"] == 0.0)


def test_covariance_layouts_agree(dev):
    _say("[gpu] covariance layouts")
    w = synth.WORKLOADS["orbital"]
    S = synth.make_library(w)
    X, s = synth.make_cube(w, p1=200)
    full = _gpu(S, X, s, dev, cov="full")["cov"]
    packed = _gpu(S, X, s, dev, cov="packed")["cov"]
    diag = _gpu(S, X, s, dev, cov="diag")["cov"]
    N = S.shape[0]
    il = np.tril_indices(N)
    assert np.array_equal(packed, full[:, il[0], il[1]])
    assert np.array_equal(diag, np.diagonal(full, axis1=1, axis2=2))
    g = _gpu(S, X, s, dev, cov=None)
    assert g["cov"] is None


def test_noise_covariance(dev):
    _say("[gpu] full noise covariance (eqs. 5-6)")
    rng = np.random.default_rng(23)
    N, L = 12, 100
    S = synth.mineral_spectra(N, L, rng).astype(np.float32)
    Q = rng.standard_normal((L, L))
    C = (Q @ Q.T / L + np.diag(rng.uniform(0.5, 2.0, L))) * 1e-4
    X = (rng.dirichlet(np.ones(N), 300) @ S.astype(float) + 0.01 * rng.standard_normal((300, L))).astype(np.float32)
    s = rng.uniform(0.5, 2.0, 300).astype(np.float32)
    g = _gpu(S, X, s, dev, C=C)
    r = oracle.unmix(S, X, s, C=C)
    _compare(g, r, S, X, C=C)


def test_noise_free_exact_recovery(dev):
    _say("[gpu] dyadic exact recovery")
    rng = np.random.default_rng(11)
    N, L = 8, 64
    S = (rng.integers(1, 256, (N, L)) / 256.0).astype(np.float32)
    A = np.zeros((40, N))
    for p in range(40):
        idx = rng.choice(N, 3, replace=False)
        A[p, idx] = (0.5, 0.25, 0.25)
    X = (A @ S.astype(np.float64)).astype(np.float32)
    g = _gpu(S, X, np.full(40, 0.01, np.float32), dev)
    assert np.abs(g["a"] - A).max() <= 1e-9


def _cov_rel_err(g, r, mask):
    cg, cr = g["cov"][mask], r["cov"][mask]
    nat = g["sigma"][mask] ** 2 / g["gamma"]
    scale = np.maximum(np.abs(cr).reshape(len(cr), -1).max(1), nat)[:, None, None]
    return (np.abs(cg - cr) / scale).max() if len(cg) else 0.0


def test_covariance_large_free_sets(dev):
    """Free sets above 15 coefficients (and uncertified pixels, whose
    covariance spans every index) go through the one-wavefront-per-pixel
    covariance path; the small path takes the rest of the same cube."""
    _say("[gpu] covariance of large free sets N=40")
    w = synth.custom_workload(40, 160, 300, seed=77, n_extra=4, k_max=30, sigma=(1e-4, 2e-4))
    S = synth.make_library(w)
    X, s = synth.make_cube(w)
    g = _gpu(S, X, s, dev, cov="full")
    r = oracle.unmix(S, X, s)
    ok = (g["status"] == 0) & (r["status"] == 0)
    free = (r["a"] > 0).sum(1)
    assert (ok & (free > 15)).sum() >= 50, (ok.sum(), np.bincount(free))
    assert (ok & (free <= 15)).sum() >= 5
    assert np.abs(g["a"][ok] - r["a"][ok]).max() <= 1e-6
    assert _cov_rel_err(g, r, ok) <= 1e-6
    # the same layouts from both paths
    N = S.shape[0]
    packed = _gpu(S, X, s, dev, cov="packed")["cov"]
    diag = _gpu(S, X, s, dev, cov="diag")["cov"]
    il = np.tril_indices(N)
    assert np.array_equal(packed, g["cov"][:, il[0], il[1]])
    assert np.array_equal(diag, np.diagonal(g["cov"], axis1=1, axis2=2))
    # stopped after three iterations: every pixel uncertified, covariance from
    # the last iterate's Gh + diag(lambda / a) over all 40 coefficients
    g3 = _gpu(S, X, s, dev, cov="full", maxit=3)
    r3 = oracle.unmix(S, X, s, maxit=3)
    assert (g3["status"] == oracle.MAXIT).all() and (r3["status"] == oracle.MAXIT).all()
    assert np.abs(g3["a"] - r3["a"]).max() <= 1e-9
    assert _cov_rel_err(g3, r3, np.ones(len(X), bool)) <= 1e-6


@pytest.mark.parametrize("N", [96, 128])
def test_covariance_above_64_coefficients(dev, N):
    """Covariances over more than 64 coefficients reach the upper columns of
    the one-wavefront-per-pixel sweep (a lane's second column).  Two cases:
    certified free sets of 78..N coefficients (a library of disjoint channel
    supports, near-uniform mixtures with some spectra dropped), and every
    pixel of a mineral workload stopped after three iterations (uncertified:
    the covariance of the last iterate spans all N coefficients)."""
    _say(f"[gpu] covariance above 64 coefficients N={N}")
    rng = np.random.default_rng(N)
    L, P = 2 * N, 64
    S = pins.disjoint_library(N, L, rng)
    wts = rng.dirichlet(np.full(N, 50.0), P)
    for p in range(P):
        wts[p, rng.choice(N, rng.integers(0, N - 64), replace=False)] = 0.0
    wts /= wts.sum(1, keepdims=True)
    X = (wts @ S.astype(float) + 1e-4 * rng.standard_normal((P, L))).astype(np.float32)
    s = rng.uniform(0.5, 2.0, P).astype(np.float32)
    r = oracle.unmix(S, X, s)
    free = (r["a"] > 0).sum(1)
    assert (r["status"] == 0).all() and free.min() > 64, (np.bincount(r["status"]), free.min())
    for cov in ("full", "packed"):
        g = _gpu(S, X, s, dev, cov=cov)
        assert (g["status"] == 0).all(), g["status"]
        assert np.abs(g["a"] - r["a"]).max() <= 1e-9
        if cov == "full":
            assert _cov_rel_err(g, r, np.ones(P, bool)) <= 1e-6
        else:
            il = np.tril_indices(N)
            gf = {"cov": np.zeros((P, N, N)), "sigma": g["sigma"], "gamma": g["gamma"]}
            gf["cov"][:, il[0], il[1]] = g["cov"]
            gf["cov"][:, il[1], il[0]] = g["cov"]
            assert _cov_rel_err(gf, r, np.ones(P, bool)) <= 1e-6
    w = synth.custom_workload(N, 2 * N, 96, seed=900 + N, n_extra=4, k_max=N - 8, sigma=(1e-4, 2e-4))
    S = synth.make_library(w)
    X, s = synth.make_cube(w)
    g3 = _gpu(S, X, s, dev, cov="full", maxit=3)
    r3 = oracle.unmix(S, X, s, maxit=3)
    assert (g3["status"] == oracle.MAXIT).all() and (r3["status"] == oracle.MAXIT).all()
    assert np.abs(g3["a"] - r3["a"]).max() <= 1e-9
    assert _cov_rel_err(g3, r3, np.ones(len(X), bool)) <= 1e-6


def _straddling(N, L, P, seed, noise=0.005):
    """Mixtures whose coefficient sums spread around one (the sum constraint
    of sum-lower-than-one binds for some pixels only)."""
    rng = np.random.default_rng(seed)
    w = synth.custom_workload(N, L, P, seed=seed, n_extra=min(4, N - 1), k_max=max(1, min(4, N - 4)))
    S = synth.make_library(w)
    A = rng.dirichlet(np.ones(N), P) * rng.uniform(0.6, 1.4, (P, 1))
    X = (A @ S.astype(np.float64) + noise * rng.standard_normal((P, L))).astype(np.float32)
    s = rng.uniform(0.5, 2.0, P).astype(np.float32)
    return S, X, s


@pytest.mark.parametrize("constraint", ["slo", "pos"])
@pytest.mark.parametrize("N", [8, 36, 48, 64, 80])
def test_constraint_options(dev, constraint, N):
    """Sum-lower-than-one and positivity only against the oracle, on the tile
    kernel (N = 8, 36, 48, 64) and the lane-group kernel (N = 80), FP64 and
    mixed (whose FP32 stage is the lane-group kernel at every N)."""
    _say(f"[gpu] constraint {constraint} N={N}")
    # three channels per spectrum above N = 64: with two, 7 % of the oracle's
    # own pixels end uncertified on this mixture of all spectra
    S, X, s = _straddling(N, max(2 * N, 96) if N <= 64 else 3 * N, 403, seed=100 + N)
    code = {"slo": oracle.SLO, "pos": oracle.POS}[constraint]
    r = oracle.unmix(S, X, s, constraint=code)
    if constraint == "slo":
        below = r["a"].sum(1) < 1.0 - 1e-9
        assert 20 <= below.sum() <= 383, below.sum()
    for precision in ("fp64", "mixed"):
        g = _gpu(S, X, s, dev, precision=precision, constraint=constraint)
        _compare(g, r, S, X, constraint=constraint, a_tol=1e-6 if precision == "fp64" else 1e-3,
                 f_tol=1e-9 if precision == "fp64" else 1e-4)
        if constraint == "slo":
            assert (g["a"].sum(1) <= 1.0 + 1e-9).all()


def test_constraint_uncertified_covariance(dev):
    """Three iterations: the covariance of the last iterate carries the slack
    corner -s/nu (sum-lower-than-one) or no sum row (positivity only), on both
    covariance paths (free sets of 12 and of 40 coefficients)."""
    _say("[gpu] uncertified covariance with the slack corner")
    for N in (12, 40):
        S, X, s = _straddling(N, 96, 150, seed=300 + N)
        for constraint, code in (("slo", oracle.SLO), ("pos", oracle.POS)):
            g = _gpu(S, X, s, dev, cov="full", constraint=constraint, maxit=3)
            r = oracle.unmix(S, X, s, constraint=code, maxit=3)
            assert (g["status"] == oracle.MAXIT).all() and (r["status"] == oracle.MAXIT).all()
            assert np.abs(g["a"] - r["a"]).max() <= 1e-9
            assert _cov_rel_err(g, r, np.ones(len(X), bool)) <= 1e-6


@pytest.mark.parametrize("n_extra", [4, 12])
@pytest.mark.parametrize("constraint", ["sto", "slo", "pos"])
def test_paper_extra_library(dev, constraint, n_extra):
    """Libraries carrying the paper's additional spectra (Sec. 2.5): 32
    minerals plus 4 (N = 36, tile kernel) or 12 (N = 44, VALU kernel).  The
    extras are linearly dependent, so the minimiser may be non-unique; the
    least objective is unique.  Compared: the objective, within the bound on
    an interior iterate's excess (complementarity gap and dual residual)
    where either side is uncertified; coefficients and covariance where
    both sides certified a strictly complementary solution (then the
    minimiser is unique); feasibility everywhere."""
    from paper_1402_2518_amd import linmin
    _say(f"[gpu] paper extra library n_extra={n_extra} {constraint}")
    w = synth.WORKLOADS["orbital"]
    M = synth.make_library(w)[:32]
    S_g = np.concatenate([M, linmin.extra_spectra(w.L, n_extra)])
    S_o = np.concatenate([M, oracle.extra_spectra(w.L, n_extra).astype(np.float32)])
    assert np.abs(S_g.view(np.int32).astype(np.int64) - S_o.view(np.int32).astype(np.int64)).max() <= 1
    X, s = synth.make_cube(w, p0=5000, p1=5600)
    code = {"sto": oracle.STO, "slo": oracle.SLO, "pos": oracle.POS}[constraint]
    r = oracle.unmix(S_o, X, s, constraint=code)
    pairs = len(S_o) + (1 if constraint == "slo" else 0)
    for precision in ("fp64", "mixed"):
        g = _gpu(S_g, X, s, dev, precision=precision, constraint=constraint)
        assert np.isfinite(g["a"]).all() and (g["a"] >= 0).all()
        tot = g["a"].sum(1)
        if constraint == "sto":
            assert np.abs(tot - 1).max() <= 1e-12
        elif constraint == "slo":
            assert tot.max() <= 1 + 1e-12
        exact = (g["status"] == 0) & (r["status"] == 0)
        loose = ((g["status"] | r["status"]) & oracle.INEXACT) != 0
        gap = np.array([pins.objective_gap_bound(S_o, X[p], s[p], g["a"][p].sum() + r["a"][p].sum(), pairs)
                        for p in range(len(X))])
        rnd = 1e-9 if precision == "fp64" else 1e-4
        dF = np.abs(g["objective"] - r["F"])
        lim = np.where(loose, gap, 0.0) + rnd * r["F"]
        assert (dF <= lim).all(), float((dF / lim).max())
        if exact.any():
            da = np.abs(g["a"][exact] - r["a"][exact]).max()
            assert da <= (1e-6 if precision == "fp64" else 1e-3), da
            assert _cov_rel_err(g, r, exact) <= (1e-6 if precision == "fp64" else 1e-3)
        _say(f"  {precision}: certified both {exact.sum()}/{len(X)}, inexact either {loose.sum()}")


def _batch_item(N, L, P, seed):
    n_extra = min(4, N - 1) if N > 1 else 0
    w = synth.custom_workload(N, L, max(P, 1), seed=seed, n_extra=n_extra,
                              k_max=max(1, min(4, N - n_extra)))
    S = synth.make_library(w)
    X, s = synth.make_cube(w, p1=P)
    return S, X, s


BATCH_SPECS = [(2, 64, 300), (5, 64, 1), (16, 128, 2049), (24, 128, 0), (36, 240, 1000), (40, 128, 17),
               (48, 240, 700), (64, 128, 513), (96, 128, 300), (36, 240, 64), (8, 64, 1500)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_single_calls(dev, precision):
    """A batch of cubes with their own libraries (N from 2 to 96, L from 64 to
    240, P from 0 to 2,049, one library with a full noise covariance) gives
    every cube exactly the bytes a single call gives it, on two runs in a row
    of the same plan; the first pixels of every cube also match the oracle."""
    from paper_1402_2518_amd import linmin
    _say(f"[gpu] batch of {len(BATCH_SPECS) + 1} cubes, {precision}")
    data = [_batch_item(N, L, P, seed=700 + i) + (None,) for i, (N, L, P) in enumerate(BATCH_SPECS)]
    rng = np.random.default_rng(29)
    Sn = synth.mineral_spectra(12, 100, rng).astype(np.float32)
    Q = rng.standard_normal((100, 100))
    Cn = (Q @ Q.T / 100 + np.diag(rng.uniform(0.5, 2.0, 100))) * 1e-4
    Xn = (rng.dirichlet(np.ones(12), 250) @ Sn.astype(float) + 0.01 * rng.standard_normal((250, 100))).astype(np.float32)
    data.append((Sn, Xn, rng.uniform(0.5, 2.0, 250).astype(np.float32), Cn))
    libs, items = [], []
    for S, X, s, C in data:
        lib = linmin.Library(S, C)
        Xt = torch.from_numpy(np.ascontiguousarray(X, np.float32).reshape(-1, S.shape[1])).to(dev)
        st = torch.from_numpy(np.ascontiguousarray(s[:len(X)], np.float32)).to(dev)
        libs.append(lib)
        items.append((lib, Xt, st))
    b = linmin.Batch(items, precision=precision, cov="full")
    assert b.device_bytes() > 0
    singles = [lib.unmix(Xt, st, precision=precision, cov="full") for lib, Xt, st in items]
    for run in range(2):
        # scribble over the outputs so that the second run has to rewrite them
        for r in b.results:
            for t in r.values():
                if t is not None:
                    t.fill_(7)
        b.run()
        torch.cuda.synchronize()
        for i, (r, one) in enumerate(zip(b.results, singles)):
            for k in ("a", "cov", "status", "iters", "objective"):
                assert torch.equal(r[k].nan_to_num(3.5), one[k].nan_to_num(3.5)), (run, i, k)
    for i, ((S, X, s, C), r) in enumerate(zip(data, b.results)):
        k = min(len(X), 64)
        if k == 0:
            continue
        ro = oracle.unmix(S, X[:k], s[:k], C=C)
        ga = r["a"][:k].cpu().numpy()
        tol = 1e-6 if precision == "fp64" else 1e-3
        assert np.abs(ga - ro["a"]).max() <= tol, (i, np.abs(ga - ro["a"]).max())
    b.close()
    for lib in libs:
        lib.close()


@pytest.mark.parametrize("constraint", ["sto", "pos"])
def test_dependent_spectra_first(dev, constraint):
    """The paper's 12 additional spectra placed before 24 minerals (N = 36,
    the 4x4-tile kernel at T = 9): nearly singular diagonal blocks come first
    and every later block depends on their elimination.  Such a library is
    factored without explicit block inverses; the objective must stay within
    the gap bound of an uncertified iterate, and no pixel may lose positive
    definiteness where the oracle kept it."""
    from paper_1402_2518_amd import linmin
    _say(f"[gpu] dependent spectra first, {constraint}")
    w = synth.WORKLOADS["orbital"]
    M = synth.make_library(w)[:24]
    S_g = np.concatenate([linmin.extra_spectra(w.L, 12), M])
    S_o = np.concatenate([oracle.extra_spectra(w.L, 12).astype(np.float32), M])
    X, s = synth.make_cube(w, p0=9000, p1=9400)
    code = {"sto": oracle.STO, "pos": oracle.POS}[constraint]
    r = oracle.unmix(S_o, X, s, constraint=code, cov=False)
    g = _gpu(S_g, X, s, dev, cov=None, constraint=constraint)
    notpd = ((g["status"] & oracle.NOT_PD) != 0) & ((r["status"] & oracle.NOT_PD) == 0)
    assert not notpd.any(), int(notpd.sum())
    loose = ((g["status"] | r["status"]) & (oracle.INEXACT | oracle.MAXIT)) != 0
    gap = np.array([pins.objective_gap_bound(S_o, X[p], s[p], g["a"][p].sum() + r["a"][p].sum(), len(S_o))
                    for p in range(len(X))])
    dF = np.abs(g["objective"] - r["F"])
    assert (dF <= np.where(loose, gap, 0.0) + 1e-9 * r["F"]).all()
    exact = (g["status"] == 0) & (r["status"] == 0)
    if exact.any():
        assert np.abs(g["a"][exact] - r["a"][exact]).max() <= 1e-6


def test_serving_mix_identical_alone(dev):
    """Requests of four resident libraries (N = 8..96) arriving within 50 ms
    run concurrently under an HBM budget that admits only some at a time;
    every third cube arrives in pinned host memory and is copied in by the
    server; each result equals the same request served alone, bit for bit,
    and sampled pixels match the oracle."""
    from paper_1402_2518_amd import linmin, serve
    _say("[gpu] serving loop: 24 overlapping requests")
    rng = np.random.default_rng(77)
    shapes = [(8, 64), (36, 240), (48, 128), (96, 128)]
    libs, pools, hostS = {}, {}, {}
    for i, (N, L) in enumerate(shapes):
        w = synth.custom_workload(N, L, 4000, seed=900 + i)
        S = synth.make_library(w)
        X, s = synth.make_cube(w)
        libs[i] = linmin.Library(S)
        pools[i] = (torch.from_numpy(X).to(dev), torch.from_numpy(s).to(dev), X, s,
                    torch.from_numpy(X).pin_memory(), torch.from_numpy(s).pin_memory())
        hostS[i] = S
    reqs = []
    for rid in range(24):
        k = int(rng.integers(0, len(shapes)))
        P = int(round(np.exp(rng.uniform(np.log(50), np.log(3000)))))
        off = int(rng.integers(0, 4000 - P + 1))
        Xd, sd, _, _, Xh, sh = pools[k]
        if rid % 3 == 2:
            Xd, sd = Xh, sh
        reqs.append(serve.Request(rid, k, Xd[off:off + P], sd[off:off + P], arrival=float(rng.uniform(0, 0.05))))
        reqs[-1].off = off
    fps = sorted(serve.footprint(libs[r.lib], r.cube.shape[0], "fp64", "full", r.cube.device.type == "cpu")
                 for r in reqs)
    budget = 3 * fps[len(fps) // 2]
    srv = serve.Server(libs, streams=4, slots=6, hbm_budget=budget, cov="full")
    done = srv.run(reqs)
    torch.cuda.synchronize()
    assert sorted(r.rid for r in done) == list(range(24))
    assert srv.stats["max_running"] >= 2
    assert srv.stats["max_bytes"] <= max(budget, fps[-1])
    for r in done:
        alone = libs[r.lib].unmix(r.cube.to(dev), r.sigma.to(dev), precision="fp64", cov="full")
        torch.cuda.synchronize()
        for key in ("a", "cov", "status", "iters", "objective"):
            assert torch.equal(r.out[key].nan_to_num(3.5), alone[key].nan_to_num(3.5)), (r.rid, key)
    assert sum(r.cube.device.type == "cpu" for r in done) == 8
    for r in done[:6]:
        _, _, X, s, _, _ = pools[r.lib]
        k = min(8, r.cube.shape[0])
        ro = oracle.unmix(hostS[r.lib], X[r.off:r.off + k], s[r.off:r.off + k], cov=False)
        assert np.abs(r.out["a"][:k].cpu().numpy() - ro["a"]).max() <= 1e-6
    summary = serve.latency_summary(done)
    _say(f"  {summary}")
    for lib in libs.values():
        lib.close()


def test_detection_kernels_on_synthetic_arrays(dev):
    """Thresholds (eq. 8) and detection rules on the same seeded arrays on
    both sides: thresholds to reduction-order rounding, decisions exactly."""
    from paper_1402_2518_amd import linmin
    _say("[gpu] detection kernels on seeded arrays")
    rng = np.random.default_rng(61)
    P, N = 20_011, 37
    present = rng.random((P, N)) < 0.25
    present[:, 5] = True                      # never absent: NaN threshold
    A = np.where(present, rng.uniform(0.02, 0.6, (P, N)), np.abs(0.003 * rng.standard_normal((P, N))))
    thr_o = oracle.thresholds(A, present)
    At = torch.from_numpy(A).to(dev)
    thr_g = linmin.thresholds(At, torch.from_numpy(present.astype(np.uint8)).to(dev)).cpu().numpy()
    assert np.isnan(thr_g[5]) and np.isnan(thr_o[5])
    ok = ~np.isnan(thr_o)
    assert np.abs(thr_g[ok] - thr_o[ok]).max() <= 1e-13 * np.abs(thr_o[ok]).max()
    s1 = np.abs(0.05 * rng.standard_normal((P, N)))
    rms = rng.uniform(0.0, 0.02, P)
    thr = rng.uniform(0.01, 0.1, N)
    d_o = oracle.detect(A, s1, rms, thr, rms_max=0.012)
    d_g = linmin.detect(At, torch.from_numpy(s1).to(dev), torch.from_numpy(rms).to(dev),
                        torch.from_numpy(thr).to(dev), 0.012).cpu().numpy()
    assert np.array_equal(d_g.astype(bool), d_o) and 0.05 < d_o.mean() < 0.5


def test_detection_pipeline_against_the_oracle(dev):
    """Unmix, RMS and 1-sigma maps, thresholds from the true presence, and
    detection, each side from its own coefficients: maps to the unmixing
    tolerances, thresholds to 1e-9, decisions equal except at near-ties."""
    from paper_1402_2518_amd import linmin
    _say("[gpu] detection pipeline")
    w = synth.custom_workload(12, 96, 3000, seed=12)
    S = synth.make_library(w)
    X, s, Atrue = synth.make_cube(w, with_truth=True)
    present = Atrue > 0
    r = oracle.unmix(S, X, s)
    rms_o, s1_o = oracle.rms_map(S, X, r["a"]), oracle.sigma1_map(r["cov"])
    thr_o = oracle.thresholds(r["a"], present)
    lib = linmin.Library(S)
    Xd, sd = torch.from_numpy(X).to(dev), torch.from_numpy(s).to(dev)
    g = lib.unmix(Xd, sd, cov="full")
    rms_g, s1_g = lib.error_maps(Xd, g["a"], g["cov"], cov="full")
    pres_t = torch.from_numpy(present.astype(np.uint8)).to(dev)
    thr_g = linmin.thresholds(g["a"], pres_t)
    rms_max = float(np.percentile(rms_o, 90))
    det_g = linmin.detect(g["a"], s1_g, rms_g, thr_g, rms_max).cpu().numpy().astype(bool)
    det_o = oracle.detect(r["a"], s1_o, rms_o, thr_o, rms_max)
    ok = (g["status"].cpu().numpy() == 0) & (r["status"] == 0)
    rms_h, s1_h = rms_g.cpu().numpy(), s1_g.cpu().numpy()
    assert np.abs(rms_h / rms_o - 1).max() <= 1e-8
    scale = np.maximum(s1_o[ok].max(1, keepdims=True), s[ok, None] / np.sqrt(lib.gamma))
    assert (np.abs(s1_h[ok] - s1_o[ok]) / scale).max() <= 1e-6
    thr_h = thr_g.cpu().numpy()
    fin = ~np.isnan(thr_o)   # the extras are present everywhere: no threshold
    assert np.array_equal(np.isnan(thr_h), ~fin) and fin.sum() == 8
    assert np.abs(thr_h[fin] - thr_o[fin]).max() <= 1e-9
    a_o, thr = r["a"], thr_o[None, :]
    near = (np.abs(a_o - thr) <= 1e-6) | (np.abs(s1_o - a_o) <= 1e-6 * np.maximum(a_o, 1e-12)) | \
           (np.abs(rms_o - rms_max)[:, None] <= 1e-8 * rms_max)
    assert ((det_g == det_o) | near).all() and det_o.sum() > 0
    lib.close()
    # with a noise covariance the RMS stays the plain reflectance residual
    rng = np.random.default_rng(23)
    Sn = synth.mineral_spectra(10, 80, rng).astype(np.float32)
    Q = rng.standard_normal((80, 80))
    C = (Q @ Q.T / 80 + np.diag(rng.uniform(0.5, 2.0, 80))) * 1e-4
    Xn = (rng.dirichlet(np.ones(10), 400) @ Sn.astype(float) + 0.01 * rng.standard_normal((400, 80))).astype(np.float32)
    rn = oracle.unmix(Sn, Xn, None, C=C, cov=False)
    libn = linmin.Library(Sn, C)
    Xnd = torch.from_numpy(Xn).to(dev)
    gn = libn.unmix(Xnd, None, cov=None)
    rms_n, _ = libn.error_maps(Xnd, gn["a"])
    assert np.abs(rms_n.cpu().numpy() / oracle.rms_map(Sn, Xn, rn["a"]) - 1).max() <= 1e-8
    libn.close()


@pytest.mark.parametrize("constraint", ["sto", "pos"])
def test_second_pass_against_the_oracle(dev, constraint):
    """Second pass: each pixel unmixed again with a subset of the spectra
    (about half, some pixels one or two, one pixel none) against the
    oracle's unmix of each pixel's sub-library."""
    from paper_1402_2518_amd import linmin
    _say(f"[gpu] second pass {constraint}")
    w = synth.custom_workload(16, 96, 300, seed=16)
    S = synth.make_library(w)
    X, s = synth.make_cube(w)
    rng = np.random.default_rng(5)
    keep = rng.random((300, 16)) < 0.5
    keep[:20] = False
    keep[:10, 3] = True                            # one spectrum
    keep[10:20, 1] = keep[10:20, 7] = True         # two spectra
    keep[20] = False                               # none: reported non-finite
    code = {"sto": oracle.STO, "pos": oracle.POS}[constraint]
    r = oracle.second_pass(S, X, s, keep, constraint=code)
    lib = linmin.Library(S)
    g = lib.unmix(torch.from_numpy(X).to(dev), torch.from_numpy(s).to(dev), cov="full", constraint=constraint,
                  keep=torch.from_numpy(keep.astype(np.uint8)).to(dev))
    ga, gst = g["a"].cpu().numpy(), g["status"].cpu().numpy()
    assert gst[20] & oracle.NONFINITE and np.isnan(ga[20]).all()
    rows = np.arange(300) != 20
    assert np.abs(ga[rows] - r["a"][rows]).max() <= 1e-6
    assert (ga[rows][~keep[rows]] == 0).all()
    ok = rows & (gst == 0) & (r["status"] == 0)
    assert ok.mean() > 0.9
    assert _cov_rel_err({"cov": g["cov"].cpu().numpy(), "sigma": s.astype(float), "gamma": lib.gamma},
                        {"cov": r["cov"]}, ok) <= 1e-6
    lib.close()


def test_batch_run_in_a_graph(dev):
    """A planned batch enqueues kernels only, so one run can be captured in a
    HIP graph; every replay (with eager work and synchronisation between
    them) reproduces the eager run bit for bit."""
    from paper_1402_2518_amd import linmin
    _say("[gpu] batch run captured in a graph")
    data = [_batch_item(N, L, P, seed=800 + i) for i, (N, L, P) in
            enumerate([(8, 64, 700), (36, 240, 1500), (48, 128, 333), (96, 128, 200)])]
    libs, items = [], []
    for S, X, s in data:
        lib = linmin.Library(S)
        libs.append(lib)
        items.append((lib, torch.from_numpy(X).to(dev), torch.from_numpy(s).to(dev)))
    b = linmin.Batch(items, precision="mixed", cov="packed")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        b.run(side)
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in r.items() if v is not None} for r in b.results]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        b.run(side)
    for rep in range(3):
        for r in b.results:
            for t in r.values():
                if t is not None:
                    t.fill_(9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = items[0][1].sum().item()  # eager work between replays
        for i, (r, want) in enumerate(zip(b.results, ref)):
            for k, v in want.items():
                assert torch.equal(r[k].nan_to_num(3.5), v.nan_to_num(3.5)), (rep, i, k)
    del g
    b.close()
    for lib in libs:
        lib.close()


_VALU_CHECK = r"""
import os, sys
sys.path.insert(0, os.getcwd())
sys.path.insert(0, os.path.join(os.getcwd(), "tests"))
import numpy as np, torch
import oracle
from paper_1402_2518_amd import linmin, synth
worst = 0.0
for N, L in ((8, 64), (36, 240), (48, 128), (64, 128)):
    w = synth.custom_workload(N, L, 600, seed=950 + N)
    S = synth.make_library(w)
    X, s = synth.make_cube(w)
    lib = linmin.Library(S)
    g = lib.unmix(torch.from_numpy(X).to("cuda:0"), torch.from_numpy(s).to("cuda:0"), cov="full")
    torch.cuda.synchronize()
    r = oracle.unmix(S, X, s)
    ok = (g["status"].cpu().numpy() == 0) & (r["status"] == 0)
    assert ok.mean() > 0.95, (N, ok.mean())
    worst = max(worst, float(np.abs(g["a"].cpu().numpy() - r["a"]).max()))
    cg, cr = g["cov"].cpu().numpy()[ok], r["cov"][ok]
    scale = np.maximum(np.abs(cr).reshape(len(cr), -1).max(1), s[ok].astype(float) ** 2 / lib.gamma)[:, None, None]
    assert (np.abs(cg - cr) / scale).max() <= 1e-6, N
    lib.close()
print("worst", worst)
assert worst <= 1e-6
"""


def test_lane_group_fp64_kernel_at_tile_sizes(dev):
    """The lane-group FP64 kernel is complete for every N (the tile kernel
    takes N <= 64 by default); run it in a child process with the tile
    kernel switched off and check it against the oracle."""
    import subprocess
    _say("[gpu] lane-group FP64 kernel at N = 8..64 (child process)")
    env = dict(os.environ, LINMIN_FP64_KERNEL="valu")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _VALU_CHECK], cwd=root, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.parametrize("constraint", ["sto", "slo"])
def test_batch_mixes_factorisations_and_constraints(dev, constraint):
    """One batch holding a well-conditioned library (explicit-inverse tile
    factorisation), the paper's additional spectra placed first (stable
    factorisation, same N), and a lane-group size, under a non-default
    constraint option: each cube equals its single call bit for bit."""
    from paper_1402_2518_amd import linmin
    _say(f"[gpu] batch with both factorisations, {constraint}")
    w = synth.WORKLOADS["orbital"]
    S1 = synth.make_library(w)
    S2 = np.concatenate([linmin.extra_spectra(w.L, 12), synth.make_library(w)[:24]])
    X, s = synth.make_cube(w, p1=900)
    S3, X3, s3 = _batch_item(80, 240, 300, seed=990)
    items, libs = [], []
    for S, XX, ss in ((S1, X, s), (S2, X, s), (S3, X3, s3)):
        lib = linmin.Library(S)
        libs.append(lib)
        items.append((lib, torch.from_numpy(XX).to(dev), torch.from_numpy(ss).to(dev)))
    b = linmin.Batch(items, precision="fp64", cov="full", constraint=constraint)
    b.run()
    torch.cuda.synchronize()
    for i, ((lib, Xd, sd), r) in enumerate(zip(items, b.results)):
        one = lib.unmix(Xd, sd, cov="full", constraint=constraint)
        torch.cuda.synchronize()
        for k in ("a", "cov", "status", "iters", "objective"):
            assert torch.equal(r[k].nan_to_num(3.5), one[k].nan_to_num(3.5)), (i, k)
    b.close()
    for lib in libs:
        lib.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["orbital", "precision"])
def test_full_size_launch_sampled(dev, name, precision):
    """The whole cube in one call, as the benchmark times it (orbital:
    524,288 pixels at N = 36; precision: 307,200 at N = 64, L = 438), in
    both precisions with full covariance; 512 pixels spread over the cube
    (both ends and the last, ragged chunk included) against the oracle."""
    from paper_1402_2518_amd import linmin
    w = synth.WORKLOADS[name]
    _say(f"[gpu] full-size launch {name} P={w.P} {precision}")
    S = synth.make_library(w)
    X, s = synth.make_cube(w)
    lib = linmin.Library(S)
    g = lib.unmix(torch.from_numpy(X).to(dev), torch.from_numpy(s).to(dev), precision=precision, cov="full")
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([np.arange(8), np.arange(w.P - 8, w.P), rng.choice(w.P, 496, replace=False)]))
    it = torch.from_numpy(idx).to(dev)
    gs = {"a": g["a"][it].cpu().numpy(), "cov": g["cov"][it].cpu().numpy(), "status": g["status"][it].cpu().numpy(),
          "iters": g["iters"][it].cpu().numpy(), "objective": g["objective"][it].cpu().numpy(),
          "gamma": lib.gamma, "sigma": s[idx].astype(float)}
    r = oracle.unmix(S, X[idx], s[idx])
    _compare(gs, r, S, X[idx], a_tol=1e-6 if precision == "fp64" else 1e-3,
             f_tol=1e-9 if precision == "fp64" else 1e-4)
    assert int((g["status"] != 0).sum()) <= 0.01 * w.P
    lib.close()
