"""CPU oracle for LinMin unmixing (plain FP64 C, OpenMP over pixels).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its binding) never does.  The C source is
``linmin_oracle.c``; ``build()`` compiles it with gcc into
``liblinmin_oracle.so`` next to it.

The oracle solves, per pixel, the renormalised least-squares problem of the
paper (Sec. 2.3, eq. 6) under positivity and sum-to-one (Sec. 2.2, eqs. 3-4)
with a primal-dual interior-point method plus an exact finishing step, and
returns the coefficient covariance from the Hessian (end of Sec. 2.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "linmin_oracle.c")
LIB = os.path.join(HERE, "liblinmin_oracle.so")

MAXIT, NONFINITE, BAD_SIGMA, NOT_PD, DEGENERATE, INEXACT = 1, 2, 4, 8, 16, 32


class Opts(ctypes.Structure):
    _fields_ = [("maxit", ctypes.c_int), ("max_polish", ctypes.c_int),
                ("tol_mu", ctypes.c_double), ("tol_d", ctypes.c_double),
                ("tol_p", ctypes.c_double), ("eta", ctypes.c_double),
                ("lambda0", ctypes.c_double), ("tau", ctypes.c_double),
                ("deg_tol", ctypes.c_double), ("constraint", ctypes.c_int)]


# constraint options of IPLS besides a >= 0
STO, SLO, POS = 0, 1, 2  # sum-to-one, sum-lower-than-one, positivity only


def build(force: bool = True, src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle source with gcc (-O2, OpenMP) into ``out``."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


_libs: dict = {}


def _load(path: str | None = None):
    """Load the oracle library (``path`` selects another build of the same source)."""
    key = path or LIB
    if key not in _libs:
        if path is None and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        lib = ctypes.CDLL(key)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        lib.lo_default_opts.argtypes = [ctypes.POINTER(Opts)]
        lib.lo_renormalise.argtypes = [fp, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        lib.lo_renormalise.restype = ctypes.c_int
        lib.lo_unmix.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, fp, fp, ctypes.c_long,
                                 ctypes.POINTER(Opts), dp, dp, dp,
                                 ctypes.POINTER(ctypes.c_ubyte), ctypes.POINTER(ctypes.c_int),
                                 dp, dp, ctypes.c_int]
        lib.lo_unmix.restype = ctypes.c_int
        lib.lo_max_threads.restype = ctypes.c_int
        _libs[key] = lib
    return _libs[key]


def default_opts(lib: str | None = None, **kw) -> Opts:
    o = Opts()
    _load(lib).lo_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ct))


def max_threads() -> int:
    return int(_load().lo_max_threads())


def renormalise(S: np.ndarray, C: np.ndarray | None = None, lib: str | None = None):
    """Return ``(Sp, Lc)``: ``S' = S Lc`` with ``C^{-1} = Lc Lc^T`` (eq. 5)."""
    S = np.ascontiguousarray(S, dtype=np.float32)
    N, L = S.shape
    Sp = np.empty((N, L))
    Lc = None
    Cc = None
    if C is not None:
        Cc = np.ascontiguousarray(C, dtype=np.float64)
        if Cc.shape != (L, L):
            raise ValueError("C must be L x L")
        Lc = np.empty((L, L))
    rc = _load(lib).lo_renormalise(_ptr(S, ctypes.c_float), L, N, _ptr(Cc, ctypes.c_double),
                                _ptr(Sp, ctypes.c_double), _ptr(Lc, ctypes.c_double))
    if rc == -4:
        raise ValueError("noise covariance is not symmetric positive definite")
    if rc != 0:
        raise RuntimeError(f"lo_renormalise failed: {rc}")
    return Sp, Lc


def unmix(S: np.ndarray, X: np.ndarray, sigma: np.ndarray | None = None,
          C: np.ndarray | None = None, cov: bool = True, threads: int = 0,
          lib: str | None = None, **opts):
    """Unmix every row of ``X`` against library ``S`` (rows = spectra).

    Returns a dict with ``a`` (P x N), ``cov`` (P x N x N or None), ``F``,
    ``status``, ``iters``, ``lam`` (scaled multipliers) and ``nu``.
    """
    Sp, Lc = renormalise(S, C, lib=lib)
    N, L = Sp.shape
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2 or X.shape[1] != L:
        raise ValueError("X must be P x L")
    P = X.shape[0]
    sg = None if sigma is None else np.ascontiguousarray(sigma, dtype=np.float32)
    A = np.empty((P, N))
    CV = np.empty((P, N, N)) if cov else None
    F = np.empty(P)
    st = np.empty(P, np.uint8)
    it = np.empty(P, np.int32)
    lam = np.empty((P, N))
    nu = np.empty(P)
    o = default_opts(lib, **opts)
    rc = _load(lib).lo_unmix(_ptr(Sp, ctypes.c_double), _ptr(Lc, ctypes.c_double), L, N,
                          _ptr(X, ctypes.c_float), _ptr(sg, ctypes.c_float), P, ctypes.byref(o),
                          _ptr(A, ctypes.c_double), _ptr(CV, ctypes.c_double),
                          _ptr(F, ctypes.c_double), _ptr(st, ctypes.c_ubyte),
                          _ptr(it, ctypes.c_int), _ptr(lam, ctypes.c_double),
                          _ptr(nu, ctypes.c_double), int(threads))
    if rc != 0:
        raise RuntimeError(f"lo_unmix failed: {rc}")
    return {"a": A, "cov": CV, "F": F, "status": st, "iters": it, "lam": lam, "nu": nu}


def extra_spectra(L: int, n: int = 4, wavelengths: np.ndarray | None = None) -> np.ndarray:
    """The additional spectra of Sec. 2.5, in the order of the table of
    additional spectra after the references, as an ``n x L`` FP64 array.

    Spectral position ``t`` runs linearly from 0 at the first wavelength to
    1 at the last (channel index when ``wavelengths`` is None).  The four are
    a level at one, a level at 1e-4, and slopes ``t`` and ``1 - t``.  The
    twelve add cosine and sine of periods four and two times the spectral
    domain (the "1/4" and "1/2" entries: that fraction of a cycle across the
    domain), each with both signs since the coefficients are non-negative.
    """
    if n not in (4, 12):
        raise ValueError("n must be 4 or 12")
    if wavelengths is None:
        w = np.arange(L, dtype=np.float64)
    else:
        w = np.asarray(wavelengths, dtype=np.float64)
    t = (w - w[0]) / (w[-1] - w[0])
    rows = [np.ones(L), np.full(L, 1e-4), t, 1.0 - t]
    if n == 12:
        for cycles in (0.25, 0.5):
            c, s = np.cos(2 * np.pi * cycles * t), np.sin(2 * np.pi * cycles * t)
            rows += [c, s, -c, -s]
    return np.stack(rows)


# ---------------------------------------------------------------------------
# Detection post-processing (Sec. 3.1 eq. 8 and the rules of Sec. 4)
# ---------------------------------------------------------------------------
def rms_map(S: np.ndarray, X: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Root-mean-square of each pixel's fit residual y - a S over its L
    channels, in reflectance units (not whitened by a noise covariance)."""
    Sd, Xd = np.asarray(S, np.float64), np.asarray(X, np.float64)
    R = Xd - np.asarray(A, np.float64) @ Sd
    return np.sqrt((R * R).sum(1) / Sd.shape[1])


def sigma1_map(cov: np.ndarray) -> np.ndarray:
    """1-sigma error of every coefficient: square roots of the covariance
    diagonal (P x N from P x N x N)."""
    return np.sqrt(np.maximum(np.diagonal(np.asarray(cov, np.float64), axis1=1, axis2=2), 0.0))


def thresholds(A: np.ndarray, present: np.ndarray) -> np.ndarray:
    """Detection threshold of eq. 8 for every endmember i: half the sum of
    (mean - 2 std) of its coefficients on the pixels where it is present and
    (mean + 6 std) where it is absent; population standard deviations.  NaN
    for an endmember without present or without absent pixels."""
    A = np.asarray(A, np.float64)
    present = np.asarray(present, bool)
    out = np.full(A.shape[1], np.nan)
    for i in range(A.shape[1]):
        pos, neg = A[present[:, i], i], A[~present[:, i], i]
        if len(pos) and len(neg):
            out[i] = 0.5 * (pos.mean() - 2.0 * pos.std() + neg.mean() + 6.0 * neg.std())
    return out


def detect(A: np.ndarray, sigma1: np.ndarray, rms: np.ndarray, thr: np.ndarray, rms_max: float) -> np.ndarray:
    """Detection rules of Sec. 4: endmember i is detected in pixel p when its
    coefficient exceeds the threshold, its 1-sigma error is below the
    coefficient, and the pixel's RMS is below the noise level rms_max."""
    A = np.asarray(A, np.float64)
    return (A > np.asarray(thr)[None, :]) & (np.asarray(sigma1) < A) & (np.asarray(rms)[:, None] < rms_max)


def second_pass(S: np.ndarray, X: np.ndarray, sigma, keep: np.ndarray, C=None, constraint: int = STO):
    """Second pass of the conclusion: each pixel unmixed again with only the
    spectra kept for it (keep: P x N bool), by the oracle on that sub-library;
    coefficients and covariance scattered back to N (zeros elsewhere).
    Pixels that keep no spectrum get NaN."""
    X = np.asarray(X)
    P, N = X.shape[0], S.shape[0]
    a = np.zeros((P, N))
    cov = np.zeros((P, N, N))
    status = np.zeros(P, np.uint8)
    F = np.zeros(P)
    for p in range(P):
        idx = np.flatnonzero(keep[p])
        if len(idx) == 0:
            a[p], cov[p], F[p] = np.nan, np.nan, np.nan
            continue
        s = None if sigma is None else np.asarray(sigma)[p:p + 1]
        r = unmix(np.ascontiguousarray(S[idx]), X[p:p + 1], s, C=C, constraint=constraint)
        a[p, idx] = r["a"][0]
        cov[p][np.ix_(idx, idx)] = r["cov"][0]
        status[p] = r["status"][0]
        F[p] = r["F"][0]
    return {"a": a, "cov": cov, "status": status, "F": F}
