"""Seeded synthetic reference libraries and hyperspectral cubes.

This module only draws inputs.  It holds none of the unmixing arithmetic: a
cube is produced with the linear mixing model of the paper (Sec. 2.1, eq. 1),
``X = A.S + E``, used here as a forward model with Gaussian zero-mean noise.
Both the HIP path and the CPU oracle take their inputs from here, and nothing
else is shared between them.

Layout (matches the C-ABI):

* library ``S``: ``N x L`` float32, one reference spectrum per row (the paper's
  ``S``, Sec. 2.1).
* cube ``X``: ``P x L`` float32, pixel-major (one spectrum per row, the paper's
  ``X``).
* ``sigma``: ``P`` float32 per-pixel noise scale ``s_p``.

Workloads (sizes and distributions):

* ``tiny``       N=8 minerals,  L=64,  P=1,000, 1-3 active minerals,
                 Dirichlet(1) abundances, sigma = 0.005 on every channel.
* ``orbital``    N=36 = 32 minerals + 4 extra spectra, L=240,
                 P = 128 x 4,096 = 524,288, 1-4 active minerals plus all four
                 extras with Dirichlet(1) weights, s_p ~ U[0.002, 0.01].
* ``precision``  N=64 = 60 minerals + 4 extras, L=438, P = 640 x 480 = 307,200,
                 distributions as ``orbital``.

Mineral spectra: a random quadratic continuum (coefficients U[-1,1]) min-max
mapped onto [lo, hi] with lo ~ U[0.1, 0.45], hi ~ U[lo+0.05, 0.6], multiplied
by 1-4 Gaussian absorption bands ``1 - d exp(-(j-c)^2 / (2 w^2))`` with depth
d ~ U[0.05, 0.4], width w ~ U[2, 8] channels and centre c ~ U[0, L-1].  The four
extra spectra (flat, slope and two broad smooth curves) stand in for the
paper's additional continuum spectra (Sec. 2.5); the paper's exact sets of 4
and 12 are a library builder of the product, not an input recipe.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

CHUNK = 8192  # pixels per independently seeded chunk; fixes the byte stream


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_minerals: int
    n_extra: int
    L: int
    P: int
    k_max: int            # active minerals per pixel: U{1..k_max}
    extras_active: bool   # every pixel also mixes all extra spectra
    sigma_lo: float
    sigma_hi: float
    lib_seed: int
    cube_seed: int

    @property
    def N(self) -> int:
        return self.n_minerals + self.n_extra


WORKLOADS = {
    "tiny": Workload("tiny", 8, 0, 64, 1000, 3, False, 0.005, 0.005, 1001, 2001),
    "orbital": Workload("orbital", 32, 4, 240, 128 * 4096, 4, True, 0.002, 0.01, 1002, 2002),
    "precision": Workload("precision", 60, 4, 438, 640 * 480, 4, True, 0.002, 0.01, 1003, 2003),
}


def mineral_spectra(n: int, L: int, rng: np.random.Generator) -> np.ndarray:
    """``n x L`` float64 synthetic mineral reflectance spectra in (0, 0.6]."""
    j = np.arange(L, dtype=np.float64)
    x = j / max(L - 1, 1)
    out = np.empty((n, L))
    for i in range(n):
        q = rng.uniform(-1.0, 1.0, 3)
        cont = q[0] + q[1] * x + q[2] * x * x
        lo = rng.uniform(0.1, 0.45)
        hi = rng.uniform(lo + 0.05, 0.6)
        span = cont.max() - cont.min()
        cont = lo + (hi - lo) * ((cont - cont.min()) / span if span > 0 else 0.5)
        r = cont.copy()
        for _ in range(int(rng.integers(1, 5))):
            c = rng.uniform(0.0, L - 1.0)
            w = rng.uniform(2.0, 8.0)
            d = rng.uniform(0.05, 0.4)
            r *= 1.0 - d * np.exp(-((j - c) ** 2) / (2.0 * w * w))
        out[i] = r
    return out


def extra_spectra(L: int) -> np.ndarray:
    """``4 x L``: flat 1, linear slope, and two broad smooth bumps."""
    x = np.arange(L, dtype=np.float64) / max(L - 1, 1)
    return np.stack([
        np.ones(L),
        x,
        np.exp(-((x - 0.3) ** 2) / (2 * 0.35 ** 2)),
        np.exp(-((x - 0.8) ** 2) / (2 * 0.4 ** 2)),
    ])


def make_library(w: Workload | str) -> np.ndarray:
    """Reference library ``S`` (``N x L`` float32) for a workload."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    rng = np.random.default_rng(w.lib_seed)
    rows = [mineral_spectra(w.n_minerals, w.L, rng)]
    if w.n_extra:
        rows.append(extra_spectra(w.L)[: w.n_extra])
    return np.ascontiguousarray(np.concatenate(rows).astype(np.float32))


def _chunk(w: Workload, S32: np.ndarray, c: int, noise: bool):
    p0 = c * CHUNK
    n = min(CHUNK, w.P - p0)
    rng = np.random.default_rng([w.cube_seed, c])
    nm, N = w.n_minerals, w.N
    k = rng.integers(1, w.k_max + 1, size=n)
    ranks = np.argsort(np.argsort(rng.random((n, nm)), axis=1), axis=1)
    mask = np.zeros((n, N), dtype=bool)
    mask[:, :nm] = ranks < k[:, None]
    if w.extras_active:
        mask[:, nm:] = True
    e = rng.exponential(size=(n, N))
    e[~mask] = 0.0
    A = e / e.sum(axis=1, keepdims=True)
    s = rng.uniform(w.sigma_lo, w.sigma_hi, size=n) if w.sigma_hi > w.sigma_lo \
        else np.full(n, w.sigma_lo)
    eps = rng.standard_normal((n, w.L))
    X = A @ S32.astype(np.float64)
    if noise:
        X += s[:, None] * eps
    return X.astype(np.float32), s.astype(np.float32), A


def make_cube(w: Workload | str, S: np.ndarray | None = None, p0: int = 0,
              p1: int | None = None, noise: bool = True, with_truth: bool = False):
    """Pixels ``[p0, p1)`` of a workload's cube.

    Returns ``(X, sigma)`` (float32, ``(p1-p0) x L`` and ``p1-p0``) and, with
    ``with_truth``, the true abundances ``A`` (float64).  Any pixel range gives
    the same bytes as the corresponding slice of the full cube.  With
    ``noise=False`` the spectra are exact mixtures (sigma is still drawn).
    """
    if isinstance(w, str):
        w = WORKLOADS[w]
    if S is None:
        S = make_library(w)
    p1 = w.P if p1 is None else p1
    if not 0 <= p0 <= p1 <= w.P:
        raise ValueError("bad pixel range")
    n = p1 - p0
    X = np.empty((n, w.L), np.float32)
    sig = np.empty(n, np.float32)
    A = np.empty((n, w.N)) if with_truth else None
    for c in range(p0 // CHUNK, (p1 + CHUNK - 1) // CHUNK if n else p0 // CHUNK):
        cx, cs, ca = _chunk(w, S, c, noise)
        lo, hi = max(p0, c * CHUNK), min(p1, c * CHUNK + len(cs))
        X[lo - p0:hi - p0] = cx[lo - c * CHUNK:hi - c * CHUNK]
        sig[lo - p0:hi - p0] = cs[lo - c * CHUNK:hi - c * CHUNK]
        if with_truth:
            A[lo - p0:hi - p0] = ca[lo - c * CHUNK:hi - c * CHUNK]
    return (X, sig, A) if with_truth else (X, sig)


def make_cube_device(w: Workload, S: np.ndarray, device, chunk: int = 65536):
    """The whole cube of ``w`` generated on a torch device, for workloads
    too large to draw on the host in reasonable time.  Same distributions as
    :func:`make_cube` (1..k_max active minerals chosen uniformly, every extra
    spectrum active when ``extras_active``, Dirichlet(1) weights as normalised
    exponentials, s_p ~ U[sigma_lo, sigma_hi], Gaussian noise), drawn from a
    torch generator seeded with ``cube_seed``: a different byte stream.
    Returns ``(X, sigma)`` as float32 device tensors.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(w.cube_seed)
    nm, N, P = w.n_minerals, w.N, w.P
    St = torch.from_numpy(np.ascontiguousarray(S, np.float32)).to(device=device, dtype=torch.float64)
    X = torch.empty((P, w.L), dtype=torch.float32, device=device)
    sig = torch.empty(P, dtype=torch.float32, device=device)
    for p0 in range(0, P, chunk):
        n = min(chunk, P - p0)
        k = torch.randint(1, max(w.k_max, 1) + 1, (n, 1), generator=g, device=device)
        mask = torch.zeros((n, N), dtype=torch.bool, device=device)
        if nm:
            ranks = torch.rand((n, nm), generator=g, device=device).argsort(1).argsort(1)
            mask[:, :nm] = ranks < k
        if w.extras_active:
            mask[:, nm:] = True
        e = torch.empty((n, N), dtype=torch.float64, device=device).exponential_(generator=g)
        e = torch.where(mask, e, torch.zeros_like(e))
        A = e / e.sum(1, keepdim=True)
        sg = torch.rand(n, dtype=torch.float64, generator=g, device=device) * (w.sigma_hi - w.sigma_lo) + w.sigma_lo
        eps = torch.randn((n, w.L), dtype=torch.float64, generator=g, device=device)
        X[p0:p0 + n] = (A @ St + sg[:, None] * eps).to(torch.float32)
        sig[p0:p0 + n] = sg.to(torch.float32)
    return X, sig


BATCH_N = (16, 24, 36, 48, 64, 96)
BATCH_L = (128, 240, 438)


def batch_workloads(n_cubes: int = 200, seed: int = 4242, p_lo: float = 1e3, p_hi: float = 2e5):
    """The many-cube batch: each cube draws its own library size N from
    BATCH_N and channel count L from BATCH_L, and a pixel count log-uniform in
    [p_lo, p_hi]; minerals, extras, abundances and noise as ``precision``
    (4 extras, 1-4 active minerals, s_p ~ U[0.002, 0.01])."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_cubes):
        N = int(rng.choice(BATCH_N))
        L = int(rng.choice(BATCH_L))
        P = int(round(math.exp(rng.uniform(math.log(p_lo), math.log(p_hi)))))
        out.append(custom_workload(N, L, P, seed=30_000 + i))
    return out


def custom_workload(N: int, L: int, P: int, seed: int, n_extra: int = 4,
                    k_max: int = 4, sigma=(0.002, 0.01)) -> Workload:
    """A workload of arbitrary shape with the ``orbital`` distributions."""
    if n_extra > N:
        raise ValueError("n_extra > N")
    return Workload(f"custom{N}x{L}x{P}s{seed}", N - n_extra, n_extra, L, P,
                    min(k_max, N - n_extra) if N > n_extra else 0,
                    n_extra > 0, sigma[0], sigma[1], 10_000 + seed, 20_000 + seed)
