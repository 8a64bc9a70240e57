"""Thin Python binding of lib_linmin (``include/linmin.h``) over ctypes.

Argument marshalling only: torch provides device memory and streams, every
step of the unmixing runs in the library's HIP kernels.  The shared library
``liblinmin.so`` must have been built (``paper_1402_2518_amd.build``); there
is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblinmin.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSPD, EUNSUPPORTED, ESCRATCH = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
COV_NONE, COV_FULL, COV_PACKED, COV_DIAG = 0, 1, 2, 3
STO, SLO, POS = 0, 1, 2  # sum-to-one, sum-lower-than-one, positivity only
PX_MAXIT, PX_NONFINITE, PX_BAD_SIGMA, PX_NOT_PD, PX_DEGENERATE, PX_INEXACT = 1, 2, 4, 8, 16, 32
N_MAX = 128
# interior-point kernel families and stages (linmin_set_kernel)
KERNEL_DEFAULT, KERNEL_ROWCYCLIC, KERNEL_TILE, KERNEL_GROUP, KERNEL_TILE32 = 0, 1, 2, 3, 4
STAGE_FP64, STAGE_FP32 = 0, 1
KERNELS = {"default": KERNEL_DEFAULT, "rowcyclic": KERNEL_ROWCYCLIC, "tile": KERNEL_TILE, "group": KERNEL_GROUP,
           "tile32": KERNEL_TILE32}

NOALLOC_SCRATCH_BYTES = 64 << 20  # LINMIN_NOALLOC_SCRATCH_BYTES

EXPORTS = ("linmin_default_opts", "linmin_create_library", "linmin_unmix", "linmin_unmix_noalloc",
           "linmin_workspace_bytes",
           "linmin_library_info", "linmin_library_gram", "linmin_destroy_library", "linmin_strerror",
           "linmin_extra_spectra", "linmin_batch_create", "linmin_batch_run", "linmin_batch_device_bytes",
           "linmin_batch_destroy", "linmin_error_maps", "linmin_thresholds", "linmin_detect",
           "linmin_set_kernel", "linmin_get_kernel")


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("cov_layout", ctypes.c_int), ("maxit", ctypes.c_int),
                ("max_polish", ctypes.c_int), ("constraint", ctypes.c_int), ("tol_mu", ctypes.c_double),
                ("tol_d", ctypes.c_double),
                ("tol_p", ctypes.c_double), ("eta", ctypes.c_double), ("lambda0", ctypes.c_double),
                ("tau", ctypes.c_double), ("deg_tol", ctypes.c_double), ("mu_switch", ctypes.c_double),
                ("status", ctypes.c_void_p), ("iters", ctypes.c_void_p), ("objective", ctypes.c_void_p),
                ("stage_events", ctypes.c_void_p), ("keep", ctypes.c_void_p)]


class Job(ctypes.Structure):
    _fields_ = [("lib", ctypes.c_void_p), ("cube", ctypes.c_void_p), ("P", ctypes.c_int64),
                ("sigma", ctypes.c_void_p), ("out_coeffs", ctypes.c_void_p), ("out_cov", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("iters", ctypes.c_void_p), ("objective", ctypes.c_void_p)]


class LinminError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


_lib = None


TUNING_PATH = os.path.join(HERE, "tuning.json")


def load(path: str = LIB_PATH, tuning: bool = True) -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built).  On the first
    load, the measured kernel choices of ``tuning.json`` (written by
    :mod:`paper_1402_2518_amd.autotune`) are installed, unless ``tuning`` is
    false or the environment sets ``LINMIN_TUNING=0``."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise FileNotFoundError(f"{path} is missing: build it with paper_1402_2518_amd.build.build()")
        lib = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        lib.linmin_default_opts.argtypes = [ctypes.POINTER(Opts)]
        lib.linmin_default_opts.restype = None
        lib.linmin_create_library.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]
        lib.linmin_create_library.restype = ctypes.c_int
        lib.linmin_unmix.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp, ctypes.POINTER(Opts), vp]
        lib.linmin_unmix.restype = ctypes.c_int
        lib.linmin_unmix_noalloc.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp, ctypes.POINTER(Opts), vp]
        lib.linmin_unmix_noalloc.restype = ctypes.c_int
        lib.linmin_workspace_bytes.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(Opts)]
        lib.linmin_workspace_bytes.restype = ctypes.c_size_t
        lib.linmin_library_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_double)]
        lib.linmin_library_info.restype = ctypes.c_int
        lib.linmin_library_gram.argtypes = [vp, vp]
        lib.linmin_library_gram.restype = ctypes.c_int
        lib.linmin_destroy_library.argtypes = [vp]
        lib.linmin_destroy_library.restype = ctypes.c_int
        lib.linmin_extra_spectra.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp]
        lib.linmin_extra_spectra.restype = ctypes.c_int
        lib.linmin_batch_create.argtypes = [ctypes.POINTER(Job), ctypes.c_int, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        lib.linmin_batch_create.restype = ctypes.c_int
        lib.linmin_batch_run.argtypes = [vp, vp]
        lib.linmin_batch_run.restype = ctypes.c_int
        lib.linmin_batch_device_bytes.argtypes = [vp]
        lib.linmin_batch_device_bytes.restype = ctypes.c_size_t
        lib.linmin_batch_destroy.argtypes = [vp]
        lib.linmin_batch_destroy.restype = ctypes.c_int
        i64, dbl = ctypes.c_int64, ctypes.c_double
        lib.linmin_error_maps.argtypes = [vp, i64, vp, vp, vp, ctypes.c_int, vp, vp, vp]
        lib.linmin_error_maps.restype = ctypes.c_int
        lib.linmin_thresholds.argtypes = [ctypes.c_int, i64, vp, vp, vp, vp]
        lib.linmin_thresholds.restype = ctypes.c_int
        lib.linmin_detect.argtypes = [ctypes.c_int, i64, vp, vp, vp, vp, dbl, vp, vp]
        lib.linmin_detect.restype = ctypes.c_int
        lib.linmin_set_kernel.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.linmin_set_kernel.restype = ctypes.c_int
        lib.linmin_get_kernel.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        lib.linmin_get_kernel.restype = ctypes.c_int
        lib.linmin_strerror.argtypes = [ctypes.c_int]
        lib.linmin_strerror.restype = ctypes.c_char_p
        _lib = lib
        if tuning and os.environ.get("LINMIN_TUNING", "1") != "0" and os.path.exists(TUNING_PATH):
            from . import autotune
            autotune.install(TUNING_PATH)
    return _lib


def strerror(code: int) -> str:
    return load().linmin_strerror(int(code)).decode()


def set_kernel(N: int, stage: int, family, lanes: int = 0) -> None:
    """Interior-point kernel family (and, for ``"group"``, lanes per pixel;
    0 = default width) for libraries of the padded size of N in this process
    (``linmin_set_kernel``); ``family`` is a name of ``KERNELS`` or its code."""
    fam = KERNELS[family] if isinstance(family, str) else int(family)
    rc = load().linmin_set_kernel(int(N), int(stage), fam, int(lanes))
    if rc != OK:
        raise LinminError(rc, "linmin_set_kernel")


def get_kernel(N: int, stage: int) -> int:
    """Family a library of N uses for ``stage`` now (``linmin_get_kernel``)."""
    return get_kernel_lanes(N, stage)[0]


def get_kernel_lanes(N: int, stage: int) -> tuple:
    """``(family, lanes)`` a library of N uses for ``stage`` now; lanes is
    the group width for group kernels, else 0."""
    ln = ctypes.c_int(0)
    rc = load().linmin_get_kernel(int(N), int(stage), ctypes.byref(ln))
    if rc < 0:
        raise LinminError(rc, "linmin_get_kernel")
    return rc, ln.value


def default_opts(**kw) -> Opts:
    o = Opts()
    load().linmin_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def extra_spectra(L: int, n: int = 4, wavelengths=None) -> np.ndarray:
    """The additional spectra of Sec. 2.5 (``n`` = 4 or 12) as an ``n x L``
    float32 array, from ``linmin_extra_spectra``."""
    out = np.empty((n, L), np.float32)
    wl = None if wavelengths is None else np.ascontiguousarray(wavelengths, dtype=np.float64)
    if wl is not None and wl.shape != (L,):
        raise ValueError("wavelengths must hold L values")
    rc = load().linmin_extra_spectra(int(L), int(n), None if wl is None else wl.ctypes.data_as(ctypes.c_void_p),
                                     out.ctypes.data_as(ctypes.c_void_p))
    if rc != OK:
        raise LinminError(rc, "linmin_extra_spectra")
    return out


_PREC = {"fp64": FP64, "mixed": MIXED}
_COV = {None: COV_NONE, "none": COV_NONE, "full": COV_FULL, "packed": COV_PACKED, "diag": COV_DIAG}
_CONS = {"sto": STO, "slo": SLO, "pos": POS}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Library:
    """A reference library (rows of ``S`` are spectra) and optional noise
    covariance ``C`` (L x L), prepared on the current HIP device."""

    def __init__(self, S: np.ndarray, C: np.ndarray | None = None):
        S = np.ascontiguousarray(S, dtype=np.float32)
        if S.ndim != 2:
            raise ValueError("S must be N x L")
        self.N, self.L = S.shape
        Cc = None if C is None else np.ascontiguousarray(C, dtype=np.float64)
        h = ctypes.c_void_p()
        rc = load().linmin_create_library(S.ctypes.data_as(ctypes.c_void_p), self.L, self.N,
                                          None if Cc is None else Cc.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.byref(h))
        if rc != OK:
            raise LinminError(rc, "linmin_create_library")
        self._h = h
        g = ctypes.c_double()
        load().linmin_library_info(self._h, None, None, ctypes.byref(g))
        self.gamma = g.value

    def gram(self) -> np.ndarray:
        G = np.empty((self.N, self.N))
        rc = load().linmin_library_gram(self._h, G.ctypes.data_as(ctypes.c_void_p))
        if rc != OK:
            raise LinminError(rc, "linmin_library_gram")
        return G

    def close(self):
        if getattr(self, "_h", None):
            load().linmin_destroy_library(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, P: int, precision: str = "fp64", cov: str | None = "full") -> int:
        o = default_opts(precision=_PREC[precision], cov_layout=_COV[cov])
        return int(load().linmin_workspace_bytes(self._h, int(P), ctypes.byref(o)))

    def unmix_into(self, cube, sigma, out_a, out_cov=None, status=None, iters=None, objective=None,
                   precision: str = "fp64", cov: str | None = "full", stream=None, events=None, keep=None,
                   noalloc: bool = False, **opts):
        """Enqueue one unmix on ``stream`` into caller-provided device tensors.

        ``noalloc``: call ``linmin_unmix_noalloc`` (work areas in the
        library's fixed device array, nothing allocated; calls on one GPU
        must not overlap in time).

        ``events``: optional four ``torch.cuda.Event(enable_timing=True)``
        recorded before the projections, the solve, the covariance and after.
        ``keep``: optional P x N uint8 device tensor, the spectra each pixel
        keeps (second pass); the others are held at zero.
        """
        import torch
        if cube.dtype != torch.float32 or not cube.is_contiguous() or cube.dim() != 2:
            raise ValueError("cube must be a contiguous P x L float32 tensor")
        P = cube.shape[0]
        if cube.shape[1] != self.L:
            raise ValueError("cube has the wrong number of channels")
        if sigma is not None and (sigma.dtype != torch.float32 or sigma.numel() != P or not sigma.is_contiguous()):
            raise ValueError("sigma must be a contiguous float32 tensor of P values")
        N = self.N
        per = {None: 0, "none": 0, "full": N * N, "packed": N * (N + 1) // 2, "diag": N}[cov]

        def _check(t, name, dtype, numel):
            if t is None:
                return
            if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel or t.device != cube.device:
                raise ValueError(f"{name} must be a contiguous {dtype} tensor of {numel} values on {cube.device}")

        if out_a is None:
            raise ValueError("out_a is required")
        _check(out_a, "out_a", torch.float64, P * N)
        if per == 0 and out_cov is not None:
            raise ValueError(f"out_cov given but cov={cov!r}")
        if per > 0 and out_cov is None:
            raise ValueError(f"cov={cov!r} needs out_cov")
        _check(out_cov, "out_cov", torch.float64, P * per)
        _check(status, "status", torch.uint8, P)
        _check(iters, "iters", torch.int32, P)
        _check(objective, "objective", torch.float64, P)
        if isinstance(opts.get("constraint"), str):
            opts["constraint"] = _CONS[opts["constraint"]]
        o = default_opts(precision=_PREC[precision], cov_layout=_COV[cov], **opts)
        o.status = None if status is None else status.data_ptr()
        o.iters = None if iters is None else iters.data_ptr()
        o.objective = None if objective is None else objective.data_ptr()
        _check(keep, "keep", torch.uint8, P * N)
        o.keep = None if keep is None else keep.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream()
        ev_arr = None
        if events is not None:
            if len(events) != 4:
                raise ValueError("events must hold 4 timing events")
            for e in events:
                e.record(stream)  # makes sure the underlying HIP event exists
            ev_arr = (ctypes.c_void_p * 4)(*[ctypes.c_void_p(e.cuda_event) for e in events])
            o.stage_events = ctypes.cast(ev_arr, ctypes.c_void_p)
        fn = load().linmin_unmix_noalloc if noalloc else load().linmin_unmix
        rc = fn(self._h, _ptr(cube), int(P), _ptr(sigma), _ptr(out_a), _ptr(out_cov),
                ctypes.byref(o), ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise LinminError(rc, "linmin_unmix_noalloc" if noalloc else "linmin_unmix")

    def error_maps(self, cube, coeffs, cov_out=None, cov: str = "full", stream=None):
        """RMS map (P) of the fit residual y - a S in reflectance units, and
        the 1-sigma error map (P x N) from a covariance output (None: not
        computed)."""
        import torch
        P = coeffs.shape[0]
        rms = torch.empty(P, dtype=torch.float64, device=coeffs.device)
        s1 = None if cov_out is None else torch.empty((P, self.N), dtype=torch.float64, device=coeffs.device)
        if stream is None:
            stream = torch.cuda.current_stream()
        rc = load().linmin_error_maps(self._h, int(P), _ptr(cube), _ptr(coeffs), _ptr(cov_out),
                                      _COV[cov] if cov_out is not None else 0, _ptr(rms), _ptr(s1),
                                      ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise LinminError(rc, "linmin_error_maps")
        return rms, s1

    def unmix(self, cube, sigma=None, precision: str = "fp64", cov: str | None = "full",
              stream=None, **opts):
        """Unmix a device cube (P x L float32 torch tensor).

        Returns a dict of device tensors: ``a`` (P x N float64), ``cov`` (per
        ``cov`` layout, or None), ``status`` (uint8), ``iters`` (int32),
        ``objective`` (float64).
        """
        import torch
        dev = cube.device
        P = cube.shape[0]
        a = torch.empty((P, self.N), dtype=torch.float64, device=dev)
        shape = {None: None, "none": None, "full": (P, self.N, self.N),
                 "packed": (P, self.N * (self.N + 1) // 2), "diag": (P, self.N)}[cov]
        cv = None if shape is None else torch.empty(shape, dtype=torch.float64, device=dev)
        st = torch.empty(P, dtype=torch.uint8, device=dev)
        it = torch.empty(P, dtype=torch.int32, device=dev)
        obj = torch.empty(P, dtype=torch.float64, device=dev)
        self.unmix_into(cube, sigma, a, cv, st, it, obj, precision=precision, cov=cov, stream=stream, **opts)
        return {"a": a, "cov": cv, "status": st, "iters": it, "objective": obj}


def _cov_shape(cov, P, N):
    return {None: None, "none": None, "full": (P, N, N), "packed": (P, N * (N + 1) // 2), "diag": (P, N)}[cov]


class Batch:
    """Many cubes, each with its own :class:`Library`, planned once
    (``linmin_batch_create``) and unmixed by :meth:`run` in a few fused
    launches.  ``items``: a sequence of ``(library, cube, sigma)`` with cube a
    contiguous P x L float32 device tensor and sigma a P float32 device tensor
    or None.  Output tensors are allocated here and reused by every run:
    ``results[i]`` holds ``a``, ``cov``, ``status``, ``iters``, ``objective``
    of item i.
    """

    def __init__(self, items, precision: str = "fp64", cov: str | None = "full", events=None, **opts):
        import torch
        if isinstance(opts.get("constraint"), str):
            opts["constraint"] = _CONS[opts["constraint"]]
        self._opts = default_opts(precision=_PREC[precision], cov_layout=_COV[cov], **opts)
        self._ev = None
        if events is not None:
            # four timing events recorded by every run: before the projections,
            # the solve, the covariance, and after
            if len(events) != 4:
                raise ValueError("events must hold 4 timing events")
            for e in events:
                e.record()  # makes sure the underlying HIP event exists
            self._ev = (ctypes.c_void_p * 4)(*[ctypes.c_void_p(e.cuda_event) for e in events])
            self._opts.stage_events = ctypes.cast(self._ev, ctypes.c_void_p)
        self.items = list(items)
        self.results = []
        jobs = (Job * max(1, len(self.items)))()
        for i, (lib, cube, sigma) in enumerate(self.items):
            if cube.dtype != torch.float32 or not cube.is_contiguous() or cube.dim() != 2 or cube.shape[1] != lib.L:
                raise ValueError(f"item {i}: cube must be a contiguous P x {lib.L} float32 tensor")
            P, N, dev = cube.shape[0], lib.N, cube.device
            if sigma is not None and (sigma.dtype != torch.float32 or sigma.numel() != P or not sigma.is_contiguous()):
                raise ValueError(f"item {i}: sigma must be a contiguous float32 tensor of P values")
            shp = _cov_shape(cov, P, N)
            r = {"a": torch.empty((P, N), dtype=torch.float64, device=dev),
                 "cov": None if shp is None else torch.empty(shp, dtype=torch.float64, device=dev),
                 "status": torch.empty(P, dtype=torch.uint8, device=dev),
                 "iters": torch.empty(P, dtype=torch.int32, device=dev),
                 "objective": torch.empty(P, dtype=torch.float64, device=dev)}
            self.results.append(r)
            jobs[i] = Job(lib._h.value, cube.data_ptr(), P, None if sigma is None else sigma.data_ptr(),
                          r["a"].data_ptr(), None if r["cov"] is None else r["cov"].data_ptr(),
                          r["status"].data_ptr(), r["iters"].data_ptr(), r["objective"].data_ptr())
        h = ctypes.c_void_p()
        rc = load().linmin_batch_create(jobs, len(self.items), ctypes.byref(self._opts), ctypes.byref(h))
        if rc != OK:
            raise LinminError(rc, "linmin_batch_create")
        self._h = h

    def device_bytes(self) -> int:
        return int(load().linmin_batch_device_bytes(self._h))

    def run(self, stream=None):
        """Enqueue every item on ``stream`` (default: torch's current stream)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        rc = load().linmin_batch_run(self._h, ctypes.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise LinminError(rc, "linmin_batch_run")

    def close(self):
        if getattr(self, "_h", None):
            load().linmin_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def thresholds(coeffs, present, stream=None):
    """Thresholds of eq. 8 (N, float64 device tensor) from P x N coefficients
    and a P x N uint8 mask of where each endmember is present."""
    import torch
    P, N = coeffs.shape
    if present.dtype != torch.uint8 or present.shape != coeffs.shape or not present.is_contiguous():
        raise ValueError("present must be a contiguous P x N uint8 tensor")
    if coeffs.dtype != torch.float64 or not coeffs.is_contiguous():
        raise ValueError("coeffs must be a contiguous float64 tensor")
    out = torch.empty(N, dtype=torch.float64, device=coeffs.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = load().linmin_thresholds(int(N), int(P), _ptr(coeffs), _ptr(present), _ptr(out),
                                  ctypes.c_void_p(stream.cuda_stream))
    if rc != OK:
        raise LinminError(rc, "linmin_thresholds")
    return out


def detect(coeffs, sigma1, rms, thr, rms_max: float, stream=None):
    """Detection rules of Sec. 4 as a P x N uint8 device tensor."""
    import torch
    P, N = coeffs.shape
    for name, t, n in (("coeffs", coeffs, P * N), ("sigma1", sigma1, P * N), ("rms", rms, P), ("thr", thr, N)):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be a contiguous float64 tensor of {n} values")
    out = torch.empty((P, N), dtype=torch.uint8, device=coeffs.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = load().linmin_detect(int(N), int(P), _ptr(coeffs), _ptr(sigma1), _ptr(rms), _ptr(thr), float(rms_max),
                              _ptr(out), ctypes.c_void_p(stream.cuda_stream))
    if rc != OK:
        raise LinminError(rc, "linmin_detect")
    return out

