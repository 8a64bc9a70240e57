"""Request loop for unmixing cubes as they arrive (continuous batching).

Libraries stay resident on the device with their Gram matrices (one
:class:`linmin.Library` each).  A request names a library and a device cube.
Requests wait in arrival order.  A waiting request is admitted as soon as an
execution slot is free and its HBM footprint (outputs and the call's
workspace) fits in the budget next to the requests already running; a request
that does not fit does not block smaller ones behind it, unless it has waited
longer than a bound, after which nothing passes it until it has started (so
no request starves).  An admitted request is one ``linmin_unmix`` call on one
of a few HIP streams, ordered after the work that was queued on the caller's
stream when it was admitted (where its cube was produced), so requests of
different libraries and sizes run on the device at the same time and new ones
start while earlier ones are still running.  Every pixel is
solved independently, so a request's result does not depend on what else was
running.

A request's cube may also arrive in (pinned) host memory: it is then copied
to the device on a copy stream of its own, and the unmix call waits for that
copy only, so transfers of arriving cubes overlap the solves of earlier ones.

Host-side scheduling only: the arithmetic is in the library's kernels.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np

from . import linmin

_COV_PER = {None: lambda n: 0, "none": lambda n: 0, "full": lambda n: n * n,
            "packed": lambda n: n * (n + 1) // 2, "diag": lambda n: n}


@dataclasses.dataclass
class Request:
    rid: int
    lib: str             # key of a resident library
    cube: object         # P x L float32 tensor, on the device or in pinned host memory
    sigma: object        # P float32 tensor (same place as cube) or None
    arrival: float       # seconds from the start of the run
    keep: bool = True    # keep the outputs after completion
    # filled by the server
    t_start: float = float("nan")
    t_done: float = float("nan")
    footprint: int = 0
    out: dict | None = None
    cube_dev: object = None  # device copy of a host cube while the request runs


def footprint(lib: linmin.Library, P: int, precision: str, cov: str | None, host_input: bool = False) -> int:
    """Device bytes a request holds while it runs: its outputs, the
    workspace of the call and, for a cube in host memory, its device copy."""
    n = lib.N
    outs = P * (8 * n + 8 * _COV_PER[cov](n) + 1 + 4 + 8)
    inputs = P * (4 * lib.L + 4) if host_input else 0
    return outs + inputs + lib.workspace_bytes(P, precision, cov)


def admissible(head_bytes: int, used_bytes: int, budget: int, running: int, slots: int) -> bool:
    """Admission rule: a free slot and room in the HBM budget (a request
    larger than the whole budget is admitted alone, so it cannot wait
    forever)."""
    if running >= slots:
        return False
    if running == 0:
        return True
    return used_bytes + head_bytes <= budget


def pick(waiting, used_bytes: int, budget: int, running: int, slots: int, now: float, max_pass_s: float):
    """Index in ``waiting`` (arrival order) of the next request to admit, or
    None.  The oldest request that fits goes first; a request that does not
    fit is passed over by later ones only while it has waited less than
    ``max_pass_s`` seconds."""
    for i, r in enumerate(waiting):
        if admissible(r.footprint, used_bytes, budget, running, slots):
            return i
        if running >= slots or now - r.arrival >= max_pass_s:
            return None
    return None


class Server:
    def __init__(self, libraries: dict, streams: int = 4, slots: int = 8, hbm_budget: int = 64 << 30,
                 precision: str = "fp64", cov: str | None = "full", max_pass_s: float = 0.25):
        import torch
        self.libs = libraries
        self.max_pass_s = float(max_pass_s)
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.copy_stream = torch.cuda.Stream()  # host-to-device copies of arriving cubes
        self.slots = slots
        self.budget = int(hbm_budget)
        self.precision = precision
        self.cov = cov
        self.stats = {"max_running": 0, "max_bytes": 0}

    def _launch(self, r: Request, k: int):
        import torch
        lib = self.libs[r.lib]
        P, n = r.cube.shape[0], lib.N
        st = self.streams[k % len(self.streams)]
        dev = torch.device("cuda", torch.cuda.current_device()) if r.cube.device.type == "cpu" else r.cube.device
        if r.cube.device.type == "cpu":
            # copy the arriving cube on the copy stream; the solve waits for it
            cs = self.copy_stream
            with torch.cuda.stream(cs):
                cube = r.cube.to(dev, non_blocking=True)
                sigma = None if r.sigma is None else r.sigma.to(dev, non_blocking=True)
            st.wait_stream(cs)
            cube.record_stream(st)
            if sigma is not None:
                sigma.record_stream(st)
            r.cube_dev = (cube, sigma)  # held until the request completes
        else:
            # the cube (and sigma) may still be in production on the caller's
            # stream: order this request after it, and tell the caching
            # allocator that the side stream uses them
            cube, sigma = r.cube, r.sigma
            st.wait_stream(torch.cuda.current_stream(dev))
            cube.record_stream(st)
            if sigma is not None:
                sigma.record_stream(st)
        with torch.cuda.stream(st):
            shp = {None: None, "none": None, "full": (P, n, n), "packed": (P, n * (n + 1) // 2),
                   "diag": (P, n)}[self.cov]
            out = {"a": torch.empty((P, n), dtype=torch.float64, device=dev),
                   "cov": None if shp is None else torch.empty(shp, dtype=torch.float64, device=dev),
                   "status": torch.empty(P, dtype=torch.uint8, device=dev),
                   "iters": torch.empty(P, dtype=torch.int32, device=dev),
                   "objective": torch.empty(P, dtype=torch.float64, device=dev)}
            lib.unmix_into(cube, sigma, out["a"], out["cov"], out["status"], out["iters"], out["objective"],
                           precision=self.precision, cov=self.cov, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return out, ev

    def run(self, requests: list[Request], poll_s: float = 2e-4) -> list[Request]:
        """Serve ``requests`` (their arrival times relative to now); return
        them completed, in completion order."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: deque[Request] = deque()
        running: list[tuple[Request, object]] = []
        done: list[Request] = []
        used = 0
        k = 0
        for r in pending:
            r.footprint = footprint(self.libs[r.lib], r.cube.shape[0], self.precision, self.cov,
                                    host_input=r.cube.device.type == "cpu")
        t0 = time.perf_counter()
        while pending or waiting or running:
            now = time.perf_counter() - t0
            busy = False
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            for item in list(running):
                r, ev = item
                if ev.query():
                    r.t_done = time.perf_counter() - t0
                    used -= r.footprint
                    running.remove(item)
                    r.cube_dev = None
                    if not r.keep:
                        r.out = None
                    done.append(r)
                    busy = True
            while waiting:
                i = pick(waiting, used, self.budget, len(running), self.slots, now, self.max_pass_s)
                if i is None:
                    break
                r = waiting[i]
                del waiting[i]
                r.t_start = time.perf_counter() - t0
                r.out, ev = self._launch(r, k)
                k += 1
                used += r.footprint
                running.append((r, ev))
                self.stats["max_running"] = max(self.stats["max_running"], len(running))
                self.stats["max_bytes"] = max(self.stats["max_bytes"], used)
                busy = True
            if not busy:
                time.sleep(poll_s)
        return done


def poisson_arrivals(rate: float, seconds: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate on [0, seconds)."""
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            return np.array(out)
        out.append(t)


def latency_summary(done: list[Request]) -> dict:
    lat = np.array([r.t_done - r.arrival for r in done]) * 1e3
    wait = np.array([r.t_start - r.arrival for r in done]) * 1e3
    pix = sum(int(r.cube.shape[0]) for r in done)
    span = max(r.t_done for r in done) - min(r.arrival for r in done)
    return {"requests": len(done), "pixels": pix, "pixels_per_s": pix / span,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "queue_wait_ms": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
            "span_s": span}
