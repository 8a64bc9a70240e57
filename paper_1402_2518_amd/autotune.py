"""Measured choice of the interior-point kernel per library size (the tuning
table of lib_linmin).

Every kernel family of the library (row-cyclic and four-pixel FP64 tiles,
FP32 tiles, lane groups of each compiled width) solves the same problem; which
is fastest depends on the library size N and on the device.  This module times
every candidate compiled for a size on a synthetic cube with the orbital
cube's distributions, checks that it reproduces the coefficients of the
default kernel, and writes the fastest per (size, stage) to ``tuning.json``
next to this file, which :func:`linmin.load` installs with
``linmin_set_kernel``.

Run on the target GPU::

    python -m paper_1402_2518_amd.autotune [--sizes 8,16,...] [--pixels P]

The FP64 stage is tuned first (plain FP64 unmix calls); the FP32 stage of the
mixed form is then tuned with the chosen FP64 kernel in place.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import linmin, synth

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning.json")
SIZES = (8, 16, 24, 32, 36, 48, 64, 96, 128)
FAMILY_NAMES = {v: k for k, v in linmin.KERNELS.items()}


def candidates(N: int, stage: int) -> list[tuple[int, int]]:
    """(family, lanes) pairs compiled for the padded size of N and stage."""
    out = []
    lib = linmin.load()
    for fam in (linmin.KERNEL_ROWCYCLIC, linmin.KERNEL_TILE, linmin.KERNEL_TILE32):
        if lib.linmin_set_kernel(N, stage, fam, 0) == linmin.OK:
            out.append((fam, 0))
    for g in (1, 2, 4, 8, 16, 32):
        if lib.linmin_set_kernel(N, stage, linmin.KERNEL_GROUP, g) == linmin.OK:
            out.append((linmin.KERNEL_GROUP, g))
    lib.linmin_set_kernel(N, stage, linmin.KERNEL_DEFAULT, 0)
    return out


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune_size(N: int, L: int, P: int, reps: int, dev, log=print) -> list[dict]:
    """Entries for N: the FP64 stage, then the FP32 stage."""
    import torch
    w = synth.custom_workload(N, max(L, N), P, seed=5000 + N, n_extra=min(4, N - 1), k_max=4)
    S = synth.make_library(w)
    X, s = synth.make_cube_device(w, S, dev)
    lib = linmin.Library(S)
    entries = []
    try:
        for stage, precision in ((linmin.STAGE_FP64, "fp64"), (linmin.STAGE_FP32, "mixed")):
            ref = lib.unmix(X, s, precision=precision, cov="none")
            torch.cuda.synchronize()
            a_ref, st_ref = ref["a"].cpu().numpy(), ref["status"].cpu().numpy()
            times, rejected = {}, {}
            for fam, lanes in candidates(N, stage):
                name = FAMILY_NAMES[fam] + (f"/{lanes}" if lanes else "")
                linmin.set_kernel(N, stage, fam, lanes)
                out = lib.unmix(X, s, precision=precision, cov="none")
                torch.cuda.synchronize()
                a, st = out["a"].cpu().numpy(), out["status"].cpu().numpy()
                both = (st == 0) & (st_ref == 0)
                da = float(np.abs(a[both] - a_ref[both]).max()) if both.any() else 0.0
                if da > 1e-6 or (st != st_ref).mean() > 1e-3:
                    rejected[name] = {"max_abs_coeff_diff": da, "status_mismatch": float((st != st_ref).mean())}
                    log(f"  N={N} {precision} {name}: rejected {rejected[name]}")
                    continue
                ms = _time(lambda: lib.unmix(X, s, precision=precision, cov="none"), reps)
                times[name] = (ms, fam, lanes)
                log(f"  N={N} {precision} {name}: {ms:.3f} ms ({1e6 * ms / P:.1f} ns/pixel)")
            best = min(times, key=lambda k: times[k][0])
            _, fam, lanes = times[best]
            linmin.set_kernel(N, stage, fam, lanes)  # keep it for the next stage's measurement
            entries.append({"N": N, "stage": "fp64" if stage == linmin.STAGE_FP64 else "fp32",
                            "family": FAMILY_NAMES[fam], "lanes": lanes,
                            "ms": {k: round(v[0], 4) for k, v in times.items()},
                            "rejected": rejected})
            log(f"N={N} {precision}: {best}")
    finally:
        lib.close()
    return entries


def install(path: str = TABLE) -> int:
    """Install the choices of a tuning table; returns how many were taken
    (entries naming a kernel this build does not have are skipped)."""
    with open(path) as f:
        table = json.load(f)
    n = 0
    for e in table.get("entries", []):
        stage = linmin.STAGE_FP64 if e["stage"] == "fp64" else linmin.STAGE_FP32
        rc = linmin.load().linmin_set_kernel(int(e["N"]), stage, linmin.KERNELS[e["family"]], int(e.get("lanes", 0)))
        n += rc == linmin.OK
    return n


def main(argv=None) -> None:
    import torch
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sizes", default=",".join(map(str, SIZES)))
    ap.add_argument("--L", type=int, default=240)
    ap.add_argument("--pixels", type=int, default=131072)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    linmin.load(tuning=False)
    t0 = time.time()
    entries = []
    for N in (int(x) for x in args.sizes.split(",")):
        P = args.pixels if N <= 64 else max(args.pixels // 4, 4096)
        entries += tune_size(N, args.L, P, args.reps, dev)
    prop = torch.cuda.get_device_properties(dev)
    table = {"device": prop.name, "arch": getattr(prop, "gcnArchName", ""), "L": args.L,
             "pixels": args.pixels, "workload": "orbital-cube distributions (1-4 minerals + 4 extras, "
             "sigma ~ U[0.002, 0.01]), cov none", "seconds": round(time.time() - t0, 1), "entries": entries}
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"wrote {args.out}: {len(entries)} entries")


if __name__ == "__main__":
    main()
