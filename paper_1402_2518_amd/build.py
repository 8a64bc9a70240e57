"""Build lib_linmin (HIP, gfx950) into ``paper_1402_2518_amd/liblinmin.so``.

Every interior-point shape listed in ``csrc/ipm_shapes.def`` is compiled as
its own object so the shapes build in parallel.  Objects go to ``_build/``
next to this file; the shared library is linked in place.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblinmin.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", CSRC]


def shapes():
    txt = open(os.path.join(CSRC, "ipm_shapes.def")).read()
    return re.findall(r"^LM_SHAPE\((\w+),\s*(\d+),\s*(\d+)\)", txt, re.M)


def tiles():
    txt = open(os.path.join(CSRC, "ipm_shapes.def")).read()
    return re.findall(r"^LM_TILE\((\d+)\)", txt, re.M)


def tile32s():
    txt = open(os.path.join(CSRC, "ipm_shapes.def")).read()
    return re.findall(r"^LM_TILE32\((\d+)\)", txt, re.M)


def cc32s():
    txt = open(os.path.join(CSRC, "ipm_shapes.def")).read()
    return re.findall(r"^LM_CC32\((\d+),\s*(\d+)\)", txt, re.M)


def rc_tiles():
    txt = open(os.path.join(CSRC, "ipm_shapes.def")).read()
    return re.findall(r"^LM_RC\((\d+),\s*(\d+)\)", txt, re.M)


def _compile(src, obj, extra=()):
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr[-4000:]}")
    return obj


# Instruction scheduling per four-pixel FP64 tile shape.  The T = 16 shape
# (N = 49..64) runs at one wave per SIMD with spilled registers, so nothing
# hides its latencies but the order of its own instructions; LLVM's
# latency-first ("max-ilp") strategy spills less there (243 vs 312 VGPRs)
# and runs 4.5 % faster on the precision cube (69.3 vs 72.7 ms).  Every other
# interior-point shape measured slower with it (T = 9 and 12, the FP32 and
# row-cyclic kernels) and keeps the default.
TILE_FLAGS = {"16": ("-mllvm", "-amdgpu-sched-strategy=max-ilp")}


def tile_flags(t: str) -> tuple:
    """Compiler flags of the four-pixel FP64 tile shape T = t."""
    return (f"-DLM_TILE_T={t}",) + TILE_FLAGS.get(t, ())


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = []
    for name in ("gemm.hip", "setup.hip", "cov.hip", "detect.hip", "linmin.cpp", "ipm_dispatch.cpp", "noalloc.hip"):
        units.append((os.path.join(CSRC, name), os.path.join(BUILD, name + ".o"), ()))
    for t, nc, g in shapes():
        units.append((os.path.join(CSRC, "ipm.hip"), os.path.join(BUILD, f"ipm_{t}_{nc}_{g}.o"),
                      (f"-DLM_T={t}", f"-DLM_NC={nc}", f"-DLM_G={g}")))
    for t in tiles():
        units.append((os.path.join(CSRC, "ipm_tile.hip"), os.path.join(BUILD, f"ipm_tile_{t}.o"), tile_flags(t)))
    for t in tile32s():
        units.append((os.path.join(CSRC, "ipm_tile32.hip"), os.path.join(BUILD, f"ipm_tile32_{t}.o"),
                      (f"-DLM_TILE32_T={t}",)))
    for t, q in cc32s():
        units.append((os.path.join(CSRC, "ipm_cc32.hip"), os.path.join(BUILD, f"ipm_cc32_{t}_{q}.o"),
                      (f"-DLM_CC32_T={t}", f"-DLM_CC32_Q={q}")))
    for t, bb in rc_tiles():
        units.append((os.path.join(CSRC, "ipm_rc.hip"), os.path.join(BUILD, f"ipm_rc_{t}_{bb}.o"),
                      (f"-DLM_RC_T={t}", f"-DLM_RC_B={bb}")))
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_compile, s, o, e) for s, o, e in units]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(objs)} objects", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
