"""CPU-side checks of the C ABI: the library loads and exports every entry
point that include/linmin.h declares; the binding mirrors the header's
constants.  No GPU call is made."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1402_2518_amd import linmin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "linmin.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(linmin_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("linmin_create_library", "linmin_unmix", "linmin_destroy_library",
                 "linmin_workspace_bytes", "linmin_strerror", "linmin_default_opts"):
        assert want in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(linmin.LIB_PATH):
        pytest.fail("liblinmin.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(linmin.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(linmin.EXPORTS)


def test_constants_match_header():
    txt = open(HEADER).read()
    defs = dict(re.findall(r"#define (LINMIN_\w+) \(?(-?\d+)u?\)?", txt))
    assert int(defs["LINMIN_OK"]) == linmin.OK
    assert int(defs["LINMIN_EINVAL"]) == linmin.EINVAL
    assert int(defs["LINMIN_EUNSUPPORTED"]) == linmin.EUNSUPPORTED
    assert int(defs["LINMIN_ESCRATCH"]) == linmin.ESCRATCH
    m = re.search(r"#define LINMIN_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == linmin.NOALLOC_SCRATCH_BYTES
    assert int(defs["LINMIN_MIXED"]) == linmin.MIXED
    assert int(defs["LINMIN_COV_DIAG"]) == linmin.COV_DIAG
    assert int(defs["LINMIN_PX_INEXACT"]) == linmin.PX_INEXACT
    assert int(defs["LINMIN_N_MAX"]) == linmin.N_MAX
    assert (int(defs["LINMIN_STO"]), int(defs["LINMIN_SLO"]), int(defs["LINMIN_POS"])) == \
        (linmin.STO, linmin.SLO, linmin.POS)


def test_opts_struct_layout(tmp_path):
    # field offsets and size of linmin_opts and linmin_job as the C compiler
    # lays them out from the header, against the ctypes mirrors
    include = os.path.join(ROOT, "include")
    src = tmp_path / "layout.c"
    fields = [f for f, _ in linmin.Opts._fields_]
    jfields = [f for f, _ in linmin.Job._fields_]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "linmin.h"', "int main(void) {",
             '  printf("%zu\\n", sizeof(linmin_opts));', '  printf("%zu\\n", sizeof(linmin_job));']
    lines += [f'  printf("%zu\\n", offsetof(linmin_opts, {f}));' for f in fields]
    lines += [f'  printf("%zu\\n", offsetof(linmin_job, {f}));' for f in jfields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", include, str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == ctypes.sizeof(linmin.Opts) and vals[1] == ctypes.sizeof(linmin.Job)
    assert vals[2:2 + len(fields)] == [getattr(linmin.Opts, f).offset for f in fields]
    assert vals[2 + len(fields):] == [getattr(linmin.Job, f).offset for f in jfields]


def test_strerror_and_defaults_without_gpu():
    lib = linmin.load()
    assert lib.linmin_strerror(-4).decode().startswith("matrix not")
    o = linmin.default_opts()
    assert o.maxit == 200 and o.tol_mu == 1e-13 and o.precision == linmin.FP64
    assert o.mu_switch == 1e-10
    assert o.constraint == linmin.STO
    h = ctypes.c_void_p()
    # argument errors are reported before any device work
    import numpy as np
    S = np.ones((5, 3), np.float32)
    assert lib.linmin_create_library(S.ctypes.data_as(ctypes.c_void_p), 3, 5, None, ctypes.byref(h)) == linmin.EINVAL
    assert lib.linmin_create_library(None, 3, 2, None, ctypes.byref(h)) == linmin.EINVAL
    assert lib.linmin_unmix(None, None, 0, None, None, None, None, None) == linmin.EINVAL
    assert lib.linmin_destroy_library(None) == linmin.EINVAL
    # batches: misuse is reported before any device work
    assert lib.linmin_batch_create(None, 0, None, None) == linmin.EINVAL
    assert lib.linmin_batch_create(None, -1, None, ctypes.byref(h)) == linmin.EINVAL
    assert lib.linmin_batch_create(None, 2, None, ctypes.byref(h)) == linmin.EINVAL
    bad = linmin.default_opts(precision=7)
    assert lib.linmin_batch_create(None, 0, ctypes.byref(bad), ctypes.byref(h)) == linmin.EINVAL
    assert lib.linmin_batch_run(None, None) == linmin.EINVAL
    assert lib.linmin_batch_destroy(None) == linmin.EINVAL
    assert lib.linmin_batch_device_bytes(None) == 0
    keep_opts = linmin.default_opts()
    keep_opts.keep = 16  # any non-NULL pointer: batches refuse the per-pixel selection before device work
    assert lib.linmin_batch_create(None, 0, ctypes.byref(keep_opts), ctypes.byref(h)) == linmin.EINVAL
    # detection entry points check their arguments first
    assert lib.linmin_error_maps(None, 5, None, None, None, 1, None, None, None) == linmin.EINVAL
    assert lib.linmin_thresholds(0, 5, None, None, None, None) == linmin.EINVAL
    assert lib.linmin_thresholds(4, 5, None, None, None, None) == linmin.EINVAL
    assert lib.linmin_detect(129, 5, None, None, None, None, 1.0, None, None) == linmin.EINVAL
    assert lib.linmin_detect(4, 5, None, None, None, None, 1.0, None, None) == linmin.EINVAL
    assert lib.linmin_detect(4, 0, None, None, None, None, 1.0, None, None) == linmin.OK


def test_job_struct_layout():
    # linmin_job: library handle, cube, P, sigma, then five output pointers
    assert ctypes.sizeof(linmin.Job) == 9 * 8
    assert linmin.Job.P.offset == 16


def test_kernel_choice_without_gpu():
    # the choice of interior-point kernel family is host state only
    txt = open(HEADER).read()
    defs = dict(re.findall(r"#define (LINMIN_\w+) \(?(-?\d+)u?\)?", txt))
    assert (int(defs["LINMIN_KERNEL_ROWCYCLIC"]), int(defs["LINMIN_KERNEL_TILE"]), int(defs["LINMIN_KERNEL_GROUP"]),
            int(defs["LINMIN_KERNEL_TILE32"])) == (linmin.KERNEL_ROWCYCLIC, linmin.KERNEL_TILE,
                                                  linmin.KERNEL_GROUP, linmin.KERNEL_TILE32)
    assert (int(defs["LINMIN_STAGE_FP64"]), int(defs["LINMIN_STAGE_FP32"])) == (linmin.STAGE_FP64, linmin.STAGE_FP32)
    lib = linmin.load()
    # the measured table is installed at load: every entry is in force
    from paper_1402_2518_amd import autotune
    import json
    table = json.load(open(linmin.TUNING_PATH))["entries"] if os.path.exists(linmin.TUNING_PATH) else []
    for e in table:
        st = linmin.STAGE_FP64 if e["stage"] == "fp64" else linmin.STAGE_FP32
        assert linmin.get_kernel_lanes(e["N"], st) == (linmin.KERNELS[e["family"]], e["lanes"]), e
    # the default rule (matrix cores first), with the table's choices cleared
    for n in range(1, linmin.N_MAX + 1):
        for st in (linmin.STAGE_FP64, linmin.STAGE_FP32):
            linmin.set_kernel(n, st, "default")
    try:
        _default_rule(lib)
    finally:
        if table:
            assert autotune.install(linmin.TUNING_PATH) == len(table)


def _default_rule(lib):
    assert linmin.get_kernel(36, linmin.STAGE_FP64) == linmin.KERNEL_TILE
    assert linmin.get_kernel(96, linmin.STAGE_FP64) == linmin.KERNEL_ROWCYCLIC
    assert linmin.get_kernel(36, linmin.STAGE_FP32) == linmin.KERNEL_TILE32
    assert linmin.get_kernel(64, linmin.STAGE_FP32) == linmin.KERNEL_TILE32  # column-cyclic FP32 tiles
    assert linmin.get_kernel(8, linmin.STAGE_FP32) == linmin.KERNEL_TILE32
    try:
        linmin.set_kernel(33, linmin.STAGE_FP64, "group")  # same padded size as 36
        assert linmin.get_kernel(36, linmin.STAGE_FP64) == linmin.KERNEL_GROUP
        assert linmin.get_kernel(32, linmin.STAGE_FP64) == linmin.KERNEL_TILE
    finally:
        linmin.set_kernel(36, linmin.STAGE_FP64, "default")
    assert linmin.get_kernel(36, linmin.STAGE_FP64) == linmin.KERNEL_TILE
    # not compiled for that size or stage; out of range
    assert lib.linmin_set_kernel(96, linmin.STAGE_FP64, linmin.KERNEL_TILE, 0) == linmin.EUNSUPPORTED
    assert lib.linmin_set_kernel(36, linmin.STAGE_FP32, linmin.KERNEL_TILE, 0) == linmin.EUNSUPPORTED
    assert lib.linmin_set_kernel(36, linmin.STAGE_FP32, linmin.KERNEL_GROUP, 3) == linmin.EUNSUPPORTED
    assert lib.linmin_set_kernel(36, linmin.STAGE_FP32, linmin.KERNEL_TILE32, 8) == linmin.EINVAL
    assert lib.linmin_set_kernel(0, linmin.STAGE_FP64, 0, 0) == linmin.EINVAL
    assert lib.linmin_set_kernel(129, linmin.STAGE_FP64, 0, 0) == linmin.EINVAL
    assert lib.linmin_set_kernel(36, 2, 0, 0) == linmin.EINVAL
    assert lib.linmin_set_kernel(36, linmin.STAGE_FP64, 9, 0) == linmin.EINVAL
    assert lib.linmin_get_kernel(36, 5, None) == linmin.EINVAL
    # group widths: the default is the first listed shape, others by choice
    try:
        linmin.set_kernel(64, linmin.STAGE_FP32, "group")
        assert linmin.get_kernel_lanes(64, linmin.STAGE_FP32) == (linmin.KERNEL_GROUP, 16)
        linmin.set_kernel(64, linmin.STAGE_FP32, "group", 8)
        assert linmin.get_kernel_lanes(64, linmin.STAGE_FP32) == (linmin.KERNEL_GROUP, 8)
    finally:
        linmin.set_kernel(64, linmin.STAGE_FP32, "default")
    assert linmin.get_kernel_lanes(64, linmin.STAGE_FP32) == (linmin.KERNEL_TILE32, 0)
