"""linmin_unmix_noalloc (work areas in the library's fixed device array)
against linmin_unmix (stream-ordered allocations) through the C ABI.

Both run the same kernels on the same inputs, and no byte of the work area
is read before the call writes it, so the outputs must be identical bit for
bit, also when the array still holds a larger previous call's data.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _outputs(lib, P, N, cov):
    dev = torch.device("cuda:0")
    per = {"full": N * N, "diag": N}[cov]
    return {"a": torch.full((P, N), np.nan, dtype=torch.float64, device=dev),
            "cov": torch.full((P * per,), np.nan, dtype=torch.float64, device=dev),
            "status": torch.full((P,), 255, dtype=torch.uint8, device=dev),
            "iters": torch.full((P,), -1, dtype=torch.int32, device=dev),
            "objective": torch.full((P,), np.nan, dtype=torch.float64, device=dev)}


def _run(lib, Xt, st, N, precision, cov, noalloc):
    o = _outputs(lib, Xt.shape[0], N, cov)
    lib.unmix_into(Xt, st, o["a"], o["cov"], o["status"], o["iters"], o["objective"],
                   precision=precision, cov=cov, noalloc=noalloc)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def test_noalloc_matches_unmix():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1402_2518_amd import linmin, synth
    linmin.load()
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS["orbital"]
    S = synth.make_library(w)
    X, s = synth.make_cube(w, p1=40000)
    lib = linmin.Library(S)
    N = lib.N
    Xt, st = torch.from_numpy(X).to(dev), torch.from_numpy(s).to(dev)
    # two calls in a row, the second smaller (the array keeps the first
    # call's data), in both precisions and two covariance layouts
    for P, precision, cov in ((40000, "fp64", "full"), (3001, "fp64", "full"),
                              (40000, "mixed", "full"), (517, "mixed", "diag")):
        _say(f"[gpu] noalloc vs unmix P={P} {precision} cov={cov}")
        assert lib.workspace_bytes(P, precision, cov) <= linmin.NOALLOC_SCRATCH_BYTES
        ref = _run(lib, Xt[:P], st[:P], N, precision, cov, noalloc=False)
        got = _run(lib, Xt[:P], st[:P], N, precision, cov, noalloc=True)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (k, P, precision, cov)
        assert (ref["status"] == 0).mean() > 0.95
    # a call beyond the array is refused before anything is enqueued
    P = 200000
    assert lib.workspace_bytes(P, "fp64", "full") > linmin.NOALLOC_SCRATCH_BYTES
    big = torch.zeros((P, lib.L), dtype=torch.float32, device=dev)
    o = _outputs(lib, P, N, "diag")
    with pytest.raises(linmin.LinminError) as e:
        lib.unmix_into(big, None, o["a"], o["cov"], o["status"], None, None, cov="diag", noalloc=True)
    assert e.value.code == linmin.ESCRATCH
    torch.cuda.synchronize()
    assert (o["status"].cpu().numpy() == 255).all()
    lib.close()
