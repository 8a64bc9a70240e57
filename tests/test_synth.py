"""Generator checks: shapes, value ranges, support sizes, determinism."""
import numpy as np
import pytest

from paper_1402_2518_amd import synth


def test_library_shapes_and_ranges():
    for name, w in synth.WORKLOADS.items():
        S = synth.make_library(w)
        assert S.shape == (w.N, w.L) and S.dtype == np.float32
        m = S[: w.n_minerals]
        assert m.min() > 0.0 and m.max() <= 0.6 + 1e-6
        assert np.array_equal(S, synth.make_library(w))
        if w.n_extra:
            assert np.all(S[w.n_minerals] == 1.0)


def test_cube_ranges_support_and_slices():
    w = synth.WORKLOADS["orbital"]
    S = synth.make_library(w)
    X, s, A = synth.make_cube(w, S, p1=3 * synth.CHUNK + 17, with_truth=True)
    assert X.dtype == np.float32 and s.dtype == np.float32
    assert (s >= 0.002).all() and (s <= 0.01).all()
    assert np.allclose(A.sum(1), 1.0)
    k = (A[:, : w.n_minerals] > 0).sum(1)
    assert k.min() == 1 and k.max() == 4
    assert (A[:, w.n_minerals:] > 0).all()
    # any pixel range reproduces the same bytes as the corresponding slice
    X2, s2 = synth.make_cube(w, S, p0=synth.CHUNK - 5, p1=2 * synth.CHUNK + 9)
    assert np.array_equal(X2, X[synth.CHUNK - 5: 2 * synth.CHUNK + 9])
    assert np.array_equal(s2, s[synth.CHUNK - 5: 2 * synth.CHUNK + 9])
    # noise level consistent with sigma
    resid = X.astype(float) - A @ S.astype(float)
    assert 0.9 < np.median(np.std(resid, axis=1) / s) < 1.1


def test_tiny_workload():
    w = synth.WORKLOADS["tiny"]
    X, s, A = synth.make_cube(w, with_truth=True)
    assert X.shape == (1000, 64) and (s == np.float32(0.005)).all()
    k = (A > 0).sum(1)
    assert k.min() == 1 and k.max() == 3


def test_device_cube_generator_distribution():
    torch = pytest.importorskip("torch")
    w = synth.custom_workload(20, 64, 3000, seed=5)
    S = synth.make_library(w)
    X, s = synth.make_cube_device(w, S, "cpu", chunk=1024)
    X2, s2 = synth.make_cube_device(w, S, "cpu", chunk=1024)
    assert torch.equal(X, X2) and torch.equal(s, s2)  # seeded
    assert X.shape == (3000, 64) and X.dtype == torch.float32
    sn = s.numpy()
    assert sn.min() >= 0.002 and sn.max() <= 0.01
    Xh, sh = synth.make_cube(w, S)
    # same distribution as the host generator: means and spreads agree
    assert abs(float(X.mean()) - Xh.mean()) < 0.01 and abs(float(X.std()) - Xh.std()) < 0.01
    assert abs(sn.mean() - sh.mean()) < 3e-4


def test_batch_workloads():
    ws = synth.batch_workloads(200)
    assert len(ws) == 200
    assert {w.N for w in ws} == set(synth.BATCH_N) and {w.L for w in ws} == set(synth.BATCH_L)
    P = np.array([w.P for w in ws])
    assert P.min() >= 1000 and P.max() <= 200_000 and 5e6 < P.sum() < 1.1e7
    assert all(w.N <= w.L and w.n_extra == 4 for w in ws)
