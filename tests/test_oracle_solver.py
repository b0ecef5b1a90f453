"""Pins of the oracle's nested solver (section 2): dense LU, free-field FFT, gauge covariance (CPU)."""
import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests import helpers as H


def _fields(L, kappa, seed, eps=0.25):
    U = synth.gauge_field(L, eps, seed)
    return U, synth.clover_inverse(L, U, 1.0, kappa)


@pytest.mark.parametrize("outer_kind", [0, 1])
def test_solve_matches_dense_lu(orc, outer_kind):
    L, B, S = (4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2)
    kappa = 0.125
    U, F = _fields(L, kappa, 41)
    b = synth.gaussian_spinor(L, 42)
    D = H.dense_operator(lambda p: orc.dslash(L, U, F, kappa, p), 256)
    xs = np.linalg.solve(D, b.reshape(-1))
    x, st, ok = orc.solve(L, B, S, U, F, orc.params(kappa, outer_kind=outer_kind), b, tol=1e-10)
    assert ok and st["relres"] <= 1e-10
    rr = np.linalg.norm(b.reshape(-1) - D @ x.reshape(-1)) / np.linalg.norm(b)
    assert rr <= 1.01e-10
    assert np.linalg.norm(x.reshape(-1) - xs) / np.linalg.norm(xs) < 1e-8


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1)])
def test_free_field_solve_matches_fft(orc, bc):
    L, B, S = (4, 4, 4, 8), (2, 2, 2, 4), (2, 2, 2, 2)
    kappa = 0.1
    U, F = synth.unit_gauge(L), synth.unit_clover(L)
    b = synth.gaussian_spinor(L, 43)
    x, st, ok = orc.solve(L, B, S, U, F, orc.params(kappa), b, tol=1e-12, bc=bc)
    assert ok
    xf = H.free_field_solve(L, kappa, b, bc=bc)
    assert np.linalg.norm(x - xf) / np.linalg.norm(xf) < 1e-10


def test_solve_gauge_covariance(orc):
    L, B, S = (8, 4, 4, 4), (4, 2, 2, 2), (2, 2, 2, 2)
    kappa = 0.125
    V = int(np.prod(L))
    U, F = _fields(L, kappa, 44)
    g = synth.random_su3_field(V, 45)
    b = synth.gaussian_spinor(L, 46)
    prm = orc.params(kappa)
    x, _, ok1 = orc.solve(L, B, S, U, F, prm, b, tol=1e-12)
    xg, _, ok2 = orc.solve(L, B, S, H.gauge_transform(L, U, g), H.transform_clover(F, g), prm,
                           H.transform_spinor(b, g), tol=1e-12)
    assert ok1 and ok2
    want = H.transform_spinor(x, g)
    assert np.linalg.norm(xg - want) / np.linalg.norm(want) < 1e-10


def test_inner_solver_reduces_residual(orc):
    L, B, S = (8, 8, 4, 4), (4, 4, 2, 2), (2, 2, 2, 2)
    kappa = 0.125
    U, F = _fields(L, kappa, 47)
    r = synth.gaussian_spinor(L, 48)
    e, it = orc.inner_bicgstab(L, B, S, U, F, orc.params(kappa, tol_inner=1e-3), r)
    res = np.linalg.norm(r - orc.dslash(L, U, F, kappa, e)) / np.linalg.norm(r)
    assert it >= 1 and res <= 1e-3 * 1.0001


@pytest.mark.slow
def test_plain_method_8to4(orc):
    """The plain-method workload: 8^4, kappa 0.120, 4^4 blocks, 2^4 sub-blocks, 4 SSOR sweeps."""
    L, B, S = (8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2)
    kappa = 0.120
    U, F = _fields(L, kappa, 1)
    b = synth.gaussian_spinor(L, 1001)
    x, st, ok = orc.solve(L, B, S, U, F, orc.params(kappa), b, tol=1e-10)
    assert ok and st["relres"] <= 1e-10
    r = b - orc.dslash(L, U, F, kappa, x)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
