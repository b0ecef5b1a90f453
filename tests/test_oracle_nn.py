"""Pins of the oracle's learned stage: Wilson special case, gauge equivariance, adjoint,
finite-difference gradients, Adam (CPU)."""
import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests import helpers as H


def _rand_w(rng, cout, cin, scale=0.3):
    return scale * (rng.normal(size=(9, cout, cin, 4, 4)) + 1j * rng.normal(size=(9, cout, cin, 4, 4)))


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1)])
def test_layer_wilson_special_case(orc, bc):
    """One channel, W_0 = 1, W_{+mu} = -kappa (1 - gamma_mu), W_{-mu} = -kappa (1 + gamma_mu) is D at F = 1."""
    L = (4, 4, 4, 6)
    kappa = 0.13
    U = synth.gauge_field(L, 0.3, 8)
    g = [orc.gamma(mu) for mu in range(4)]
    W = np.zeros((9, 1, 1, 4, 4), np.complex128)
    W[0, 0, 0] = np.eye(4)
    for mu in range(4):
        W[1 + 2 * mu, 0, 0] = -kappa * (np.eye(4) - g[mu])
        W[2 + 2 * mu, 0, 0] = -kappa * (np.eye(4) + g[mu])
    psi = synth.gaussian_spinor(L, 9)
    out = orc.nn_layer(L, U, W, psi[None], bc)[0]
    want = orc.dslash(L, U, synth.unit_clover(L), kappa, psi, bc=bc)
    assert np.abs(out - want).max() < 1e-13


def test_layer_and_network_gauge_equivariance(orc):
    L = (4, 4, 4, 4)
    V = 256
    rng = np.random.default_rng(3)
    U = synth.gauge_field(L, 0.3, 10)
    gt = synth.random_su3_field(V, 11)
    Ug = H.gauge_transform(L, U, gt)
    x = np.stack([synth.gaussian_spinor(L, 12 + c) for c in range(3)])
    W = _rand_w(rng, 2, 3)
    lhs = orc.nn_layer(L, Ug, W, np.stack([H.transform_spinor(xc, gt) for xc in x]))
    rhs = np.stack([H.transform_spinor(o, gt) for o in orc.nn_layer(L, U, W, x)])
    assert np.abs(lhs - rhs).max() < 1e-12
    Ws = [_rand_w(rng, co, ci, 0.2) for ci, co in orc.NN_SHAPES]
    r = synth.gaussian_spinor(L, 20)
    z1, _ = orc.nn_forward(L, Ug, Ws, H.transform_spinor(r, gt))
    z0, _ = orc.nn_forward(L, U, Ws, r)
    assert np.abs(z1 - H.transform_spinor(z0, gt)).max() < 1e-11 * np.abs(z0).max()


def test_layer_adjoint_identity(orc):
    L = (4, 4, 4, 4)
    rng = np.random.default_rng(4)
    U = synth.gauge_field(L, 0.3, 13)
    W = _rand_w(rng, 3, 2)
    x = np.stack([synth.gaussian_spinor(L, 30 + c) for c in range(2)])
    y = np.stack([synth.gaussian_spinor(L, 40 + c) for c in range(3)])
    for bc in [(1, 1, 1, 1), (1, 1, 1, -1)]:
        lhs = np.vdot(y, orc.nn_layer(L, U, W, x, bc))
        rhs = np.vdot(orc.nn_layer_adjoint(L, U, W, y, bc), x)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_layer_linearity(orc):
    L = (4, 4, 4, 4)
    rng = np.random.default_rng(5)
    U = synth.gauge_field(L, 0.3, 14)
    W = _rand_w(rng, 2, 1)
    a, b = synth.gaussian_spinor(L, 50)[None], synth.gaussian_spinor(L, 51)[None]
    z = 0.7 + 0.2j
    lhs = orc.nn_layer(L, U, W, a + z * b)
    assert np.abs(lhs - orc.nn_layer(L, U, W, a) - z * orc.nn_layer(L, U, W, b)).max() < 1e-12


def test_network_gradient_finite_differences(orc):
    """dL/dRe W + i dL/dIm W of the full three-layer network against central differences."""
    L = (4, 4, 4, 4)
    rng = np.random.default_rng(6)
    U = synth.gauge_field(L, 0.25, 15)
    Ws = [_rand_w(rng, co, ci, 0.15) for ci, co in orc.NN_SHAPES]
    r = synth.gaussian_spinor(L, 60)
    e = synth.gaussian_spinor(L, 61)
    loss, grads = orc.nn_loss_grad(L, U, Ws, r, e)
    h = 1e-6
    for k in range(3):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in Ws[k].shape)
            for part, unit in ((0, 1.0), (1, 1j)):
                Wp = [W.copy() for W in Ws]
                Wm = [W.copy() for W in Ws]
                Wp[k][idx] += h * unit
                Wm[k][idx] -= h * unit
                fd = (orc.nn_loss_grad(L, U, Wp, r, e)[0] - orc.nn_loss_grad(L, U, Wm, r, e)[0]) / (2 * h)
                an = grads[k][idx].real if part == 0 else grads[k][idx].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (k, idx, part, fd, an)


def test_flat_weight_layout_roundtrip(orc):
    rng = np.random.default_rng(7)
    w = rng.normal(size=orc.nn_param_count())
    assert orc.nn_param_count() == 23040
    assert np.array_equal(orc.nn_flatten(orc.nn_unflatten(w)), w)


def test_adam_first_steps(orc):
    """First Adam step moves every parameter by lr*g/(|g|+eps) against the gradient; with a
    constant gradient the bias-corrected moments stay g and g^2 on later steps."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    orc.adam_step(p, g, m, v, 0.01, 1)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8))
    orc.adam_step(p, g, m, v, 0.01, 2)
    assert np.allclose(p, -0.02 * g / (np.abs(g) + 1e-8))
