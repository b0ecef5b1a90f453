"""Pins of the oracle's spin algebra, gauge fields and clover term (CPU)."""
import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests import helpers as H


def test_gamma_clifford_and_hermitian(orc):
    g = [orc.gamma(mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * np.eye(4) * (mu == nu), atol=0)
    g5 = orc.gamma(4)
    assert np.array_equal(g5, np.diag([1, 1, -1, -1]).astype(complex))
    assert np.allclose(g[0] @ g[1] @ g[2] @ g[3], g5)
    # the generator's basis is the same one
    assert np.array_equal(np.stack(g), synth.gamma_matrices())


def test_projectors_rank_two_and_sigma_block_diagonal(orc):
    g = [orc.gamma(mu) for mu in range(4)]
    for mu in range(4):
        for s in (1, -1):
            P = np.eye(4) - s * g[mu]
            assert np.linalg.matrix_rank(P) == 2
            assert np.allclose(P @ P, 2 * P)
        for nu in range(4):
            sig = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
            assert np.allclose(sig, sig.conj().T)
            assert np.all(sig[:2, 2:] == 0) and np.all(sig[2:, :2] == 0)


def test_su3_fields_and_plaquette(orc):
    L = (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.25, 1)
    Ud = np.swapaxes(U.conj(), -1, -2)
    assert np.abs(Ud @ U - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
    # weak field: plaquette near 1, and exactly 1 for the unit field
    assert 0.80 < orc.plaquette(L, U) < 0.90
    assert orc.plaquette(L, synth.unit_gauge(L)) == pytest.approx(1.0, abs=1e-15)


def test_clover_unit_field_and_inverse(orc):
    L = (4, 4, 4, 4)
    F1 = orc.clover_inv(L, synth.unit_gauge(L), 1.0, 0.125)
    assert np.abs(F1 - np.eye(6)).max() < 1e-15
    U = synth.gauge_field(L, 0.25, 3)
    A = orc.clover_A(L, U, 1.0, 0.125)
    # A is hermitian and commutes with gamma5 (no coupling between the chiral halves)
    assert np.abs(A - np.swapaxes(A.conj(), -1, -2)).max() < 1e-15
    assert np.abs(A[:, :6, 6:]).max() == 0 and np.abs(A[:, 6:, :6]).max() == 0
    F = orc.clover_inv(L, U, 1.0, 0.125)
    for k in range(2):
        blk = A[:, 6 * k : 6 * k + 6, 6 * k : 6 * k + 6]
        assert np.abs(F[:, k] @ blk - np.eye(6)).max() < 1e-13
    # the input generator's clover field agrees with the oracle's
    assert np.abs(synth.clover_inverse(L, U, 1.0, 0.125) - F).max() < 1e-13


def test_clover_gauge_covariance(orc):
    L = (4, 4, 4, 4)
    V = 256
    U = synth.gauge_field(L, 0.3, 5)
    g = synth.random_su3_field(V, 77)
    F = orc.clover_inv(L, U, 1.0, 0.13)
    Fg = orc.clover_inv(L, H.gauge_transform(L, U, g), 1.0, 0.13)
    assert np.abs(Fg - H.transform_clover(F, g)).max() < 1e-13


def _abelian_flux_links(L, mu, nu, k):
    """U_nu(n) = exp(i phi n_mu T), T = diag(1, -1, 0), phi = 2 pi k / L_mu; all other links 1.
    Every mu-nu plaquette leaf around any site is then exp(i phi T) (the flux closes
    periodically because phi L_mu is a multiple of 2 pi and T has integer eigenvalues)."""
    V = int(np.prod(L))
    U = synth.unit_gauge(L).copy()
    phi = 2 * np.pi * k / L[mu]
    nmu = H.coords(L)[:, mu]
    ph = np.exp(1j * phi * np.outer(nmu, [1.0, -1.0, 0.0]))  # [V, 3] diagonal of exp(i phi n_mu T)
    U[:, nu] = 0
    for a in range(3):
        U[:, nu, a, a] = ph[:, a]
    assert U.shape == (V, 4, 3, 3)
    return U, phi


@pytest.mark.parametrize("mu,nu", [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)])
def test_clover_uniform_abelian_flux_closed_form(orc, mu, nu):
    """Eq. (2.2)'s clover term for a uniform abelian flux through the mu-nu planes.  The four
    leaves are exp(i phi T), so the clover field strength is exactly F_mu_nu = sin(phi) T, every
    other plane carries none, and A = 1 - (c_SW kappa / 2) sum_{rho != sigma} sigma_rho_sigma
    F_rho_sigma = 1 - c_SW kappa sigma_mu_nu (x) sin(phi) T.  sigma_mu_nu squares to 1, so A has
    eigenvalues 1 - c_SW kappa sin(phi) (4 times), 1 + c_SW kappa sin(phi) (4 times) and 1 (4
    times), and on sigma_mu_nu = +1 spinors of colour 0 it is 1 - c_SW kappa sin(phi).  A wrong
    normalisation (kappa/2 over mu < nu, 1/(4i)) moves the eigenvalues; a flipped sign or a
    reversed leaf orientation swaps the last eigenvalue with 1 + c_SW kappa sin(phi)."""
    L = (6, 4, 8, 4)
    csw, kappa = 1.3, 0.11
    U, phi = _abelian_flux_links(L, mu, nu, 1)
    A = orc.clover_A(L, U, csw, kappa)
    s = np.sin(phi)
    want = np.sort(np.r_[np.full(4, 1 - csw * kappa * s), np.full(4, 1 + csw * kappa * s), np.ones(4)])
    g = [orc.gamma(m) for m in range(4)]
    sig = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
    assert np.abs(sig @ sig - np.eye(4)).max() < 1e-15
    w, X = np.linalg.eigh(sig)
    plus = X[:, w > 0]  # the two spinors with sigma_mu_nu = +1
    for n in (0, 17, 100, int(np.prod(L)) - 1):
        An = A[n]
        assert np.abs(np.sort(np.linalg.eigvalsh(An)) - want).max() < 1e-14
        for j in range(2):
            chi = np.kron(plus[:, j], np.array([1.0, 0.0, 0.0]))  # index 3*alpha + a
            assert np.abs(An @ chi - (1 - csw * kappa * s) * chi).max() < 1e-14
