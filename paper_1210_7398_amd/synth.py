"""Seeded synthetic inputs: SU(3) gauge fields, their inverse clover field, sources.

This module holds no solver arithmetic.  It produces the input fields that the
solver takes as given: the gauge links U, the inverse clover field F (an input
to the library, see eq. 2.2 of Boku et al., arXiv:1210.7398), and right-hand
sides.  The paper names no gauge ensemble, so seed-fixed fields of the paper's
lattice shapes stand in for them.

Interchange layout (numpy, complex128, site n = x + Lx*(y + Ly*(z + Lz*t))):
  links   [V, 4, 3, 3]   U_mu(n)[a, b], the link from n to n+mu
  clover  [V, 2, 6, 6]   two chiral 6x6 blocks, row index 3*(alpha-2k)+a
  spinor  [V, 4, 3]
"""
import numpy as np

# Gell-Mann matrices
_GM = np.zeros((8, 3, 3), np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1] = -1j
_GM[1][1, 0] = 1j
_GM[2][0, 0] = 1
_GM[2][1, 1] = -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2] = -1j
_GM[4][2, 0] = 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2] = -1j
_GM[6][2, 1] = 1j
_GM[7] = np.diag([1, 1, -2]) / np.sqrt(3)


def volume(L):
    return int(np.prod(L))


def su3_from_normals(h, eps):
    """exp(i eps H) with H = sum_a h_a lambda_a / 2 (traceless hermitian), via eigh."""
    H = np.einsum("...a,aij->...ij", h, _GM) * 0.5
    w, vec = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", vec, ph, vec.conj())


def gauge_field(L, eps, seed, device=None):
    """U_mu(n) = exp(i eps H), H Gaussian traceless hermitian, drawn as normals of shape
    (Lt, Lz, Ly, Lx, 4, 8) from numpy's default_rng(seed); returns [V, 4, 3, 3] (numpy).
    With a torch device the exponential is taken there and a torch tensor is returned (same
    draws; the eigendecomposition rounds differently)."""
    Lx, Ly, Lz, Lt = L
    rng = np.random.default_rng(seed)
    V = volume(L)
    h = rng.normal(size=(Lt, Lz, Ly, Lx, 4, 8)).reshape(V, 4, 8)
    if device is not None:
        import torch

        U = torch.empty((V, 4, 3, 3), dtype=torch.complex128, device=device)
        gm = torch.from_numpy(_GM).to(device)
        chunk = 1 << 20
        for s in range(0, V, chunk):
            hc = torch.from_numpy(h[s : s + chunk]).to(device).to(torch.complex128)
            X = (1j * eps * 0.5) * torch.einsum("...a,aij->...ij", hc, gm)
            U[s : s + chunk] = _su3_exp_torch(X)
        return U
    U = np.empty((V, 4, 3, 3), np.complex128)
    chunk = 1 << 18
    for s in range(0, V, chunk):
        U[s : s + chunk] = su3_from_normals(h[s : s + chunk], eps)
    return U


def _su3_exp_torch(X, squarings=6, order=10):
    """exp(X) for traceless anti-hermitian 3x3 X by scaling and squaring of a Taylor series
    (|X| / 2^6 < 0.05 here, so order 10 is exact to rounding), then projected onto SU(3):
    rows 0 and 1 orthonormalised, row 2 = conj(row0 x row1)."""
    import torch

    Y = X / (2**squarings)
    eye = torch.eye(3, dtype=X.dtype, device=X.device).expand_as(Y)
    E = eye.clone()
    term = eye.clone()
    for k in range(1, order + 1):
        term = (term @ Y) / k
        E = E + term
    for _ in range(squarings):
        E = E @ E
    r0 = E[..., 0, :]
    r0 = r0 / torch.linalg.vector_norm(r0, dim=-1, keepdim=True)
    r1 = E[..., 1, :]
    r1 = r1 - (r0.conj() * r1).sum(-1, keepdim=True) * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.linalg.cross(r0, r1).conj()
    return torch.stack([r0, r1, r2], dim=-2)


def _inverse_torch(A):
    """Batched inverse by Gauss-Jordan elimination without pivoting (A = 1 - small term here,
    so the pivots stay near 1)."""
    import torch

    n = A.shape[-1]
    M = torch.cat([A, torch.eye(n, dtype=A.dtype, device=A.device).expand_as(A)], dim=-1).clone()
    for k in range(n):
        M[..., k, :] = M[..., k, :] / M[..., k, k : k + 1]
        f = M[..., :, k : k + 1].clone()
        f[..., k, :] = 0
        M = M - f * M[..., k : k + 1, :]
    return M[..., n:].contiguous()


def unit_gauge(L):
    V = volume(L)
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()


def random_su3_field(V, seed, eps=1.0):
    """One SU(3) matrix per site (for gauge transformations)."""
    rng = np.random.default_rng(seed)
    return su3_from_normals(rng.normal(size=(V, 8)), eps)


def gaussian_spinor(L, seed):
    """Complex Gaussian source: Re and Im i.i.d. N(0,1) per component, [V, 4, 3]."""
    rng = np.random.default_rng(seed)
    V = volume(L)
    return (rng.normal(size=(V, 4, 3)) + 1j * rng.normal(size=(V, 4, 3))).astype(np.complex128)


def point_source(L, spin, colour, site=0):
    V = volume(L)
    b = np.zeros((V, 4, 3), np.complex128)
    b[site, spin, colour] = 1.0
    return b


# --- chiral gamma basis used by the whole project (gamma5 = diag(1,1,-1,-1)) ------------
_PAULI = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], np.complex128)


def gamma_matrices():
    g = np.zeros((4, 4, 4), np.complex128)
    for k in range(3):
        g[k, :2, 2:] = -1j * _PAULI[k]
        g[k, 2:, :2] = 1j * _PAULI[k]
    g[3, :2, 2:] = np.eye(2)
    g[3, 2:, :2] = np.eye(2)
    return g


def _shift(f, L, mu, step):
    """Field at n + step*mu (periodic), for a torch tensor f of shape [V, ...]."""
    import torch

    Lx, Ly, Lz, Lt = L
    g = f.reshape((Lt, Lz, Ly, Lx) + tuple(f.shape[1:]))
    return torch.roll(g, -step, dims=3 - mu).reshape(f.shape)


def clover_inverse(L, U, csw, kappa, device=None):
    """Inverse clover field F(n) = (1 - c_SW kappa sum_{mu<nu} sigma_mu_nu F_mu_nu(n))^-1 as two
    chiral 6x6 blocks [V, 2, 6, 6]; F_mu_nu is the four-leaf clover (Q - Q^+)/(8i), traceless,
    sigma_mu_nu = (i/2)[gamma_mu, gamma_nu].  Periodic gauge field (no fermion phases).
    Computed with torch on the host (batched 3x3 products), returned as numpy."""
    import torch

    V = volume(L)
    g = gamma_matrices()
    on_dev = isinstance(U, torch.Tensor)
    dev = U.device if on_dev else torch.device("cpu")
    Ut = U if on_dev else torch.from_numpy(np.ascontiguousarray(U))
    dag = lambda m: m.conj().transpose(-1, -2).contiguous()
    # A is block diagonal in the chiral basis: build its two 6x6 blocks directly
    A = torch.zeros((V, 2, 6, 6), dtype=torch.complex128, device=dev)
    A[:] = torch.eye(6, dtype=torch.complex128, device=dev)
    eye3 = torch.eye(3, dtype=torch.complex128, device=dev)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Umu = Ut[:, mu].contiguous()
            Unu = Ut[:, nu].contiguous()
            Umu_pnu = _shift(Umu, L, nu, 1)
            Unu_pmu = _shift(Unu, L, mu, 1)
            Umu_mmu = _shift(Umu, L, mu, -1)
            Unu_mmu = _shift(Unu, L, mu, -1)
            Umu_mmu_pnu = _shift(Umu_mmu, L, nu, 1)
            Umu_mmu_mnu = _shift(Umu_mmu, L, nu, -1)
            Unu_mmu_mnu = _shift(Unu_mmu, L, nu, -1)
            Umu_mnu = _shift(Umu, L, nu, -1)
            Unu_mnu = _shift(Unu, L, nu, -1)
            Unu_pmu_mnu = _shift(Unu_pmu, L, nu, -1)
            Q = Umu @ Unu_pmu @ dag(Umu_pnu) @ dag(Unu)
            Q += Unu @ dag(Umu_mmu_pnu) @ dag(Unu_mmu) @ Umu_mmu
            Q += dag(Umu_mmu) @ dag(Unu_mmu_mnu) @ Umu_mmu_mnu @ Unu_mnu
            Q += dag(Unu_mnu) @ Umu_mnu @ Unu_pmu_mnu @ dag(Umu)
            Fmn = (Q - dag(Q)) / 8j
            tr = Fmn.diagonal(dim1=1, dim2=2).sum(-1) / 3.0
            Fmn -= tr[:, None, None] * eye3
            sig = torch.from_numpy(0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])).to(dev)
            for k in range(2):
                sk = sig[2 * k : 2 * k + 2, 2 * k : 2 * k + 2]
                blk = sk[None, :, None, :, None] * Fmn[:, None, :, None, :]
                A[:, k] -= csw * kappa * blk.reshape(V, 6, 6)
    if on_dev:
        return _inverse_torch(A)
    return np.ascontiguousarray(torch.linalg.inv(A).numpy())


def unit_clover(L):
    V = volume(L)
    return np.broadcast_to(np.eye(6, dtype=np.complex128), (V, 2, 6, 6)).copy()
