"""Test-side helpers: gauge transformations, dense probing, free-field closed forms.

These hold no solver arithmetic of the GPU path; they build the independent
checks that pin the oracle (closed forms, dense linear algebra)."""
import numpy as np

from paper_1210_7398_amd import synth


def shift(f, L, mu, step):
    Lx, Ly, Lz, Lt = L
    g = f.reshape((Lt, Lz, Ly, Lx) + f.shape[1:])
    return np.roll(g, -step, axis=3 - mu).reshape(f.shape)


def gauge_transform(L, U, g):
    """U^g_mu(n) = g(n) U_mu(n) g(n+mu)^dagger."""
    Ug = np.empty_like(U)
    for mu in range(4):
        gp = shift(g, L, mu, 1)
        Ug[:, mu] = g @ U[:, mu] @ np.swapaxes(gp.conj(), -1, -2)
    return Ug


def transform_spinor(psi, g):
    return np.einsum("nab,nsb->nsa", g, psi)


def transform_clover(F, g):
    G6 = np.zeros((g.shape[0], 6, 6), np.complex128)
    G6[:, :3, :3] = g
    G6[:, 3:, 3:] = g
    Gd = np.swapaxes(G6.conj(), -1, -2)
    return np.stack([G6 @ F[:, k] @ Gd for k in range(2)], axis=1)


def coords(L):
    V = int(np.prod(L))
    n = np.arange(V)
    c = []
    for m in range(4):
        c.append(n % L[m])
        n = n // L[m]
    return np.stack(c, axis=1)


def block_colour(L, B):
    c = coords(L)
    return ((c // np.array(B)).sum(axis=1) % 2).astype(np.int32)


def block_id(L, B):
    c = coords(L) // np.array(B)
    nb = [L[m] // B[m] for m in range(4)]
    return c[:, 0] + nb[0] * (c[:, 1] + nb[1] * (c[:, 2] + nb[2] * c[:, 3]))


def free_field_solve(L, kappa, b, bc=(1, 1, 1, 1)):
    """x = D^-1 b for U = 1, F = 1 in momentum space:
    D(p) = a + 2 i kappa sum_mu gamma_mu sin p_mu,  a = 1 - 2 kappa sum_mu cos p_mu,
    D(p)^-1 = (a - 2 i kappa sum_mu gamma_mu sin p_mu) / (a^2 + b^2),  b^2 = 4 kappa^2 sum sin^2 p.
    Antiperiodic directions are handled by the phase twist exp(i pi n_mu / L_mu)."""
    g = synth.gamma_matrices()
    Lx, Ly, Lz, Lt = L
    c = coords(L)
    twist = np.ones(len(c), np.complex128)
    for mu in range(4):
        if bc[mu] < 0:
            twist *= np.exp(1j * np.pi * c[:, mu] / L[mu])
    bt = (b * twist.conj()[:, None, None]).reshape(Lt, Lz, Ly, Lx, 4, 3)
    bh = np.fft.fftn(bt, axes=(0, 1, 2, 3))
    ps = [2 * np.pi * np.fft.fftfreq(L[mu]) + (np.pi / L[mu] if bc[mu] < 0 else 0.0) for mu in range(4)]
    pt, pz, py, px = np.meshgrid(ps[3], ps[2], ps[1], ps[0], indexing="ij")
    P = [px, py, pz, pt]
    a = 1 - 2 * kappa * sum(np.cos(p) for p in P)
    bb = 4 * kappa**2 * sum(np.sin(p) ** 2 for p in P)
    S = sum(np.sin(P[mu])[..., None, None] * g[mu] for mu in range(4))
    Minv = (a[..., None, None] * np.eye(4) - 2j * kappa * S) / (a**2 + bb)[..., None, None]
    xh = np.einsum("tzyxab,tzyxbc->tzyxac", Minv, bh)
    x = np.fft.ifftn(xh, axes=(0, 1, 2, 3)).reshape(-1, 4, 3)
    return x * twist[:, None, None]


def dense_operator(apply, V):
    """Dense [12V, 12V] matrix of a linear map on [V,4,3] spinors, column by column."""
    N = 12 * V
    M = np.zeros((N, N), np.complex128)
    for j in range(N):
        e = np.zeros(N, np.complex128)
        e[j] = 1
        M[:, j] = apply(e.reshape(V, 4, 3)).reshape(N)
    return M


def dense_block_diagonal(apply, L, B):
    """Dense matrices [NB, 12Vb, 12Vb] of a block-diagonal map, indexed by block-local
    lexicographic site index, probing the same local position in every block at once."""
    V = int(np.prod(L))
    Vb = int(np.prod(B))
    c = coords(L)
    loc = np.zeros(V, np.int64)
    mult = 1
    for m in range(4):
        loc += (c[:, m] % B[m]) * mult
        mult *= B[m]
    bid = block_id(L, B)
    NB = V // Vb
    M = np.zeros((NB, 12 * Vb, 12 * Vb), np.complex128)
    for l in range(Vb):
        for comp in range(12):
            e = np.zeros((V, 12), np.complex128)
            e[loc == l, comp] = 1
            out = apply(e.reshape(V, 4, 3)).reshape(V, 12)
            for r in range(12):
                M[bid, 12 * loc + r, 12 * l + comp] = out[:, r]
    return M, loc, bid
