"""FP64 CPU oracle for the SAP/SSOR clover-Wilson solver (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It is a plain, slow, obviously correct
implementation of what the GPU path computes, written from the paper
(Boku et al., arXiv:1210.7398) and sharing no code with the GPU library.

Every array is numpy complex128 in the interchange layout:
  spinor  [V, 4, 3]      site n = x + Lx*(y + Ly*(z + Lz*t)), spin, colour
  links   [V, 4, 3, 3]   U_mu(n)[a, b]
  clover  [V, 2, 6, 6]   two chiral 6x6 blocks, row 3*(alpha-2k)+a

Each wrapper names the passage of the paper its C routine follows.  The NN
routines (``nn_*``) follow the linear parallel-transport convolution stated in
nn_oracle.c; they have no passage in the paper.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

c_dc_p = ctypes.POINTER(ctypes.c_double)


class Params(ctypes.Structure):
    _fields_ = [
        ("kappa", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("tol_inner", ctypes.c_double),
        ("n_ssor", ctypes.c_int),
        ("n_sap", ctypes.c_int),
        ("maxit_inner", ctypes.c_int),
        ("maxit_outer", ctypes.c_int),
        ("outer_kind", ctypes.c_int),
        ("block_solver", ctypes.c_int),
    ]


def params(kappa, omega=1.0, n_ssor=4, n_sap=4, tol_inner=1e-2, maxit_inner=50, maxit_outer=200, outer_kind=0,
           block_solver=0):
    """block_solver 0: SSOR block inverses (section 3); 1: the even-odd minimal-residual
    block solve it is compared against (``eomr``)."""
    return Params(kappa, omega, tol_inner, n_ssor, n_sap, maxit_inner, maxit_outer, outer_kind, block_solver)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b

            _b.build()
        _LIB = ctypes.CDLL(path)
    return _LIB


def _geom(L, B=None, S=None, bc=(1, 1, 1, 1)):
    B = B if B is not None else L
    S = S if S is not None else B
    g = (ctypes.c_int * 16)(*(list(L) + list(B) + list(S) + list(bc)))
    return g


def _p(a):
    assert a.dtype == np.complex128 and a.flags.c_contiguous
    return a.ctypes.data_as(c_dc_p)


def _vol(L):
    return int(np.prod(L))


def gamma(mu):
    """gamma_mu (mu = 0..3) or gamma_5 (mu = 4) of the chiral basis, 4x4 complex."""
    out = np.zeros((4, 4), np.complex128)
    lib().orc_gamma(ctypes.c_int(mu), _p(out))
    return out


def plaquette(L, U):
    f = lib().orc_plaquette
    f.restype = ctypes.c_double
    return f(_geom(L), _p(U))


def clover_A(L, U, csw, kappa):
    """A(n) = 1 - c_SW kappa sum_{mu<nu} sigma_mu_nu F_mu_nu(n), full [V,12,12] (eq. 2.2's clover term)."""
    A = np.zeros((_vol(L), 12, 12), np.complex128)
    lib().orc_clover_A(_geom(L), _p(U), ctypes.c_double(csw), ctypes.c_double(kappa), _p(A))
    return A


def clover_inv(L, U, csw, kappa):
    """F(n) = A(n)^-1 as two chiral 6x6 blocks [V,2,6,6] (the inverse clover term of eq. 2.2)."""
    F = np.zeros((_vol(L), 2, 6, 6), np.complex128)
    bad = lib().orc_clover_inv(_geom(L), _p(U), ctypes.c_double(csw), ctypes.c_double(kappa), _p(F))
    if bad:
        raise ValueError("singular clover block")
    return F


def hop(L, U, psi, mode=0, B=None, bc=(1, 1, 1, 1)):
    """H psi, with mode 0 all pairs, 1 same-block pairs, 2 pairs in different blocks."""
    out = np.zeros_like(psi)
    lib().orc_hop(_geom(L, B, None, bc), _p(U), _p(psi), _p(out), ctypes.c_int(mode))
    return out


def apply_clover(L, F, psi):
    out = np.zeros_like(psi)
    lib().orc_apply_clover(_geom(L), _p(F), _p(psi), _p(out))
    return out


def dslash(L, U, F, kappa, psi, bc=(1, 1, 1, 1)):
    """D psi of eq. (2.2)."""
    out = np.zeros_like(psi)
    lib().orc_dslash(_geom(L, None, None, bc), _p(U), _p(F), ctypes.c_double(kappa), _p(psi), _p(out))
    return out


def dslash_part(L, B, U, F, kappa, psi, part, target_colour=-1, bc=(1, 1, 1, 1)):
    """Parts of D in the block form eq. (2.3): 0 full, 1 block-diagonal, 2 off-block."""
    out = np.zeros_like(psi)
    lib().orc_dslash_part(
        _geom(L, B, None, bc), _p(U), _p(F), ctypes.c_double(kappa), _p(psi), _p(out), ctypes.c_int(part),
        ctypes.c_int(target_colour),
    )
    return out


def site_colour(L, B):
    f = lib().orc_site_colour
    g = _geom(L, B)
    return np.array([f(g, ctypes.c_long(n)) for n in range(_vol(L))], np.int32)


def ll_order(B, S):
    """Block-local lexicographic site indices in locally-lexicographic order."""
    Vb = int(np.prod(B))
    out = np.zeros(Vb, np.int32)
    lib().orc_ll_order(_geom(B, B, S), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return out


def ssor(L, B, S, U, F, prm, colour, v, order=None, bc=(1, 1, 1, 1)):
    """x = A_cc v: n_ssor SSOR sweeps per block of colour `colour` (section 3)."""
    x = np.zeros_like(v)
    if order is not None:
        order = np.ascontiguousarray(order, np.int32)
        op = order.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    else:
        op = None
    lib().orc_ssor(_geom(L, B, S, bc), _p(U), _p(F), ctypes.byref(prm), ctypes.c_int(colour), op, _p(v), _p(x))
    return x


def eomr(L, B, U, F, prm, colour, v, bc=(1, 1, 1, 1)):
    """x = A_cc v by 2 n_ssor minimal-residual steps on the even-odd reduced system of every
    block of colour `colour` (the block solver section 3 measures the SSOR against)."""
    x = np.zeros_like(v)
    lib().orc_eomr(_geom(L, B, B, bc), _p(U), _p(F), ctypes.byref(prm), ctypes.c_int(colour), _p(v), _p(x))
    return x


def dk(L, B, S, U, F, prm, v, bc=(1, 1, 1, 1)):
    """(x, w) = (K v, D K v) by Algorithm 1."""
    x = np.zeros_like(v)
    w = np.zeros_like(v)
    lib().orc_dk(_geom(L, B, S, bc), _p(U), _p(F), ctypes.byref(prm), _p(v), _p(x), _p(w))
    return x, w


def msap(L, B, S, U, F, prm, v, bc=(1, 1, 1, 1)):
    """(y, dy) = (M_SAP v, D M_SAP v) of eq. (2.4)."""
    y = np.zeros_like(v)
    dy = np.zeros_like(v)
    lib().orc_msap(_geom(L, B, S, bc), _p(U), _p(F), ctypes.byref(prm), _p(v), _p(y), _p(dy))
    return y, dy


def inner_bicgstab(L, B, S, U, F, prm, r, bc=(1, 1, 1, 1)):
    """e ~ D^-1 r by M_SAP-preconditioned BiCGStab; returns (e, iterations)."""
    e = np.zeros_like(r)
    it = lib().orc_inner_bicgstab(_geom(L, B, S, bc), _p(U), _p(F), ctypes.byref(prm), _p(r), _p(e))
    return e, it


def solve(L, B, S, U, F, prm, b, tol=1e-10, x0=None, bc=(1, 1, 1, 1)):
    """Nested solve of D x = b (section 2); returns (x, stats dict, converged)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.complex128, copy=True)
    st = np.zeros(4, np.float64)
    rc = lib().orc_solve(
        _geom(L, B, S, bc), _p(U), _p(F), ctypes.byref(prm), ctypes.c_double(tol), _p(b), _p(x),
        ctypes.c_int(0 if x0 is None else 1), st.ctypes.data_as(c_dc_p),
    )
    stats = dict(outer=int(st[0]), inner=int(st[1]), relres=float(st[2]), restarts=int(st[3]))
    return x, stats, rc == 0


# ----------------------------------------------------------------------------- learned stage
# Three linear parallel-transport convolution layers, channels 1 -> 8 -> 8 -> 1.  Weight blob
# (the library's layout): float32, layer by layer, W[9][c_out][c_in][4][4] complex as (re, im).
NN_CHANNELS = 8
NN_SHAPES = [(1, NN_CHANNELS), (NN_CHANNELS, NN_CHANNELS), (NN_CHANNELS, 1)]  # (c_in, c_out)


def nn_param_count():
    return sum(2 * 16 * 9 * ci * co for ci, co in NN_SHAPES)


def nn_unflatten(w):
    """Flat float blob -> list of complex128 arrays W[9][c_out][c_in][4][4]."""
    w = np.asarray(w, np.float64)
    out, off = [], 0
    for ci, co in NN_SHAPES:
        n = 2 * 16 * 9 * ci * co
        a = w[off : off + n].reshape(9, co, ci, 4, 4, 2)
        out.append(np.ascontiguousarray(a[..., 0] + 1j * a[..., 1]))
        off += n
    return out


def nn_flatten(Ws):
    return np.concatenate([np.stack([W.real, W.imag], -1).reshape(-1) for W in Ws]).astype(np.float64)


def _gbc(L, bc):
    return _geom(L, None, None, bc)


def nn_layer(L, U, W, x, bc=(1, 1, 1, 1)):
    """out[c'] = sum_d sum_c W[d][c'][c] T_d x[c] for x [c_in, V, 4, 3]."""
    cout, cin = W.shape[1], W.shape[2]
    x = np.ascontiguousarray(x, np.complex128)
    out = np.zeros((cout,) + x.shape[1:], np.complex128)
    lib().orc_nn_layer(_gbc(L, bc), _p(U), _p(np.ascontiguousarray(W)), ctypes.c_int(cin), ctypes.c_int(cout),
                       _p(x), _p(out))
    return out


def nn_layer_adjoint(L, U, W, gout, bc=(1, 1, 1, 1)):
    cout, cin = W.shape[1], W.shape[2]
    gout = np.ascontiguousarray(gout, np.complex128)
    gin = np.zeros((cin,) + gout.shape[1:], np.complex128)
    lib().orc_nn_layer_adjoint(_gbc(L, bc), _p(U), _p(np.ascontiguousarray(W)), ctypes.c_int(cin), ctypes.c_int(cout),
                               _p(gout), _p(gin))
    return gin


def nn_layer_wgrad(L, U, cin, cout, gout, x, bc=(1, 1, 1, 1)):
    G = np.zeros((9, cout, cin, 4, 4), np.complex128)
    lib().orc_nn_layer_wgrad(_gbc(L, bc), _p(U), ctypes.c_int(cin), ctypes.c_int(cout),
                             _p(np.ascontiguousarray(gout, np.complex128)), _p(np.ascontiguousarray(x, np.complex128)),
                             _p(G))
    return G


def nn_forward(L, U, Ws, r, bc=(1, 1, 1, 1)):
    """z = N r for a spinor r [V, 4, 3]; returns (z, activations of every layer input)."""
    acts = [r[None]]
    for W in Ws:
        acts.append(nn_layer(L, U, W, acts[-1], bc))
    return acts[-1][0], acts[:-1]


def nn_backward(L, U, Ws, r, gz, bc=(1, 1, 1, 1)):
    """Weight gradients dL/dRe W + i dL/dIm W and N^+ gz for dL/dz = gz at z = N r, by the chain
    rule through the layers (each layer's input gradient is its adjoint applied to its output
    gradient)."""
    _, acts = nn_forward(L, U, Ws, r, bc)
    g = np.asarray(gz, np.complex128)[None]
    grads = [None] * len(Ws)
    for k in range(len(Ws) - 1, -1, -1):
        W = Ws[k]
        grads[k] = nn_layer_wgrad(L, U, W.shape[2], W.shape[1], g, acts[k], bc)
        g = nn_layer_adjoint(L, U, W, g, bc)
    return grads, g[0]


def nn_loss_grad(L, U, Ws, r, e, bc=(1, 1, 1, 1)):
    """loss = |N r - e|^2 / |e|^2 and its gradients dL/dRe W + i dL/dIm W."""
    z, _ = nn_forward(L, U, Ws, r, bc)
    ee = float(np.vdot(e, e).real)
    loss = float(np.vdot(z - e, z - e).real) / ee
    grads, _ = nn_backward(L, U, Ws, r, (2.0 / ee) * (z - e), bc)
    return loss, grads


def adam_step(p, grad, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of real arrays, in place; t counts from 1."""
    m *= b1
    m += (1 - b1) * grad
    v *= b2
    v += (1 - b2) * grad * grad
    mh = m / (1 - b1**t)
    vh = v / (1 - b2**t)
    p -= lr * mh / (np.sqrt(vh) + eps)
    return p
