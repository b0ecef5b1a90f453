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
routines (``nn_*``) follow the linear parallel-transport convolution defined
in the design doc; they have no passage in the paper.
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
    ]


def params(kappa, omega=1.0, n_ssor=4, n_sap=4, tol_inner=1e-2, maxit_inner=50, maxit_outer=200, outer_kind=0):
    return Params(kappa, omega, tol_inner, n_ssor, n_sap, maxit_inner, maxit_outer, outer_kind)


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
