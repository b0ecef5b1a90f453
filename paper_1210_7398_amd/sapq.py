"""Thin ctypes binding of libsapq (include/sapq.h).

Argument marshalling only: tensors are checked (device, dtype, contiguity) and
their data pointers, with torch's current HIP stream, are handed to the C ABI.
Every step of the solver runs in the library's HIP kernels; there is no
fallback, and a missing library raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsapq.so")
_LIB = None

FP64, FP32, FP16, BF16 = 0, 1, 2, 3
OUTER_FBICGSTAB, OUTER_DEFECT = 0, 1
FLAG_GUESS, FLAG_PROFILE, FLAG_NN, FLAG_NN_FP32, FLAG_EOMR, FLAG_FALLBACK_FP32 = 1, 2, 4, 8, 16, 32
FALLBACK_NN, FALLBACK_FP32 = 1, 2
PREC = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16}
STATUS = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "ENOTSU3", -4: "ENOTCONV", -5: "EBREAKDOWN", -6: "EHIP",
          -7: "ENOMEM", -8: "ESTATE"}


class SapqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sapq {STATUS.get(code, code)}: {msg}")
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4), ("block", ctypes.c_int * 4), ("subblock", ctypes.c_int * 4),
                ("bc_sign", ctypes.c_int * 4)]


class Params(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("omega", ctypes.c_double), ("tol_inner", ctypes.c_double),
                ("n_ssor", ctypes.c_int), ("n_sap", ctypes.c_int), ("maxit_inner", ctypes.c_int),
                ("maxit_outer", ctypes.c_int), ("prec_inner", ctypes.c_int), ("outer", ctypes.c_int),
                ("flags", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("outer_its", ctypes.c_int), ("inner_its", ctypes.c_int), ("n_msap", ctypes.c_int),
                ("n_dslash64", ctypes.c_int), ("restarts", ctypes.c_int), ("n_hist", ctypes.c_int),
                ("true_relres", ctypes.c_double), ("time_s", ctypes.c_double), ("kern_ms", ctypes.c_double * 8),
                ("kern_n", ctypes.c_int * 8), ("relres_hist", ctypes.c_double * 256), ("breakdowns", ctypes.c_int),
                ("fallback", ctypes.c_int)]

    KINDS = ("phase_E", "phase_O", "face", "dslash64", "blas")

    def as_dict(self):
        return dict(outer_its=self.outer_its, inner_its=self.inner_its, n_msap=self.n_msap,
                    n_dslash64=self.n_dslash64, restarts=self.restarts, true_relres=self.true_relres,
                    time_s=self.time_s, relres_hist=list(self.relres_hist[: self.n_hist]),
                    breakdowns=self.breakdowns, fallback=self.fallback,
                    kernels={k: dict(ms=self.kern_ms[i], n=self.kern_n[i]) for i, k in enumerate(self.KINDS)
                             if self.kern_n[i]})


_P = ctypes.c_void_p
_SIGS = {
    "sapq_arena_bytes": (ctypes.c_size_t, [ctypes.POINTER(Geom), ctypes.POINTER(Params)]),
    "sapq_create": (ctypes.c_int, [ctypes.POINTER(Geom), ctypes.POINTER(Params), _P, ctypes.c_size_t, _P,
                                   ctypes.POINTER(_P)]),
    "sapq_set_params": (ctypes.c_int, [_P, ctypes.POINTER(Params)]),
    "sapq_load_gauge": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "sapq_load_clover_inv": (ctypes.c_int, [_P, _P]),
    "sapq_dslash": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "sapq_dslash_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "sapq_time_dslash": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "sapq_ssor": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "sapq_dk": (ctypes.c_int, [_P, _P, _P, _P]),
    "sapq_sap_precondition": (ctypes.c_int, [_P, _P, _P, _P]),
    "sapq_precondition": (ctypes.c_int, [_P, _P, _P, _P]),
    "sapq_inner_solve": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(ctypes.c_int)]),
    "sapq_solve": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.POINTER(Stats)]),
    "sapq_nn_param_count": (ctypes.c_size_t, []),
    "sapq_nn_set_weights": (ctypes.c_int, [_P, _P]),
    "sapq_nn_get_weights": (ctypes.c_int, [_P, _P]),
    "sapq_nn_copy_state": (ctypes.c_int, [_P, _P]),
    "sapq_nn_adam_step": (ctypes.c_int, [_P, _P, ctypes.c_float, ctypes.c_int]),
    "sapq_defect_errors": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int]),
    "sapq_nn_forward": (ctypes.c_int, [_P, _P, _P]),
    "sapq_nn_backward": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "sapq_nn_train_step": (ctypes.c_int, [_P, _P, ctypes.c_long, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                          ctypes.c_float, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "sapq_batch_arena_bytes": (ctypes.c_size_t, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "sapq_solve_batch": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_P),
                                        ctypes.POINTER(_P), ctypes.c_double, _P, ctypes.c_size_t, ctypes.POINTER(Stats)]),
    "sapq_autotune": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]),
    "sapq_autotune_batch": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_double, _P, ctypes.c_size_t,
                                           ctypes.c_char_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "sapq_phase_kernel": (ctypes.c_int, [_P]),
    "sapq_destroy": (None, [_P]),
    "sapq_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Open libsapq.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _check(code):
    if code != 0:
        raise SapqError(code, lib().sapq_last_error().decode())


def _ptr(t, V=None, shape_tail=None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a torch tensor on a GPU device")
    if t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError("expected a contiguous complex128 tensor")
    if V is not None and (t.shape[0] != V or tuple(t.shape[1:]) != shape_tail):
        raise ValueError(f"expected shape {(V,) + shape_tail}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One lattice + parameter set (one sapq context) with its own device arena."""

    def __init__(self, L, block, subblock, kappa, bc=(1, 1, 1, 1), omega=1.0, n_ssor=4, n_sap=4, tol_inner=0.1,
                 maxit_inner=50, maxit_outer=100, prec="fp32", outer="fbicgstab", device=None, nn=False,
                 nn_fp32=False, block_solver="ssor", fallback_fp32=False):
        self.L = tuple(L)
        self.V = int(L[0] * L[1] * L[2] * L[3])
        self.geom = Geom((ctypes.c_int * 4)(*L), (ctypes.c_int * 4)(*block), (ctypes.c_int * 4)(*subblock),
                         (ctypes.c_int * 4)(*bc))
        if block_solver not in ("ssor", "eomr"):
            raise ValueError("block_solver must be 'ssor' or 'eomr'")
        self.base_flags = ((FLAG_NN if nn else 0) | (FLAG_NN_FP32 if nn_fp32 else 0) |
                           (FLAG_EOMR if block_solver == "eomr" else 0) | (FLAG_FALLBACK_FP32 if fallback_fp32 else 0))
        self.params = Params(kappa, omega, tol_inner, n_ssor, n_sap, maxit_inner, maxit_outer, PREC[prec],
                             OUTER_FBICGSTAB if outer == "fbicgstab" else OUTER_DEFECT, self.base_flags)
        self.prec = prec
        n = lib().sapq_arena_bytes(ctypes.byref(self.geom), ctypes.byref(self.params))
        if n == 0:
            # reproduce the validation error message
            h = _P()
            dummy = torch.empty(256, dtype=torch.uint8, device=device or "cuda")
            _check(lib().sapq_create(ctypes.byref(self.geom), ctypes.byref(self.params),
                                     ctypes.c_void_p(dummy.data_ptr()), 256, None, ctypes.byref(h)))
        self.device = torch.device(device or "cuda")
        self.arena = torch.empty(n, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = _P()
        _check(lib().sapq_create(ctypes.byref(self.geom), ctypes.byref(self.params),
                                 ctypes.c_void_p(self.arena.data_ptr()), n, ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().sapq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **kw):
        for k, v in kw.items():
            if k == "outer":
                v = OUTER_FBICGSTAB if v == "fbicgstab" else OUTER_DEFECT
            setattr(self.params, k, v)
        _check(lib().sapq_set_params(self.h, ctypes.byref(self.params)))

    def _spinor(self):
        return torch.empty((self.V, 4, 3), dtype=torch.complex128, device=self.device)

    def load_gauge(self, U):
        dev = ctypes.c_double(0)
        _check(lib().sapq_load_gauge(self.h, _ptr(U, self.V, (4, 3, 3)), ctypes.byref(dev)))
        return dev.value

    def load_clover(self, F):
        _check(lib().sapq_load_clover_inv(self.h, _ptr(F, self.V, (2, 6, 6))))

    def dslash(self, psi, prec="fp64"):
        out = self._spinor()
        _check(lib().sapq_dslash(self.h, _ptr(out), _ptr(psi, self.V, (4, 3)), PREC[prec]))
        return out

    def time_dslash(self, psi, prec="fp64", reps=20):
        """Mean microseconds of one operator kernel launch (sapq_time_dslash)."""
        us = ctypes.c_double(0)
        _check(lib().sapq_time_dslash(self.h, _ptr(psi, self.V, (4, 3)), PREC[prec], int(reps), ctypes.byref(us)))
        return us.value

    def dslash_noalloc(self, psi, out, prec="fp64"):
        """out = D psi through the allocation-free entry point (sapq_dslash_noalloc); out is the
        caller's tensor, so the call allocates nothing."""
        _check(lib().sapq_dslash_noalloc(self.h, _ptr(out, self.V, (4, 3)), _ptr(psi, self.V, (4, 3)), PREC[prec]))
        return out

    def ssor(self, v, colour):
        x = self._spinor()
        _check(lib().sapq_ssor(self.h, _ptr(x), _ptr(v, self.V, (4, 3)), colour))
        return x

    def dk(self, v):
        x, w = self._spinor(), self._spinor()
        _check(lib().sapq_dk(self.h, _ptr(x), _ptr(w), _ptr(v, self.V, (4, 3))))
        return x, w

    def sap_precondition(self, v, with_d=True):
        y = self._spinor()
        dy = self._spinor() if with_d else None
        _check(lib().sapq_sap_precondition(self.h, _ptr(y), _ptr(dy) if with_d else None, _ptr(v, self.V, (4, 3))))
        return (y, dy) if with_d else y

    def precondition(self, v):
        """(P v, D P v) for the inner solver's preconditioner P (sapq_precondition): M_SAP, or
        N + M_SAP (1 - D N) with the learned stage on."""
        y, dy = self._spinor(), self._spinor()
        _check(lib().sapq_precondition(self.h, _ptr(y), _ptr(dy), _ptr(v, self.V, (4, 3))))
        return y, dy

    def defect_errors(self, b, xstar, n_iter):
        """Errors e_k = xstar - x_k of the plain solver's defect-correction iterates from x_0 = 0
        (sapq_defect_errors): float32 tensor [n_iter, V, 4, 3, 2]."""
        e = torch.empty((n_iter, self.V, 4, 3, 2), dtype=torch.float32, device=self.device)
        _check(lib().sapq_defect_errors(self.h, ctypes.c_void_p(e.data_ptr()), _ptr(b, self.V, (4, 3)),
                                        _ptr(xstar, self.V, (4, 3)), int(n_iter)))
        return e

    def inner_solve(self, r):
        e = self._spinor()
        it = ctypes.c_int(0)
        _check(lib().sapq_inner_solve(self.h, _ptr(e), _ptr(r, self.V, (4, 3)), ctypes.byref(it)))
        return e, it.value

    def solve(self, b, tol=1e-10, x0=None, check=True, profile=False):
        x = self._spinor() if x0 is None else x0.clone()
        self.params.flags = self.base_flags | (0 if x0 is None else FLAG_GUESS) | (FLAG_PROFILE if profile else 0)
        _check(lib().sapq_set_params(self.h, ctypes.byref(self.params)))
        st = Stats()
        rc = lib().sapq_solve(self.h, _ptr(x), _ptr(b, self.V, (4, 3)), tol, ctypes.byref(st))
        if check:
            _check(rc)
        return x, st.as_dict()

    @property
    def phase_kernel(self):
        """Name of the SAP phase kernel this context runs (sapq_phase_kernel)."""
        return {0: "four-lane", 1: "two-lane", 2: "two-lane split"}[lib().sapq_phase_kernel(self.h)]

    def autotune(self, cache_path=None):
        """Pick the fastest sub-block shape (sapq_autotune); returns it."""
        out = (ctypes.c_int * 4)()
        _check(lib().sapq_autotune(self.h, cache_path.encode() if cache_path else None, out))
        return tuple(out)

    # ------------------------------------------------------------------ learned stage
    def use_nn(self, on=True):
        """Switch the learned stage of the inner preconditioner on or off (needs nn=True at creation)."""
        self.base_flags = (self.base_flags | FLAG_NN) if on else (self.base_flags & ~FLAG_NN)
        self.params.flags = self.base_flags
        _check(lib().sapq_set_params(self.h, ctypes.byref(self.params)))

    def nn_set_weights(self, w):
        if w.dtype != torch.float32 or not w.is_contiguous() or w.numel() != nn_param_count() or w.device.type != "cuda":
            raise TypeError("expected a contiguous float32 GPU tensor with nn_param_count() entries")
        _check(lib().sapq_nn_set_weights(self.h, ctypes.c_void_p(w.data_ptr())))

    def nn_get_weights(self):
        w = torch.empty(nn_param_count(), dtype=torch.float32, device=self.device)
        _check(lib().sapq_nn_get_weights(self.h, ctypes.c_void_p(w.data_ptr())))
        return w

    def nn_copy_state_from(self, other):
        """Take over other's training state (weights and Adam moments; sapq_nn_copy_state)."""
        _check(lib().sapq_nn_copy_state(self.h, other.h))

    def nn_forward(self, psi):
        out = self._spinor()
        _check(lib().sapq_nn_forward(self.h, _ptr(out), _ptr(psi, self.V, (4, 3))))
        return out

    def nn_backward(self, grad_out, inp):
        gw = torch.empty(nn_param_count(), dtype=torch.float32, device=self.device)
        gin = self._spinor()
        _check(lib().sapq_nn_backward(self.h, ctypes.c_void_p(gw.data_ptr()), _ptr(gin), _ptr(grad_out, self.V, (4, 3)),
                                      _ptr(inp, self.V, (4, 3))))
        return gw, gin

    def nn_adam_step(self, grad_w, lr, t):
        """One Adam step of the weights with a caller-supplied gradient (sapq_nn_adam_step)."""
        if (grad_w.dtype != torch.float32 or not grad_w.is_contiguous() or grad_w.numel() != nn_param_count()
                or grad_w.device.type != "cuda"):
            raise TypeError("expected a contiguous float32 GPU tensor with nn_param_count() entries")
        _check(lib().sapq_nn_adam_step(self.h, ctypes.c_void_p(grad_w.data_ptr()), float(lr), int(t)))

    def nn_train_step(self, e, idx, lr, t):
        """e: float32 GPU tensor [n, V, 4, 3, 2] of error vectors; idx: batch indices."""
        if e.dtype != torch.float32 or not e.is_contiguous() or tuple(e.shape[1:]) != (self.V, 4, 3, 2):
            raise TypeError("expected a contiguous float32 tensor [n, V, 4, 3, 2]")
        ib = (ctypes.c_int * len(idx))(*[int(i) for i in idx])
        loss = ctypes.c_double(0)
        _check(lib().sapq_nn_train_step(self.h, ctypes.c_void_p(e.data_ptr()), e.shape[0], ib, len(idx), lr, t,
                                        ctypes.byref(loss)))
        return loss.value


# Work memory of solve_batch, kept per device between calls and grown when a call needs
# more: a fresh multi-GB allocation per call (after the caching allocator has returned its
# memory) can be mapped in a way that slows every kernel of the solve, and the batched
# solver does not need the arena cleared.  release_batch_arena() hands it back.
_BATCH_ARENA = {}


def _batch_arena(device, nbytes):
    a = _BATCH_ARENA.get(device)
    if a is not None and a.numel() >= nbytes:
        return a
    del a
    _BATCH_ARENA.pop(device, None)  # the old one is freed before the larger one is taken
    a = torch.empty(nbytes, dtype=torch.uint8, device=device)
    _BATCH_ARENA[device] = a
    return a


def release_batch_arena():
    """Drop the work memory that solve_batch keeps between calls."""
    _BATCH_ARENA.clear()


def solve_batch(solvers, sources, tol=1e-10, check=True):
    """Solve every source of every solver's field together (sapq_solve_batch).  sources[i]:
    complex128 GPU tensor [nrhs_i, V_i, 4, 3].  Returns (solutions, per-source stats dicts).
    The work memory stays allocated for the next call (release_batch_arena frees it)."""
    n = len(solvers)
    ctxs = (_P * n)(*[s.h for s in solvers])
    nrhs = (ctypes.c_int * n)(*[int(b.shape[0]) for b in sources])
    for s, b in zip(solvers, sources):
        if b.dtype != torch.complex128 or not b.is_contiguous() or tuple(b.shape[1:]) != (s.V, 4, 3):
            raise TypeError("expected contiguous complex128 sources [nrhs, V, 4, 3]")
    xs = [torch.empty_like(b) for b in sources]
    xp = (_P * n)(*[x.data_ptr() for x in xs])
    bp = (_P * n)(*[b.data_ptr() for b in sources])
    nbytes = lib().sapq_batch_arena_bytes(ctxs, n, nrhs)
    if nbytes == 0:
        raise SapqError(-1, "batch not allowed (shapes, precisions or block size)")
    arena = _batch_arena(solvers[0].device, nbytes)
    total = sum(int(b.shape[0]) for b in sources)
    st = (Stats * total)()
    rc = lib().sapq_solve_batch(ctxs, n, nrhs, xp, bp, tol, ctypes.c_void_p(arena.data_ptr()), nbytes, st)
    if check:
        _check(rc)
    return xs, [st[i].as_dict() for i in range(total)]


def autotune_batch(solvers, sources, tol=1e-10, cache_path=None):
    """Choose the batched solver's sources per workgroup and inner iterations per graph replay
    for this batch (sapq_autotune_batch); returns (nr, k_inner)."""
    n = len(solvers)
    ctxs = (_P * n)(*[s.h for s in solvers])
    nrhs = (ctypes.c_int * n)(*[int(b.shape[0]) for b in sources])
    for s, b in zip(solvers, sources):
        if b.dtype != torch.complex128 or not b.is_contiguous() or tuple(b.shape[1:]) != (s.V, 4, 3):
            raise TypeError("expected contiguous complex128 sources [nrhs, V, 4, 3]")
    xs = [torch.empty_like(b) for b in sources]
    xp = (_P * n)(*[x.data_ptr() for x in xs])
    bp = (_P * n)(*[b.data_ptr() for b in sources])
    nbytes = lib().sapq_batch_arena_bytes(ctxs, n, nrhs)
    if nbytes == 0:
        raise SapqError(-1, "batch not allowed (shapes, precisions or block size)")
    arena = _batch_arena(solvers[0].device, nbytes)
    nr, k = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().sapq_autotune_batch(ctxs, n, nrhs, xp, bp, tol, ctypes.c_void_p(arena.data_ptr()), nbytes,
                                     cache_path.encode() if cache_path else None, ctypes.byref(nr), ctypes.byref(k)))
    return nr.value, k.value


def nn_param_count():
    return int(lib().sapq_nn_param_count())
