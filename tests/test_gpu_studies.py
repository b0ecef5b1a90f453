"""GPU parity of every configuration a study or the autotuner runs, against the FP64 oracle.

The studies (bench.py --mode blocks / omega / sustained / batch) compare block solvers, block
and sub-block shapes and SSOR relaxations by time and M_SAP count.  The outer iteration checks
its true residual, so a wrong preconditioner would still converge and only its M_SAP count
would change: each configuration's block inverse and M_SAP are therefore compared with the
oracle here, on small lattices with the study's block shapes, in the phase kernel the study
runs them with (section 3, "Inverse of block operator"):
- natural-order SSOR (sub-block = block) at 4^4, 6^4 and 6^3x12 blocks;
- 6^3x12 blocks with 3^4 and 2^3x4 sub-blocks, 6^4 blocks with 2^4 sub-blocks;
- every sub-block shape the autotuner tries on 4^4 blocks;
- SSOR relaxation omega = 1.2 and 1.3 with 1 and 4 sweeps on all three phase kernels, a solve
  and a batched solve at omega = 1.3;
- the two-workgroup split kernel with more workgroups than the chip holds at once (24^3x96
  with 6^3x12 blocks: 512 workgroups per launch).
Tolerances are the FP32 chain tolerance of test_gpu_parity (2e-5), with the per-site check."""
import itertools

import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests.gpu_common import check_close, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

KERNELS = {"four-lane": "0", "two-lane": "1", "two-lane split": "2"}

# name: (lattice, block, sub-block, kappa, eps, phase kernel the library picks)
STUDY = {
    "12^3x24/6^3x12/natural": ((12, 12, 12, 24), (6, 6, 6, 12), (6, 6, 6, 12), 0.125, 0.25, "four-lane"),
    "12^3x24/6^3x12/3^4": ((12, 12, 12, 24), (6, 6, 6, 12), (3, 3, 3, 3), 0.125, 0.25, "two-lane split"),
    "12^3x24/6^3x12/2^3x4": ((12, 12, 12, 24), (6, 6, 6, 12), (2, 2, 2, 4), 0.125, 0.25, "four-lane"),
    "12^4/6^4/2^4": ((12, 12, 12, 12), (6, 6, 6, 6), (2, 2, 2, 2), 0.125, 0.25, "two-lane"),
    "12^4/6^4/natural": ((12, 12, 12, 12), (6, 6, 6, 6), (6, 6, 6, 6), 0.125, 0.25, "two-lane"),
    "8^4/4^4/natural": ((8, 8, 8, 8), (4, 4, 4, 4), (4, 4, 4, 4), 0.120, 0.25, "two-lane"),
}


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


_FIELDS = {}


def _fields(L, eps, kappa, seed=7):
    key = (L, eps, kappa, seed)
    if key not in _FIELDS:
        U = synth.gauge_field(L, eps, seed)
        _FIELDS[key] = (U, synth.clover_inverse(L, U, 1.0, kappa))
    return _FIELDS[key]


def _solver(L, B, S, kappa, U, F, **kw):
    from paper_1210_7398_amd import sapq

    s = sapq.Solver(L, B, S, kappa, **kw)
    assert s.load_gauge(to_dev(U)) < 1e-12
    s.load_clover(to_dev(F))
    return s


def _check_ssor_msap(orc, s, L, B, S, kappa, U, F, what, n_sap=2, omega=1.0, n_ssor=4, seed=301):
    v = synth.gaussian_spinor(L, seed)
    prm = orc.params(kappa, n_sap=n_sap, omega=omega, n_ssor=n_ssor)
    for colour in (0, 1):
        want = orc.ssor(L, B, S, U, F, prm, colour, v)
        check_close(to_host(s.ssor(to_dev(v), colour)), want, 2e-5, f"{what} SSOR colour {colour}")
    y_w, dy_w = orc.msap(L, B, S, U, F, prm, v)
    for k in range(2):  # twice: the split kernel's tickets and epochs carry over
        y, dy = (to_host(t) for t in s.sap_precondition(to_dev(v)))
        check_close(y, y_w, 2e-5, f"{what} M_SAP ({k})")
        check_close(dy, dy_w, 2e-5, f"{what} D M_SAP ({k})")


@pytest.mark.parametrize("name", list(STUDY))
def test_block_study_shapes(torch_cuda, orc, name):
    """The block study's shapes that no other test covers, in the phase kernel the study uses,
    and a solve to 1e-10 with the oracle's solution to 1e-8."""
    L, B, S, kappa, eps, kernel = STUDY[name]
    U, F = _fields(L, eps, kappa)
    s = _solver(L, B, S, kappa, U, F, n_sap=2)
    assert s.phase_kernel == kernel, (name, s.phase_kernel)
    _check_ssor_msap(orc, s, L, B, S, kappa, U, F, name)
    s.set_params(n_sap=4)
    b = synth.gaussian_spinor(L, 302)
    x, st = s.solve(to_dev(b), tol=1e-10)
    x = to_host(x)
    assert relerr(orc.dslash(L, U, F, kappa, x), b) <= 1e-10, st
    xo, _, ok = orc.solve(L, B, S, U, F, orc.params(kappa), b, tol=1e-12)
    assert ok
    check_close(x, xo, 1e-8, f"{name} solution")
    s.close()


# every sub-block shape sapq_autotune times on 4^4 blocks (extents 2 or 4), and the even-odd order
AUTOTUNE_SHAPES = [S for S in itertools.product((2, 4), repeat=4)] + [(0, 0, 0, 0)]


@pytest.mark.parametrize("S", AUTOTUNE_SHAPES, ids=lambda S: "x".join(map(str, S)))
def test_autotuner_candidates(torch_cuda, orc, S):
    L, B, kappa, eps = (8, 8, 8, 8), (4, 4, 4, 4), 0.125, 0.25
    U, F = _fields(L, eps, kappa)
    s = _solver(L, B, S, kappa, U, F, n_sap=1)
    v = synth.gaussian_spinor(L, 303)
    y_w, dy_w = orc.msap(L, B, S, U, F, orc.params(kappa, n_sap=1), v)
    y, dy = (to_host(t) for t in s.sap_precondition(to_dev(v)))
    check_close(y, y_w, 2e-5, f"sub-block {S} M_SAP")
    check_close(dy, dy_w, 2e-5, f"sub-block {S} D M_SAP")
    s.close()


# omega != 1: the (1 - omega) x term of every phase kernel
OMEGA_CASES = {
    "two-lane": ((8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), 0.120),
    "two-lane split": ((12, 12, 12, 24), (6, 6, 6, 12), (3, 3, 3, 6), 0.125),
    "four-lane": ((8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), 0.120),
}


@pytest.mark.parametrize("kernel", list(OMEGA_CASES))
@pytest.mark.parametrize("omega", [1.2, 1.3])
@pytest.mark.parametrize("n_ssor", [1, 4])
def test_ssor_relaxation(torch_cuda, orc, monkeypatch, kernel, omega, n_ssor):
    L, B, S, kappa = OMEGA_CASES[kernel]
    U, F = _fields(L, 0.25, kappa)
    monkeypatch.setenv("SAPQ_PARTS", KERNELS[kernel])
    s = _solver(L, B, S, kappa, U, F, n_sap=2, omega=omega, n_ssor=n_ssor)
    monkeypatch.delenv("SAPQ_PARTS")
    assert s.phase_kernel == kernel
    _check_ssor_msap(orc, s, L, B, S, kappa, U, F, f"{kernel} omega {omega} n_ssor {n_ssor}", omega=omega,
                     n_ssor=n_ssor, seed=304)
    s.close()


def test_relaxed_solve_and_batched_solve(torch_cuda, orc):
    """omega = 1.3 in a full solve (oracle solution to 1e-8) and in the batched solver, whose
    sources must match the one-source solves."""
    from paper_1210_7398_amd import sapq

    L, B, S, kappa = (8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), 0.125
    U, F = _fields(L, 0.25, kappa, seed=9)
    s = _solver(L, B, S, kappa, U, F, omega=1.3, outer="defect")
    b = np.stack([synth.gaussian_spinor(L, 305 + k) for k in range(3)])
    x1, st = s.solve(to_dev(np.ascontiguousarray(b[0])), tol=1e-10)
    x1 = to_host(x1)
    assert relerr(orc.dslash(L, U, F, kappa, x1), b[0]) <= 1e-10, st
    xo, _, ok = orc.solve(L, B, S, U, F, orc.params(kappa, omega=1.3), b[0], tol=1e-12)
    assert ok
    check_close(x1, xo, 1e-8, "omega 1.3 solution")
    xs, stats = sapq.solve_batch([s], [to_dev(b)], tol=1e-10)
    xs = to_host(xs[0])
    for k in range(b.shape[0]):
        assert relerr(orc.dslash(L, U, F, kappa, xs[k]), b[k]) <= 1e-10, stats[k]
        xk, _ = s.solve(to_dev(np.ascontiguousarray(b[k])), tol=1e-10)
        check_close(xs[k], to_host(xk), 1e-8, f"omega 1.3 batched source {k}")
    s.close()


def test_split_kernel_oversubscribed(torch_cuda, orc):
    """24^3x96 with 6^3x12 blocks: 256 blocks per colour, 512 workgroups per phase launch, twice
    what the chip holds at once (one per CU, by LDS).  The ticket order must pair the halves
    of every block whatever the start order; SSOR and M_SAP (twice) against the oracle."""
    torch = torch_cuda
    L, B, S, kappa = (24, 24, 24, 96), (6, 6, 6, 12), (3, 3, 3, 6), 0.125
    dev = torch.device("cuda:0")
    Ud = synth.gauge_field(L, 0.25, 51, device=dev)
    Fd = synth.clover_inverse(L, Ud, 1.0, kappa, device=dev)
    U, F = Ud.cpu().numpy(), Fd.cpu().numpy()
    from paper_1210_7398_amd import sapq

    s = sapq.Solver(L, B, S, kappa, n_sap=1)
    assert s.load_gauge(Ud) < 1e-12
    s.load_clover(Fd)
    del Ud, Fd
    assert s.phase_kernel == "two-lane split"
    _check_ssor_msap(orc, s, L, B, S, kappa, U, F, "24^3x96 split", n_sap=1, seed=306)
    s.close()
