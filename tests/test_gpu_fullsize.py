"""Parity at the full sizes bench.py runs, in its launch configuration.

- 24^3x48 with 6^3x12 blocks and 3^3x6 sub-blocks: the bench's default workload, fields and
  source; the phase kernel is the two-workgroup split.
- 32^3x64 with 4^4 blocks and FP16 / BF16 storage: the precision workload, with FP64 defect
  correction.

Every check is against the FP64 oracle on the host:
- SSOR and M_SAP of a whole field, to the FP32 chain tolerance of test_gpu_parity (2e-5);
- the true residual ||b - D x|| / ||b|| <= 1e-10 of full solves, with the oracle's D."""
import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests.gpu_common import check_close, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

# the bench workloads of the same names
C2 = dict(L=(24, 24, 24, 48), B=(6, 6, 6, 12), S=(3, 3, 3, 6), kappa=0.125, eps=0.25, seed=2, seed_b=1002)
C3 = dict(L=(32, 32, 32, 64), B=(4, 4, 4, 4), S=(2, 2, 2, 2), kappa=0.125, eps=0.25, seed=3, seed_b=1003)


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def c2(torch_cuda):
    U = synth.gauge_field(C2["L"], C2["eps"], C2["seed"])
    F = synth.clover_inverse(C2["L"], U, 1.0, C2["kappa"])
    return U, F


@pytest.fixture(scope="module")
def c3(torch_cuda):
    dev = torch_cuda.device("cuda:0")
    Ud = synth.gauge_field(C3["L"], C3["eps"], C3["seed"], device=dev)
    Fd = synth.clover_inverse(C3["L"], Ud, 1.0, C3["kappa"], device=dev)
    return Ud, Fd, Ud.cpu().numpy(), Fd.cpu().numpy()


def _solver(w, U_dev, F_dev, **kw):
    from paper_1210_7398_amd import sapq

    s = sapq.Solver(w["L"], w["B"], w["S"], w["kappa"], **kw)
    assert s.load_gauge(U_dev) < 1e-12
    s.load_clover(F_dev)
    return s


def test_c2_ssor_and_msap_whole_field(c2, orc):
    U, F = c2
    w = C2
    s = _solver(w, to_dev(U), to_dev(F))
    assert s.phase_kernel == "two-lane split"
    v = synth.gaussian_spinor(w["L"], 131)
    prm = orc.params(w["kappa"])
    for colour in (0, 1):
        want = orc.ssor(w["L"], w["B"], w["S"], U, F, prm, colour, v)
        check_close(to_host(s.ssor(to_dev(v), colour)), want, 2e-5, f"full-size SSOR colour {colour}")
    y_w, dy_w = orc.msap(w["L"], w["B"], w["S"], U, F, prm, v)
    y, dy = (to_host(t) for t in s.sap_precondition(to_dev(v)))
    check_close(y, y_w, 2e-5, "full-size M_SAP")
    check_close(dy, dy_w, 2e-5, "full-size D M_SAP")


def test_c2_solve_true_residual(c2, orc):
    U, F = c2
    w = C2
    s = _solver(w, to_dev(U), to_dev(F))
    b = synth.gaussian_spinor(w["L"], w["seed_b"])
    x, st = s.solve(to_dev(b), tol=1e-10)
    rr = relerr(orc.dslash(w["L"], U, F, w["kappa"], to_host(x)), b)
    assert rr <= 1e-10, (rr, st)
    assert st["true_relres"] <= 1e-10


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_c3_low_precision_solve_true_residual(c3, orc, prec):
    Ud, Fd, U, F = c3
    w = C3
    s = _solver(w, Ud, Fd, prec=prec, outer="defect", maxit_outer=400)
    assert s.phase_kernel == "two-lane"
    b = synth.gaussian_spinor(w["L"], w["seed_b"])
    x, st = s.solve(to_dev(b), tol=1e-10)
    rr = relerr(orc.dslash(w["L"], U, F, w["kappa"], to_host(x)), b)
    assert rr <= 1e-10, (rr, st)
