"""GPU parity of the even-odd site-preconditioned block solve (the block solver section 3
measures the ll-ordered SSOR against), through the C ABI, against the FP64 oracle.

Tolerances as for the SSOR chains: 2e-5 relative (FP32 arithmetic, the minimal-residual
coefficients summed in FP64), the FP16 storage tolerances of the parity tests, and the FP64
true residual of a full solve."""
import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests.gpu_common import check_close, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

# name: (lattice, block, kappa, eps, bc); the sites of one parity per lane pair (the kernel's
# register tiling) are 1 for the 4^4, 4x2x2x4 and 2^4 blocks (most pairs idle in the 2^4
# blocks) and 3 for the 6^4 blocks
GEOMS = {
    "8^4/4^4": ((8, 8, 8, 8), (4, 4, 4, 4), 0.120, 0.25, (1, 1, 1, 1)),
    "12^4/6^4 antiperiodic": ((12, 12, 12, 12), (6, 6, 6, 6), 0.125, 0.25, (1, 1, 1, -1)),
    "8x4x4x8/4x2x2x4": ((8, 4, 4, 8), (4, 2, 2, 4), 0.125, 0.3, (1, 1, 1, 1)),
    "8^4/2^4": ((8, 8, 8, 8), (2, 2, 2, 2), 0.120, 0.25, (1, 1, 1, 1)),
}
EO = (0, 0, 0, 0)


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(name, seed=11, **kw):
    from paper_1210_7398_amd import sapq

    L, B, kappa, eps, bc = GEOMS[name]
    U = synth.gauge_field(L, eps, seed)
    F = synth.clover_inverse(L, U, 1.0, kappa)
    s = sapq.Solver(L, B, EO, kappa, bc=bc, block_solver="eomr", **kw)
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    return s, L, B, kappa, bc, U, F


@pytest.mark.parametrize("name", list(GEOMS))
@pytest.mark.parametrize("n_ssor", [1, 4])
def test_block_solve_both_colours(torch_cuda, orc, name, n_ssor):
    s, L, B, kappa, bc, U, F = _setup(name, n_ssor=n_ssor)
    prm = orc.params(kappa, n_ssor=n_ssor, block_solver=1)
    v = synth.gaussian_spinor(L, 12)
    for colour in (0, 1):
        want = orc.eomr(L, B, U, F, prm, colour, v, bc=bc)
        got = to_host(s.ssor(to_dev(v), colour))
        check_close(got, want, 2e-5, f"EO-MR block solve colour {colour}")
    s.close()


@pytest.mark.parametrize("name", list(GEOMS))
def test_sap_precondition(torch_cuda, orc, name):
    s, L, B, kappa, bc, U, F = _setup(name, n_sap=3)
    v = synth.gaussian_spinor(L, 13)
    y_w, dy_w = orc.msap(L, B, EO, U, F, orc.params(kappa, n_sap=3, block_solver=1), v, bc=bc)
    y, dy = s.sap_precondition(to_dev(v))
    check_close(to_host(y), y_w, 2e-5, "EO-MR M_SAP")
    check_close(to_host(dy), dy_w, 2e-5, "EO-MR D M_SAP")
    s.close()


# M_SAP tolerances of the low-precision storage parity tests (unit roundoff 2^-11 / 2^-8)
# 3 unit roundoffs of the storage format, as for the SSOR's M_SAP (test_gpu_parity.PREC_TOL)
MSAP_TOL = {"fp16": 1.5e-3, "bf16": 1.2e-2}


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("name", ["8^4/4^4", "12^4/6^4 antiperiodic"])
def test_sap_precondition_low_precision(torch_cuda, orc, name, prec):
    s, L, B, kappa, bc, U, F = _setup(name, prec=prec)
    v = synth.gaussian_spinor(L, 14)
    y_w, dy_w = orc.msap(L, B, EO, U, F, orc.params(kappa, block_solver=1), v, bc=bc)
    y, dy = s.sap_precondition(to_dev(v))
    check_close(to_host(y), y_w, MSAP_TOL[prec], f"EO-MR M_SAP {prec}")
    check_close(to_host(dy), dy_w, MSAP_TOL[prec], f"EO-MR D M_SAP {prec}")
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("name", ["8^4/4^4", "12^4/6^4 antiperiodic"])
def test_solve_true_residual(torch_cuda, orc, name, prec):
    s, L, B, kappa, bc, U, F = _setup(name, prec=prec)
    b = synth.gaussian_spinor(L, 15)
    x, st = s.solve(to_dev(b), tol=1e-10)
    x = to_host(x)
    assert relerr(orc.dslash(L, U, F, kappa, x, bc=bc), b) <= 1e-10, st
    xo, _, ok = orc.solve(L, B, EO, U, F, orc.params(kappa, block_solver=1), b, tol=1e-12, bc=bc)
    assert ok
    check_close(x, xo, 1e-8, "EO-MR solution")
    s.close()


def test_solve_with_learned_stage(torch_cuda, orc):
    """The learned stage ahead of the MR-preconditioned M_SAP (z = N r + M_SAP (r - D N r)):
    the solve still reaches the FP64 true residual with the oracle's operator."""
    import torch

    from paper_1210_7398_amd import sapq

    s, L, B, kappa, bc, U, F = _setup("8^4/4^4", nn=True)
    g = torch.Generator(device="cpu").manual_seed(19)
    s.nn_set_weights((0.02 * torch.randn(sapq.nn_param_count(), generator=g)).float().cuda())
    s.use_nn(True)
    b = synth.gaussian_spinor(L, 20)
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert relerr(orc.dslash(L, U, F, kappa, to_host(x), bc=bc), b) <= 1e-10, st
    s.close()


def test_solve_24x24x24x48_lattice(torch_cuda, orc):
    """The 24^3x48 lattice with 6^4 blocks (256 workgroups per colour, 3 even sites per lane
    pair): FP64 true residual 1e-10 with the oracle's operator."""
    from paper_1210_7398_amd import sapq

    L, B, kappa = (24, 24, 24, 48), (6, 6, 6, 6), 0.1255
    U = synth.gauge_field(L, 0.25, 16)
    F = synth.clover_inverse(L, U, 1.0, kappa)
    s = sapq.Solver(L, B, EO, kappa, block_solver="eomr")
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    b = synth.gaussian_spinor(L, 17)
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert relerr(orc.dslash(L, U, F, kappa, to_host(x)), b) <= 1e-10, st
    s.close()


def test_refusals(torch_cuda):
    """The MR block solver needs the even-odd site order and an even number of sites per
    block; autotune and the batched solver refuse it; switching it on later needs a context
    that can run it."""
    from paper_1210_7398_amd import sapq

    L, B = (8, 8, 8, 8), (4, 4, 4, 4)
    with pytest.raises(sapq.SapqError) as e:
        sapq.Solver(L, B, (2, 2, 2, 2), 0.12, block_solver="eomr")
    assert e.value.code == -2  # SAPQ_ESHAPE
    with pytest.raises(sapq.SapqError) as e:
        sapq.Solver((6, 6, 6, 6), (3, 3, 3, 3), EO, 0.12, block_solver="eomr")
    assert e.value.code == -2  # SAPQ_ESHAPE
    with pytest.raises(sapq.SapqError) as e:  # 8^4 blocks: 384 KiB of LDS for the block vector
        sapq.Solver((16, 16, 16, 16), (8, 8, 8, 8), EO, 0.12, block_solver="eomr")
    assert e.value.code == -2  # SAPQ_ESHAPE
    s, L, B, kappa, bc, U, F = _setup("8^4/4^4")
    with pytest.raises(sapq.SapqError) as e:
        s.autotune()
    assert e.value.code == -1  # SAPQ_EINVAL
    with pytest.raises(sapq.SapqError) as e:
        sapq.solve_batch([s], [to_dev(synth.gaussian_spinor(L, 18)[None])], tol=1e-8)
    assert e.value.code == -1  # SAPQ_EINVAL
    s.close()
    t = sapq.Solver(L, B, (2, 2, 2, 2), 0.12)
    t.params.flags = sapq.FLAG_EOMR
    with pytest.raises(sapq.SapqError) as e:
        t.set_params()
    assert e.value.code == -1  # SAPQ_EINVAL
    t.close()
