"""Error paths and degenerate cases of the C ABI on the GPU: links that are not SU(3), calls
before the fields are loaded, aliased arguments, a zero source, kappa = 0, and the time-out of
a split block's wait on its partner (forced from the host, so every kernel still ends)."""
import ctypes

import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests.gpu_common import GEOMS, fields, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

NAME = "8^4/4^4/2^4"


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solver(name=NAME, load=True, **kw):
    from paper_1210_7398_amd import sapq

    L, B, S, kappa, eps, bc = GEOMS[name]
    s = sapq.Solver(L, B, S, kappa, bc=bc, **kw)
    if load:
        U, F = fields(name)
        s.load_gauge(to_dev(U))
        s.load_clover(to_dev(F))
    return s


def test_links_that_are_not_su3_are_refused(torch_cuda):
    from paper_1210_7398_amd import sapq

    L = GEOMS[NAME][0]
    U, F = fields(NAME)
    bad = U.copy()
    bad[5, 2] *= 1.001  # one link no longer unitary
    s = _solver(load=False)
    with pytest.raises(sapq.SapqError) as e:
        s.load_gauge(to_dev(bad))
    assert e.value.code == -3 and "SU(3)" in str(e.value)
    s.load_clover(to_dev(F))
    with pytest.raises(sapq.SapqError) as e:  # the refused field is not in use
        s.solve(to_dev(synth.gaussian_spinor(L, 3)), tol=1e-10)
    assert e.value.code == -8
    s.load_gauge(to_dev(U))  # a good field afterwards makes the context usable
    x, st = s.solve(to_dev(synth.gaussian_spinor(L, 3)), tol=1e-10)
    assert st["true_relres"] <= 1e-10
    s.close()


def test_calls_before_the_fields_are_loaded(torch_cuda):
    from paper_1210_7398_amd import sapq

    L = GEOMS[NAME][0]
    s = _solver(load=False)
    b = to_dev(synth.gaussian_spinor(L, 4))
    for call in (lambda: s.dslash(b), lambda: s.solve(b, tol=1e-10), lambda: s.sap_precondition(b)):
        with pytest.raises(sapq.SapqError) as e:
            call()
        assert e.value.code == -8
    s.close()


def test_aliased_dslash_arguments_are_refused(torch_cuda):
    from paper_1210_7398_amd import sapq

    L = GEOMS[NAME][0]
    s = _solver()
    psi = to_dev(synth.gaussian_spinor(L, 5))
    before = psi.clone()
    p = ctypes.c_void_p(psi.data_ptr())
    assert sapq.lib().sapq_dslash(s.h, p, p, 0) == -1
    assert torch_cuda.equal(psi, before)  # output untouched
    s.close()


def test_zero_source_gives_zero_solution(torch_cuda):
    L = GEOMS[NAME][0]
    s = _solver()
    b = torch_cuda.zeros((int(np.prod(L)), 4, 3), dtype=torch_cuda.complex128, device="cuda")
    x, st = s.solve(b, tol=1e-10)
    assert torch_cuda.count_nonzero(x) == 0 and st["true_relres"] == 0.0 and st["outer_its"] == 0
    s.close()


def test_kappa_zero_is_refused_and_tiny_kappa_solves_at_once(torch_cuda, orc):
    """kappa = 0 is outside the parameter range (EINVAL at creation).  At kappa = 1e-8 the
    operator is 1 up to 1e-8, so one outer step reaches the tolerance and x = b to 1e-7."""
    from paper_1210_7398_amd import sapq

    L, B, S, kappa, eps, bc = GEOMS[NAME]
    with pytest.raises(sapq.SapqError) as e:
        sapq.Solver(L, B, S, 0.0, bc=bc)
    assert e.value.code == -1
    U, F = fields(NAME)
    s = sapq.Solver(L, B, S, 1e-8, bc=bc)
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    b = synth.gaussian_spinor(L, 6)
    x, st = s.solve(to_dev(b), tol=1e-10)
    x = to_host(x)
    assert relerr(x, b) < 1e-7 and st["outer_its"] <= 2
    assert relerr(orc.dslash(L, U, F, 1e-8, x, bc=bc), b) <= 1e-10
    s.close()


def test_split_block_wait_time_out_is_reported(torch_cuda, monkeypatch):
    """The split kernel's bounded wait on the other half of a block: with every wait made to
    time out (SAPQ_HALO_TIMEOUT_TEST, read at context creation), the call returns SAPQ_EHIP
    with the time-out message instead of hanging or returning a wrong result silently."""
    from paper_1210_7398_amd import sapq

    name = "12^3x24/6^3x12/3^3x6"
    L = GEOMS[name][0]
    v = to_dev(synth.gaussian_spinor(L, 7))
    monkeypatch.setenv("SAPQ_HALO_TIMEOUT_TEST", "1")
    s = _solver(name)
    assert s.phase_kernel == "two-lane split"
    with pytest.raises(sapq.SapqError) as e:
        s.ssor(v, 0)
    assert e.value.code == -6 and "timed out" in str(e.value)
    s.close()
    monkeypatch.delenv("SAPQ_HALO_TIMEOUT_TEST")
    s = _solver(name)  # a context made without the switch is unaffected
    s.ssor(v, 0)
    s.close()
