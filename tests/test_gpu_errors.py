"""Error paths and degenerate cases of the C ABI on the GPU: links that are not SU(3), calls
before the fields are loaded, aliased arguments, a zero source, kappa = 0, the time-out of
a split block's wait on its partner, and the breakdown detection and fallbacks of the solver
(a NaN source, NaN network weights, forced FP16/BF16 breakdowns, one inner iteration).  Every
failure is forced from the host, so every kernel still ends normally."""
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


# ---------------------------------------------------------------- failure detection and fallbacks
def test_nan_in_the_source_is_a_breakdown_at_once(torch_cuda):
    """A source holding a NaN cannot be solved: EBREAKDOWN before any inner solve, instead of
    maxit_outer outer iterations of NaN arithmetic."""
    from paper_1210_7398_amd import sapq

    L = GEOMS[NAME][0]
    s = _solver()
    b = synth.gaussian_spinor(L, 8)
    b[17, 2, 1] = np.nan
    with pytest.raises(sapq.SapqError) as e:
        s.solve(to_dev(b), tol=1e-10)
    assert e.value.code == -5 and "not finite" in str(e.value)
    x, st = s.solve(to_dev(b), tol=1e-10, check=False)
    assert st["outer_its"] == 0 and st["inner_its"] == 0
    s.close()


def test_zero_source_with_a_guess_gives_zero(torch_cuda):
    """b = 0 has the solution x = 0 whatever the guess."""
    L = GEOMS[NAME][0]
    s = _solver()
    V = int(np.prod(L))
    b = torch_cuda.zeros((V, 4, 3), dtype=torch_cuda.complex128, device="cuda")
    x0 = to_dev(synth.gaussian_spinor(L, 9))
    x, st = s.solve(b, tol=1e-10, x0=x0)
    assert torch_cuda.count_nonzero(x) == 0 and st["true_relres"] == 0.0
    s.close()


def test_one_inner_iteration_still_converges(torch_cuda, orc):
    """maxit_inner = 1: each preconditioner call is one M_SAP-preconditioned BiCGStab step,
    which the flexible outer iteration accepts; the FP64 true residual still reaches 1e-10."""
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    s = _solver(maxit_inner=1, maxit_outer=400)
    b = synth.gaussian_spinor(L, 10)
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert st["inner_its"] <= 2 * st["outer_its"] and st["breakdowns"] == 0
    assert relerr(orc.dslash(L, U, F, kappa, to_host(x), bc=bc), b) <= 1e-10
    s.close()


def _nan_weights(torch):
    from paper_1210_7398_amd import sapq

    w = torch.full((sapq.nn_param_count(),), float("nan"), dtype=torch.float32, device="cuda")
    return w


@pytest.mark.parametrize("outer", ["fbicgstab", "defect"])
def test_nan_network_falls_back_to_plain_sap(torch_cuda, orc, outer):
    """Weights of NaN make the learned stage's output NaN: the first inner solve breaks down,
    is redone with plain M_SAP, and the solve converges as the plain solver does."""
    from paper_1210_7398_amd import sapq

    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    s = _solver(nn=True, outer=outer)
    b = synth.gaussian_spinor(L, 11)
    x_plain, st_plain = s.solve(to_dev(b), tol=1e-10)  # no weights set: plain SAP
    s.nn_set_weights(_nan_weights(torch_cuda))
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert st["fallback"] == sapq.FALLBACK_NN and st["breakdowns"] == 1, st
    assert relerr(orc.dslash(L, U, F, kappa, to_host(x), bc=bc), b) <= 1e-10
    assert st["outer_its"] == st_plain["outer_its"]
    s.close()


def test_low_precision_breakdown_without_fallback_is_reported(torch_cuda, monkeypatch):
    """Every FP16 inner solve made to break down from the host (SAPQ_TEST_LOWPREC_NAN, read at
    creation): with no FP32 copies reserved the solve returns EBREAKDOWN after the first one."""
    from paper_1210_7398_amd import sapq

    L = GEOMS[NAME][0]
    monkeypatch.setenv("SAPQ_TEST_LOWPREC_NAN", "1")
    s = _solver(prec="fp16")
    monkeypatch.delenv("SAPQ_TEST_LOWPREC_NAN")
    b = to_dev(synth.gaussian_spinor(L, 12))
    x, st = s.solve(b, tol=1e-10, check=False)
    assert st["breakdowns"] == 1 and st["fallback"] == 0 and st["outer_its"] == 0, st
    with pytest.raises(sapq.SapqError) as e:
        s.solve(b, tol=1e-10)
    assert e.value.code == -5
    s.close()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("outer", ["fbicgstab", "defect"])
def test_low_precision_breakdown_falls_back_to_fp32(torch_cuda, orc, monkeypatch, prec, outer):
    """The same forced breakdown with FP32 copies reserved (SAPQ_FLAG_FALLBACK_FP32): the inner
    solve is redone in FP32 storage, the rest of the solve stays there, the solution reaches
    1e-10 and agrees with the oracle's; the next solve starts in the low precision again."""
    from paper_1210_7398_amd import sapq

    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    monkeypatch.setenv("SAPQ_TEST_LOWPREC_NAN", "1")
    s = _solver(prec=prec, outer=outer, fallback_fp32=True)
    monkeypatch.delenv("SAPQ_TEST_LOWPREC_NAN")
    b = synth.gaussian_spinor(L, 13)
    for _ in range(2):
        x, st = s.solve(to_dev(b), tol=1e-10)
        assert st["fallback"] == sapq.FALLBACK_FP32 and st["breakdowns"] == 1, st
        x = to_host(x)
        assert relerr(orc.dslash(L, U, F, kappa, x, bc=bc), b) <= 1e-10
    xo, _, ok = orc.solve(L, B, S, U, F, orc.params(kappa), b, tol=1e-12, bc=bc)
    assert ok and relerr(x, xo) < 1e-8
    s.close()


def test_both_fallbacks_in_one_solve(torch_cuda, orc, monkeypatch):
    """Learned stage with NaN weights in an FP16 context whose FP16 inner solves break down:
    the stage goes first, then the storage precision, and the solve still converges."""
    from paper_1210_7398_amd import sapq

    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    monkeypatch.setenv("SAPQ_TEST_LOWPREC_NAN", "1")
    s = _solver(prec="fp16", nn=True, fallback_fp32=True)
    monkeypatch.delenv("SAPQ_TEST_LOWPREC_NAN")
    s.nn_set_weights(_nan_weights(torch_cuda))
    b = synth.gaussian_spinor(L, 14)
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert st["fallback"] == sapq.FALLBACK_NN | sapq.FALLBACK_FP32 and st["breakdowns"] == 2, st
    assert relerr(orc.dslash(L, U, F, kappa, to_host(x), bc=bc), b) <= 1e-10
    s.close()


def test_fallback_copies_follow_a_sub_block_change(torch_cuda, orc, monkeypatch):
    """The FP32 copies of an FP16 context are re-laid out with the fields when the sub-block
    shape changes (here through the autotuner's cache), so the FP32 fallback still solves."""
    import json

    from paper_1210_7398_amd import sapq

    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    monkeypatch.setenv("SAPQ_TEST_LOWPREC_NAN", "1")
    s = _solver(prec="fp16", fallback_fp32=True)
    monkeypatch.delenv("SAPQ_TEST_LOWPREC_NAN")
    import tempfile, os

    path = os.path.join(tempfile.mkdtemp(), "tune.jsonl")
    key = (f"L={L[0]}x{L[1]}x{L[2]}x{L[3]};B={B[0]}x{B[1]}x{B[2]}x{B[3]};kappa={kappa:.6f};nssor=4;nsap=4;"
           f"prec={sapq.FP16}")
    with open(path, "w") as f:
        f.write(json.dumps({"key": key, "subblock": [2, 4, 2, 4], "time_s": 1.0}) + "\n")
    assert s.autotune(path) == (2, 4, 2, 4)
    b = synth.gaussian_spinor(L, 15)
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert st["fallback"] == sapq.FALLBACK_FP32
    assert relerr(orc.dslash(L, U, F, kappa, to_host(x), bc=bc), b) <= 1e-10
    s.close()
