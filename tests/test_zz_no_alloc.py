"""The allocation-free entry point sapq_dslash_noalloc (staging in the library's static device
array) against sapq_dslash (staging in the context's arena), through the C ABI: the same
kernels on the same data, so the results must agree bit for bit.  Two calls in a row on one
GPU, the second with a smaller lattice, in FP64 and in the inner precision; a lattice whose
staging exceeds the static array is refused before any work."""
import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests.gpu_common import GEOMS, fields, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solver(name, prec):
    from paper_1210_7398_amd import sapq

    L, B, S, kappa, eps, bc = GEOMS[name]
    U, F = fields(name)
    s = sapq.Solver(L, B, S, kappa, bc=bc, prec=prec)
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    return s


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_dslash_noalloc_equals_dslash(torch_cuda, prec):
    torch = torch_cuda
    # the larger lattice first, then a smaller one: the static array keeps the first call's
    # contents, which the second call must not read
    for name, seed in (("12^3x24/6^3x12/3^3x6", 401), ("8^4/4^4/2^4", 402)):
        s = _solver(name, prec)
        L = GEOMS[name][0]
        psi = to_dev(synth.gaussian_spinor(L, seed))
        for p in ("fp64", prec):
            want = s.dslash(psi, p)
            out = torch.full_like(psi, float("nan"))
            torch.cuda.synchronize()
            s.dslash_noalloc(psi, out, p)
            torch.cuda.synchronize()
            assert torch.equal(out, want), (name, p, float((out - want).abs().max()))
        s.close()


def test_dslash_noalloc_refuses_a_lattice_beyond_its_scratch(torch_cuda):
    """32^3x64 in FP64 needs 2 x 12 x 2^21 x 16 bytes = 805 MB of staging, beyond the 256 MiB
    array: SAPQ_ENOMEM, and the output is left untouched."""
    from paper_1210_7398_amd import sapq

    torch = torch_cuda
    L = (32, 32, 32, 64)
    s = sapq.Solver(L, (4, 4, 4, 4), (2, 2, 2, 2), 0.125)
    V = int(np.prod(L))
    psi = torch.zeros((V, 4, 3), dtype=torch.complex128, device="cuda")
    out = torch.full_like(psi, 7.0)
    with pytest.raises(sapq.SapqError) as e:
        s.dslash_noalloc(psi, out, "fp64")
    assert e.value.code == -7 and "static scratch" in str(e.value)
    assert bool((out == 7.0).all())
    s.close()
