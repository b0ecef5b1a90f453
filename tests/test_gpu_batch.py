"""Batched solve (several fields of different sizes, several sources each) and the sub-block
autotuner, through the C ABI, against the FP64 oracle and the one-source solver."""
import json

import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests.gpu_common import check_close, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _field(L, eps, seed, kappa):
    U = synth.gauge_field(L, eps, seed)
    return U, synth.clover_inverse(L, U, 1.0, kappa)


def point_sources(L, n):
    return np.stack([synth.point_source(L, k % 4, (k // 4) % 3) for k in range(n)])


# group size 1 is the default; 4 (with 5 and 2 sources: groups of 4 + 1 and 2) and 3 run the
# multi-source workgroups, whose slices each hold one source's iterate
@pytest.mark.parametrize("group", ["1", "3", "4"])
@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_solve_batch_two_fields(torch_cuda, orc, prec, group, monkeypatch):
    from paper_1210_7398_amd import sapq

    monkeypatch.setenv("SAPQ_BATCH_NR", group)
    torch = torch_cuda
    kappa = 0.125
    B, S = (4, 4, 4, 4), (2, 2, 2, 2)
    cfg = [((8, 8, 8, 8), 0.2, 31, 5), ((8, 8, 8, 16), 0.3, 32, 2)]  # lattice, eps, seed, sources
    solvers, srcs, fields = [], [], []
    for L, eps, seed, n in cfg:
        U, F = _field(L, eps, seed, kappa)
        s = sapq.Solver(L, B, S, kappa, prec=prec, outer="defect", maxit_outer=100)
        s.load_gauge(to_dev(U))
        s.load_clover(to_dev(F))
        b = point_sources(L, n)
        b[-1] = synth.gaussian_spinor(L, seed)  # one Gaussian source too
        solvers.append(s)
        srcs.append(to_dev(b))
        fields.append((L, U, F, b))
    xs, stats = sapq.solve_batch(solvers, srcs, tol=1e-10)
    q = 0
    for (L, U, F, b), x, s in zip(fields, xs, solvers):
        x = to_host(x)
        for k in range(b.shape[0]):
            rr = relerr(orc.dslash(L, U, F, kappa, x[k]), b[k])
            assert rr <= 1e-10, (L, k, rr, stats[q])
            assert stats[q]["true_relres"] <= 1e-10
            x1, _ = s.solve(to_dev(np.ascontiguousarray(b[k])), tol=1e-10)
            check_close(x[k], to_host(x1), 1e-8, f"batched vs one-source solution {L} source {k}")
            q += 1


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_solve_batch_with_learned_stage(torch_cuda, orc, prec):
    """The learned stage inside the batched inner solver (z = N r + M_SAP (r - D N r) per source):
    every source reaches the true residual with the oracle's D, and the solutions agree with the
    one-source solver using the same stage."""
    from paper_1210_7398_amd import sapq

    torch = torch_cuda
    kappa = 0.125
    B, S = (4, 4, 4, 4), (2, 2, 2, 2)
    cfg = [((8, 8, 8, 8), 0.25, 41, 3), ((8, 8, 8, 16), 0.25, 42, 2)]
    g = torch.Generator(device="cpu").manual_seed(5)
    w = (0.02 * torch.randn(sapq.nn_param_count(), generator=g)).float().cuda()
    solvers, srcs, fields = [], [], []
    for L, eps, seed, n in cfg:
        U, F = _field(L, eps, seed, kappa)
        s = sapq.Solver(L, B, S, kappa, prec=prec, outer="defect", maxit_outer=100, nn=True)
        s.load_gauge(to_dev(U))
        s.load_clover(to_dev(F))
        s.nn_set_weights(w)
        s.use_nn(True)
        b = np.stack([synth.gaussian_spinor(L, 100 * seed + k) for k in range(n)])
        solvers.append(s)
        srcs.append(to_dev(b))
        fields.append((L, U, F, b))
    xs, stats = sapq.solve_batch(solvers, srcs, tol=1e-10)
    q = 0
    for (L, U, F, b), x, s in zip(fields, xs, solvers):
        x = to_host(x)
        for k in range(b.shape[0]):
            assert relerr(orc.dslash(L, U, F, kappa, x[k]), b[k]) <= 1e-10, (L, k, stats[q])
            x1, _ = s.solve(to_dev(np.ascontiguousarray(b[k])), tol=1e-10)
            check_close(x[k], to_host(x1), 1e-8, f"batched vs one-source solution {L} source {k}")
            q += 1


def test_autotune_picks_a_valid_subblock_and_caches(torch_cuda, orc, tmp_path):
    from paper_1210_7398_amd import sapq

    L, B, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.125
    U, F = _field(L, 0.25, 33, kappa)
    s = sapq.Solver(L, B, (2, 2, 2, 2), kappa)
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    cache = str(tmp_path / "tune.jsonl")
    S = s.autotune(cache)
    assert S == (0, 0, 0, 0) or all(sb >= 2 and B[m] % sb == 0 for m, sb in enumerate(S))
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and "subblock" in lines[0]
    assert s.autotune(cache) == S and len(open(cache).read().strip().splitlines()) == 1
    # the tuned context solves with the chosen ll ordering, which the oracle reproduces
    b = synth.gaussian_spinor(L, 34)
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert relerr(orc.dslash(L, U, F, kappa, to_host(x)), b) <= 1e-10
    v = synth.gaussian_spinor(L, 35)
    y_w, _ = orc.msap(L, B, S, U, F, orc.params(kappa), v)
    y, _ = s.sap_precondition(to_dev(v))
    check_close(to_host(y), y_w, 2e-5, "M_SAP after the sub-block change")


def test_subblock_change_relays_out_the_fields(torch_cuda, orc, tmp_path):
    """A tuning-cache hit with a sub-block shape other than the context's changes the slot
    order inside every block; the packed links and clover field (and the learned stage's link
    table) must follow it.  Checked after the change: the solve against the oracle's operator,
    M_SAP against the oracle's M_SAP with the new ll order, the network against the oracle."""
    import json

    from paper_1210_7398_amd import sapq

    torch = torch_cuda
    L, B, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.125
    U, F = _field(L, 0.25, 36, kappa)
    s = sapq.Solver(L, B, (2, 2, 2, 2), kappa)
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    cache = tmp_path / "tune.jsonl"
    first = s.autotune(str(cache))
    s.close()
    entry = json.loads(cache.read_text().splitlines()[0])
    S_new = (4, 2, 2, 4) if tuple(first) != (4, 2, 2, 4) else (2, 4, 4, 2)
    entry["subblock"] = list(S_new)
    cache.write_text(json.dumps(entry) + "\n")

    s = sapq.Solver(L, B, (2, 2, 2, 2), kappa, nn=True, nn_fp32=True)
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    assert s.autotune(str(cache)) == S_new
    b = synth.gaussian_spinor(L, 37)
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert relerr(orc.dslash(L, U, F, kappa, to_host(x)), b) <= 1e-10
    v = synth.gaussian_spinor(L, 38)
    y_w, _ = orc.msap(L, B, S_new, U, F, orc.params(kappa), v)
    y, _ = s.sap_precondition(to_dev(v))
    check_close(to_host(y), y_w, 2e-5, "M_SAP after the sub-block change")
    rng = np.random.default_rng(39)
    w = (0.15 * rng.normal(size=orc.nn_param_count())).astype(np.float32)
    w = w.view(np.uint32) & np.uint32(0xFFFF0000)  # BF16-exact weights (truncated)
    w = w.view(np.float32)
    s.nn_set_weights(torch.from_numpy(w).cuda())
    r = synth.gaussian_spinor(L, 40)
    z_w, _ = orc.nn_forward(L, U, orc.nn_unflatten(w), r)
    check_close(to_host(s.nn_forward(to_dev(r))), z_w, 1e-5, "network after the sub-block change")
    s.close()


def test_solve_batch_even_odd_order(torch_cuda, orc):
    """The batched solver with SSOR in even-odd site order (sub-block (0, 0, 0, 0)): every source
    reaches the true residual with the oracle's D and equals the one-source solve."""
    from paper_1210_7398_amd import sapq

    kappa, B, S = 0.125, (4, 4, 4, 4), (0, 0, 0, 0)
    cfg = [((8, 8, 8, 8), 0.25, 51, 3), ((8, 8, 8, 16), 0.2, 52, 2)]
    solvers, srcs, fields = [], [], []
    for L, eps, seed, n in cfg:
        U, F = _field(L, eps, seed, kappa)
        s = sapq.Solver(L, B, S, kappa, outer="defect", maxit_outer=100)
        s.load_gauge(to_dev(U))
        s.load_clover(to_dev(F))
        b = point_sources(L, n)
        solvers.append(s)
        srcs.append(to_dev(b))
        fields.append((L, U, F, b))
    xs, stats = sapq.solve_batch(solvers, srcs, tol=1e-10)
    for (L, U, F, b), x, s in zip(fields, xs, solvers):
        x = to_host(x)
        for k in range(b.shape[0]):
            assert relerr(orc.dslash(L, U, F, kappa, x[k]), b[k]) <= 1e-10
            x1, _ = s.solve(to_dev(np.ascontiguousarray(b[k])), tol=1e-10)
            check_close(x[k], to_host(x1), 1e-8, f"batched vs one-source solution {L} source {k}")
    for s in solvers:
        s.close()


def test_solve_batch_c4_fields(torch_cuda, orc):
    """The batched workload's four fields at full size (16^3x32 eps 0.2, 24^3x48 eps 0.25 and
    0.3, 32^3x64 eps 0.25; kappa 0.125, 4^4 blocks, 2^4 sub-blocks) with their 12 spin-colour
    point sources, 48 solves in one call: every solution's true residual with the oracle's FP64
    D, and the first source of every field against the one-source solver.  A second call on the
    same batch replays the captured graphs and must give the same solutions bit for bit."""
    from paper_1210_7398_amd import sapq

    torch = torch_cuda
    kappa, B, S = 0.125, (4, 4, 4, 4), (2, 2, 2, 2)
    cfg = [((16, 16, 16, 32), 0.2, 11), ((24, 24, 24, 48), 0.25, 12), ((24, 24, 24, 48), 0.3, 13),
           ((32, 32, 32, 64), 0.25, 14)]
    dev = torch.device("cuda:0")
    solvers, srcs, host = [], [], []
    for L, eps, seed in cfg:
        U = synth.gauge_field(L, eps, seed, device=dev)
        F = synth.clover_inverse(L, U, 1.0, kappa, device=dev)
        s = sapq.Solver(L, B, S, kappa, outer="defect")
        s.load_gauge(U)
        s.load_clover(F)
        host.append((L, U.cpu().numpy(), F.cpu().numpy()))
        del U, F
        solvers.append(s)
        srcs.append(to_dev(point_sources(L, 12)))
    xs, stats = sapq.solve_batch(solvers, srcs, tol=1e-10)
    xs2, _ = sapq.solve_batch(solvers, srcs, tol=1e-10)
    q = 0
    for (L, U, F), x, x2, s, b in zip(host, xs, xs2, solvers, srcs):
        assert torch.equal(x, x2), L
        xh, bh = to_host(x), to_host(b)
        for k in range(12):
            rr = relerr(orc.dslash(L, U, F, kappa, xh[k]), bh[k])
            assert rr <= 1e-10, (L, k, rr, stats[q])
            assert stats[q]["true_relres"] <= 1e-10 and stats[q]["breakdowns"] == 0
            q += 1
        x1, _ = s.solve(b[0].contiguous(), tol=1e-10)
        check_close(xh[0], to_host(x1), 1e-8, f"C4 batched vs one-source {L}")
    for s in solvers:
        s.close()
    sapq.release_batch_arena()


def test_solve_batch_nan_source_breaks_down_alone(torch_cuda, orc):
    """A source holding a NaN stops at once with a breakdown (EBREAKDOWN for the call); the
    other sources of the batch still converge."""
    from paper_1210_7398_amd import sapq

    kappa, B, S, L = 0.125, (4, 4, 4, 4), (2, 2, 2, 2), (8, 8, 8, 8)
    U, F = _field(L, 0.25, 35, kappa)
    s = sapq.Solver(L, B, S, kappa, outer="defect")
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    b = np.stack([synth.gaussian_spinor(L, 350 + k) for k in range(3)])
    b[1, 5, 0, 0] = np.nan
    with pytest.raises(sapq.SapqError) as e:
        sapq.solve_batch([s], [to_dev(b)], tol=1e-10)
    assert e.value.code == -5
    xs, st = sapq.solve_batch([s], [to_dev(b)], tol=1e-10, check=False)
    assert st[1]["breakdowns"] == 1 and st[1]["outer_its"] == 0
    x = to_host(xs[0])
    for k in (0, 2):
        assert st[k]["breakdowns"] == 0
        assert relerr(orc.dslash(L, U, F, kappa, x[k]), b[k]) <= 1e-10
    s.close()


def test_autotune_batch_picks_and_caches(torch_cuda, orc, tmp_path):
    """sapq_autotune_batch times sources per workgroup and inner iterations per graph replay,
    keeps a valid pair, caches it, and the batched solve with it still meets the oracle."""
    from paper_1210_7398_amd import sapq

    kappa, B, S = 0.125, (4, 4, 4, 4), (2, 2, 2, 2)
    cfg = [((8, 8, 8, 8), 0.25, 36, 4), ((8, 8, 8, 16), 0.25, 37, 3)]
    solvers, srcs, fields = [], [], []
    for L, eps, seed, n in cfg:
        U, F = _field(L, eps, seed, kappa)
        s = sapq.Solver(L, B, S, kappa, outer="defect")
        s.load_gauge(to_dev(U))
        s.load_clover(to_dev(F))
        b = np.stack([synth.gaussian_spinor(L, 360 + seed + k) for k in range(n)])
        solvers.append(s)
        srcs.append(to_dev(b))
        fields.append((L, U, F, b))
    cache = str(tmp_path / "batch_tune.jsonl")
    nr, k = sapq.autotune_batch(solvers, srcs, tol=1e-10, cache_path=cache)
    assert 1 <= nr <= 4 and k in (1, 2, 4)
    assert len(open(cache).read().strip().splitlines()) == 1
    rec = json.loads(open(cache).read().strip())
    cand = rec["candidates"]  # every timed (nr, k, median seconds); the chosen pair is the fastest
    assert cand and all(c[0] in (1, 2, 3, 4) and c[1] in (1, 2, 4) and c[2] > 0 for c in cand)
    fastest = min(cand, key=lambda c: c[2])
    assert (fastest[0], fastest[1]) == (nr, k) == (rec["nr"], rec["k_inner"])
    assert sapq.autotune_batch(solvers, srcs, tol=1e-10, cache_path=cache) == (nr, k)
    assert len(open(cache).read().strip().splitlines()) == 1
    xs, st = sapq.solve_batch(solvers, srcs, tol=1e-10)
    for (L, U, F, b), x in zip(fields, xs):
        x = to_host(x)
        for j in range(b.shape[0]):
            assert relerr(orc.dslash(L, U, F, kappa, x[j]), b[j]) <= 1e-10
    for s in solvers:
        s.close()
