"""GPU parity of the learned stage through the C ABI, against the FP64 oracle.

The tests use weights that BF16 represents exactly.  On the FP32-FMA path the only
differences are FP32 rounding of ~300-term sums (forward 1e-5) and of site sums over 4096
sites (weight gradients 1e-4).  The default MFMA path also rounds the transported inputs to
BF16 (2^-9 relative per term, so ~2e-3 per layer): 1e-2 for the three-layer forward, 2e-2 for
gradients."""
import numpy as np
import pytest

from paper_1210_7398_amd import synth
from tests import helpers as H
from tests.gpu_common import GEOMS, check_close, fields, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

NAME = "8^4/4^4/2^4"


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _check_weights(got, want, tol):
    """Relative 2-norm error of a weight blob below tol, and no single weight off by more than
    SITE_FACTOR * tol of the RMS weight."""
    from tests.gpu_common import SITE_FACTOR

    assert relerr(got, want) < tol, relerr(got, want)
    m = float(np.abs(got - want).max() / np.sqrt(np.mean(want**2)))
    assert m < SITE_FACTOR * tol, m


def _preconditioned_residual(s, r, use_nn):
    """|(1 - D P) r| / |r| for the inner preconditioner P of the library (sapq_precondition):
    M_SAP, or the learned stage ahead of M_SAP."""
    import torch

    s.use_nn(use_nn)
    _, dz = s.precondition(r)
    return float(torch.linalg.vector_norm(r - dz) / torch.linalg.vector_norm(r))


def bf16_exact(x):
    """Round float32 values to the nearest BF16 value (ties to even), kept as float32."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def rand_weights(orc, seed, scale=0.15):
    rng = np.random.default_rng(seed)
    return bf16_exact(scale * rng.normal(size=orc.nn_param_count()))


def make(torch, name=NAME, **kw):
    from paper_1210_7398_amd import sapq

    L, B, S, kappa, eps, bc = GEOMS[name]
    U, F = fields(name)
    kw.setdefault("nn_fp32", True)
    s = sapq.Solver(L, B, S, kappa, bc=bc, nn=True, **kw)
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    return s


def test_nn_forward_parity(torch_cuda, orc):
    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    s = make(torch)
    w = rand_weights(orc, 1)
    s.nn_set_weights(torch.from_numpy(w).cuda())
    assert np.array_equal(s.nn_get_weights().cpu().numpy(), w)
    r = synth.gaussian_spinor(L, 201)
    z_w, _ = orc.nn_forward(L, U, orc.nn_unflatten(w), r, bc)
    z = to_host(s.nn_forward(to_dev(r)))
    check_close(z, z_w, 1e-5, "network forward fp32")


def test_nn_mfma_forward_and_backward_parity(torch_cuda, orc):
    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    s = make(torch, nn_fp32=False)
    w = rand_weights(orc, 11)
    s.nn_set_weights(torch.from_numpy(w).cuda())
    r = synth.gaussian_spinor(L, 211)
    Ws = orc.nn_unflatten(w)
    z_w, _ = orc.nn_forward(L, U, Ws, r, bc)
    check_close(to_host(s.nn_forward(to_dev(r))), z_w, 1e-2, "network forward mfma")
    gz = synth.gaussian_spinor(L, 212)
    gw, gin = s.nn_backward(to_dev(gz), to_dev(r))
    grads, gin_w = orc.nn_backward(L, U, Ws, r, gz, bc)
    _check_weights(gw.cpu().numpy().astype(np.float64), orc.nn_flatten(grads), 2e-2)
    check_close(to_host(gin), gin_w, 1e-2, "input gradient mfma")


def test_nn_forward_gauge_equivariance(torch_cuda, orc):
    from paper_1210_7398_amd import sapq

    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    V = int(np.prod(L))
    g = synth.random_su3_field(V, 202)
    w = torch.from_numpy(rand_weights(orc, 2)).cuda()
    r = synth.gaussian_spinor(L, 203)
    outs = []
    for Uk, rk in ((U, r), (H.gauge_transform(L, U, g), H.transform_spinor(r, g))):
        s = sapq.Solver(L, B, S, kappa, nn=True, nn_fp32=True)
        s.load_gauge(to_dev(Uk))
        s.nn_set_weights(w)
        outs.append(to_host(s.nn_forward(to_dev(rk))))
    check_close(outs[1], H.transform_spinor(outs[0], g), 1e-5, "network equivariance")


def test_nn_backward_parity(torch_cuda, orc):
    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    s = make(torch)
    w = rand_weights(orc, 3)
    s.nn_set_weights(torch.from_numpy(w).cuda())
    r = synth.gaussian_spinor(L, 204)
    gz = synth.gaussian_spinor(L, 205)
    gw, gin = s.nn_backward(to_dev(gz), to_dev(r))
    grads, gin_w = orc.nn_backward(L, U, orc.nn_unflatten(w), r, gz, bc)
    _check_weights(gw.cpu().numpy().astype(np.float64), orc.nn_flatten(grads), 1e-4)
    check_close(to_host(gin), gin_w, 1e-5, "input gradient fp32")


def test_nn_train_step_is_adam_on_the_batch_loss(torch_cuda, orc):
    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    s = make(torch)
    w = rand_weights(orc, 4, 0.05)
    s.nn_set_weights(torch.from_numpy(w).cuda())
    es = [synth.gaussian_spinor(L, 206 + k) for k in range(2)]
    e_dev = torch.stack([torch.view_as_real(to_dev(e).to(torch.complex64)) for e in es]).contiguous()
    loss = s.nn_train_step(e_dev, [0, 1], 1e-3, 1)
    Ws = orc.nn_unflatten(w)
    ref_loss, g = 0.0, 0.0
    for e in es:
        e32 = e.astype(np.complex64).astype(np.complex128)
        r = orc.dslash(L, U, F, kappa, e32, bc=bc)
        l, gr = orc.nn_loss_grad(L, U, Ws, r, e32, bc)
        ref_loss += l / 2
        g = g + orc.nn_flatten(gr) / 2
    assert abs(loss - ref_loss) < 1e-5 * ref_loss
    dw = s.nn_get_weights().cpu().numpy().astype(np.float64) - w
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    # first Adam step: every weight moves by lr against the sign of its gradient
    assert np.allclose(dw[big], -1e-3 * np.sign(g[big]), rtol=1e-3, atol=1e-6)


@pytest.mark.parametrize("outer", ["fbicgstab", "defect"])
def test_nn_solve_true_residual(torch_cuda, orc, outer):
    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    s = make(torch, outer=outer, nn_fp32=False)
    b = synth.gaussian_spinor(L, 210)
    x0, st0 = s.solve(to_dev(b), tol=1e-10)
    s.nn_set_weights(torch.zeros(orc.nn_param_count(), dtype=torch.float32, device="cuda"))
    x1, st1 = s.solve(to_dev(b), tol=1e-10)
    # N = 0 leaves the preconditioner exactly M_SAP
    assert st1["inner_its"] == st0["inner_its"] and torch.equal(x0, x1)
    s.nn_set_weights(torch.from_numpy(rand_weights(orc, 5, 0.02)).cuda())
    x2, st2 = s.solve(to_dev(b), tol=1e-10)
    rr = relerr(orc.dslash(L, U, F, kappa, to_host(x2), bc=bc), b)
    assert rr <= 1e-10, (rr, st2)


def test_nn_training_gain(torch_cuda, orc):
    """Train on pairs from the plain SAP solver on two fields, then on a held-out field the
    learned stage must lower the residual that the inner preconditioner leaves, and the full
    solve must still reach 1e-10."""
    from paper_1210_7398_amd import sapq, train_nn

    torch = torch_cuda
    L, B, S, kappa = (8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), 0.125
    sets = []
    for seed in (21, 22):
        U = synth.gauge_field(L, 0.25, seed)
        F = synth.clover_inverse(L, U, 1.0, kappa)
        s = sapq.Solver(L, B, S, kappa, nn=True)
        s.load_gauge(to_dev(U))
        s.load_clover(to_dev(F))
        src = [to_dev(synth.gaussian_spinor(L, 1000 * seed + k)) for k in range(12)]
        sets.append((s, train_nn.make_pairs(s, src, n_iter=5)))
    w0 = train_nn.init_weights(0)
    for s, _ in sets:
        s.nn_set_weights(w0)
    losses = train_nn.train(sets, steps=240, batch=4, lr=2e-3)
    assert np.mean(losses[-20:]) < 0.8 * np.mean(losses[:20])
    w = sets[-1][0].nn_get_weights()
    U = synth.gauge_field(L, 0.25, 25)
    F = synth.clover_inverse(L, U, 1.0, kappa)
    s = sapq.Solver(L, B, S, kappa, nn=True)
    s.load_gauge(to_dev(U))
    s.load_clover(to_dev(F))
    s.nn_set_weights(w)
    # held-out pairs from the plain solver, as the training pairs are made (with the stage on,
    # the iterates would keep only the error that the network does not remove)
    s.use_nn(False)
    held = train_nn.make_pairs(s, [to_dev(synth.gaussian_spinor(L, 25001))], n_iter=4)
    gains = []
    for k in range(1, held.shape[0]):
        e = torch.view_as_complex(held[k]).to(torch.complex128).contiguous()
        r = s.dslash(e, "fp64")
        plain = _preconditioned_residual(s, r, False)
        learned = _preconditioned_residual(s, r, True)
        gains.append(plain / learned)
    print("preconditioned-residual gain per held-out iterate:", gains)
    assert np.mean(gains) > 1.0
    s.use_nn(True)
    b = synth.gaussian_spinor(L, 25002)
    x, st = s.solve(to_dev(b), tol=1e-10)
    assert relerr(orc.dslash(L, U, F, kappa, to_host(x)), b) <= 1e-10


def test_nn_copy_state_continues_adam(torch_cuda, orc):
    """Training that hands its state (weights and both Adam moments) to another context goes
    on as if uninterrupted: two Adam steps split over two contexts of the same field give the
    same weights, bit for bit, as two steps on one context.  Restarting the second step from
    the weights alone (moments reset) does not."""
    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    V = int(np.prod(L))
    a, b, c, d = (make(torch) for _ in range(4))
    w0 = torch.from_numpy(rand_weights(orc, 7)).cuda()
    g = torch.Generator().manual_seed(8)
    e = torch.randn((4, V, 4, 3, 2), generator=g, dtype=torch.float32).cuda()
    for s in (a, c, d):
        s.nn_set_weights(w0)
    c.nn_train_step(e, [0, 1], 1e-3, 1)
    c.nn_train_step(e, [2, 3], 1e-3, 2)
    a.nn_train_step(e, [0, 1], 1e-3, 1)
    b.nn_copy_state_from(a)
    b.nn_train_step(e, [2, 3], 1e-3, 2)
    assert torch.equal(b.nn_get_weights(), c.nn_get_weights())
    d.nn_train_step(e, [0, 1], 1e-3, 1)
    d.nn_set_weights(d.nn_get_weights())
    d.nn_train_step(e, [2, 3], 1e-3, 2)
    assert not torch.equal(d.nn_get_weights(), c.nn_get_weights())
    for s in (a, b, c, d):
        s.close()


def test_nn_adam_step_matches_adam(torch_cuda, orc):
    """sapq_nn_adam_step with a caller-supplied gradient is Adam (Kingma and Ba) on the FP32
    master weights: two steps against the oracle's Adam in FP64, the moments carried in the
    context between them; the layers then use the BF16-rounded result."""
    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    s = make(torch)
    rng = np.random.default_rng(31)
    w = rand_weights(orc, 30, 0.05).astype(np.float64)
    s.nn_set_weights(torch.from_numpy(w.astype(np.float32)).cuda())
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    p = w.copy()
    for t, lr in ((1, 1e-3), (2, 5e-4)):
        g = rng.normal(size=w.size).astype(np.float32)
        s.nn_adam_step(torch.from_numpy(g).cuda(), lr, t)
        orc.adam_step(p, g.astype(np.float64), m, v, lr, t)
        got = s.nn_get_weights().cpu().numpy().astype(np.float64)
        # FP32 update of O(1e-3) steps on O(0.1) weights: a few FP32 ulps of the weights
        assert np.abs(got - p).max() < 1e-6, (t, np.abs(got - p).max())
    # the forward pass uses the updated weights, rounded to BF16 like any set weights
    q = torch.from_numpy(p.astype(np.float32)).cuda()
    r = to_dev(synth.gaussian_spinor(L, 32))
    z1 = s.nn_forward(r)
    s2 = make(torch)
    s2.nn_set_weights(s.nn_get_weights())
    assert torch.equal(z1, s2.nn_forward(r))
    assert torch.allclose(q, s.nn_get_weights(), rtol=0, atol=1e-6)
    s.close()
    s2.close()


def test_defect_errors_are_the_plain_solver_iterates(torch_cuda, orc):
    """sapq_defect_errors: e_0 = x* (x_0 = 0) rounded to FP32; every later e_k = x* - x_k has
    a residual b - D x_k = D e_k (checked with the oracle's D) that the defect correction
    shrinks by about the inner tolerance per step, as section 2's outer iteration does."""
    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    s = make(torch)
    b = synth.gaussian_spinor(L, 33)
    xs, _ = s.solve(to_dev(b), tol=1e-12)
    e = s.defect_errors(to_dev(b), xs, 4)
    assert tuple(e.shape) == (4, int(np.prod(L)), 4, 3, 2)
    ek = [e[k].cpu().numpy().astype(np.float64) for k in range(4)]
    ek = [a[..., 0] + 1j * a[..., 1] for a in ek]
    x_star = to_host(xs)
    assert np.array_equal(ek[0], x_star.astype(np.complex64).astype(np.complex128))
    res = []
    for k in range(4):
        xk = x_star - ek[k]
        res.append(relerr(orc.dslash(L, U, F, kappa, xk, bc=bc), b))
    print("defect-correction residuals:", res)
    assert res[0] > 0.99  # x_0 = 0 up to FP32 rounding of e_0
    for k in range(1, 4):
        assert res[k] < 0.25 * res[k - 1], res  # inner tolerance 0.1 per step


def test_precondition_with_and_without_the_stage(torch_cuda, orc):
    """sapq_precondition: with the stage off it is M_SAP (the oracle's), with it on it is
    N + M_SAP (1 - D N), with D P v from the SAP recurrence; both against the oracle."""
    torch = torch_cuda
    L, B, S, kappa, eps, bc = GEOMS[NAME]
    U, F = fields(NAME)
    s = make(torch, nn_fp32=True)
    v = synth.gaussian_spinor(L, 34)
    y_w, dy_w = orc.msap(L, B, S, U, F, orc.params(kappa), v, bc=bc)
    y, dy = (to_host(t) for t in s.precondition(to_dev(v)))
    check_close(y, y_w, 2e-5, "P = M_SAP")
    check_close(dy, dy_w, 2e-5, "D P = D M_SAP")
    w = rand_weights(orc, 35, 0.05)
    s.nn_set_weights(torch.from_numpy(w).cuda())
    s.use_nn(True)
    z, _ = orc.nn_forward(L, U, orc.nn_unflatten(w), v, bc)
    rp = v - orc.dslash(L, U, F, kappa, z, bc=bc)
    m_w, dm_w = orc.msap(L, B, S, U, F, orc.params(kappa), rp, bc=bc)
    y, dy = (to_host(t) for t in s.precondition(to_dev(v)))
    # the FP32 network (1e-5) feeds the M_SAP chain (2e-5)
    check_close(y, z + m_w, 5e-5, "P = N + M_SAP (1 - D N)")
    check_close(dy, v - rp + dm_w, 5e-5, "D P")
    s.close()
