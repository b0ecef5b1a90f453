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
from tests.gpu_common import GEOMS, fields, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

NAME = "8^4/4^4/2^4"


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


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
    assert relerr(z, z_w) < 1e-5


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
    assert relerr(to_host(s.nn_forward(to_dev(r))), z_w) < 1e-2
    gz = synth.gaussian_spinor(L, 212)
    gw, gin = s.nn_backward(to_dev(gz), to_dev(r))
    grads, gin_w = orc.nn_backward(L, U, Ws, r, gz, bc)
    assert relerr(gw.cpu().numpy().astype(np.float64), orc.nn_flatten(grads)) < 2e-2
    assert relerr(to_host(gin), gin_w) < 1e-2


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
    assert relerr(outs[1], H.transform_spinor(outs[0], g)) < 1e-5


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
    assert relerr(gw.cpu().numpy().astype(np.float64), orc.nn_flatten(grads)) < 1e-4
    assert relerr(to_host(gin), gin_w) < 1e-5


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
        plain = train_nn.preconditioned_residual(s, r, False)
        learned = train_nn.preconditioned_residual(s, r, True)
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
