"""Training of the learned preconditioner stage on the GPU, through the C ABI.

Training pairs come from the plain SAP solver: for a Gaussian source b the nested
solve gives x* (to 1e-12), and defect-correction iterates x_0 = 0,
x_{k+1} = x_k + Inner(b - D x_k) give the pairs (r_k, e_k) = (b - D x_k, x* - x_k).
Only e_k is stored (float32, interchange layout, formed by sapq_defect_errors); the
library forms r_k = D e_k in FP32 inside sapq_nn_train_step.  The loss is the batch mean of |N r - e|^2 / |e|^2
and the update is Adam; forward, backward and the update run in the library's kernels.
"""
import sys

import numpy as np
import torch

from . import sapq, synth


def init_weights(seed, scale=0.02, device="cuda"):
    """Small random weights, except the local term of every layer, which starts near a
    multiple of the identity so that N starts close to a scaled identity map."""
    rng = np.random.default_rng(seed)
    n = sapq.nn_param_count()
    w = scale * rng.normal(size=n)
    C = 8
    shapes = [(1, C), (C, C), (C, 1)]
    off = 0
    for ci, co in shapes:
        blk = w[off : off + 2 * 16 * 9 * ci * co].reshape(9, co, ci, 4, 4, 2)
        for c in range(min(ci, co)):
            blk[0, c, c, :, :, 0] += np.eye(4) * (1.0 / np.sqrt(max(ci, co)) if ci != co else 1.0)
        off += blk.size
    return torch.tensor(w, dtype=torch.float32, device=device)


def make_pairs(solver, sources, n_iter=5, tol=1e-12):
    """Error vectors e_k = x* - x_k of defect-correction iterates of the plain SAP solver,
    k = 0 .. n_iter-1, for each source (x* its solve to tol; the iterates and errors are formed
    by the library, sapq_defect_errors); returns a float32 tensor [n, V, 4, 3, 2]."""
    out = []
    for b in sources:
        xs, _ = solver.solve(b, tol=tol, check=False)
        out.append(solver.defect_errors(b, xs, n_iter))
    return torch.cat(out)


def train(solvers_and_pairs, steps, batch=8, lr=1e-3, seed=0, log=None):
    """Adam on mini-batches drawn in turn from each (solver, e) entry (one solver per field);
    the training state (weights and Adam moments) passes from each solver to the next, so the
    solvers run one Adam.  Returns the per-step losses; log=n prints every n-th to stderr."""
    rng = np.random.default_rng(seed)
    losses = []
    prev = None
    for t in range(1, steps + 1):
        solver, e = solvers_and_pairs[(t - 1) % len(solvers_and_pairs)]
        if prev is not None and prev is not solver:
            solver.nn_copy_state_from(prev)
        idx = rng.integers(0, e.shape[0], size=batch)
        losses.append(solver.nn_train_step(e, idx, lr, t))
        prev = solver
        if log and (t % log == 0 or t == 1):
            print(f"# nn step {t}: loss {np.mean(losses[-log:]):.4f}", file=sys.stderr, flush=True)
    return losses
