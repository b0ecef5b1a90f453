"""Shared set-up of the GPU parity tests: seeded fields on the host, copies on the device."""
import functools

import numpy as np

from paper_1210_7398_amd import synth

# name: (lattice, SAP block, sub-block, kappa, eps, bc)
GEOMS = {
    "8^4/4^4/2^4": ((8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), 0.120, 0.25, (1, 1, 1, 1)),
    "12^3x24/6^3x12/3^3x6": ((12, 12, 12, 24), (6, 6, 6, 12), (3, 3, 3, 6), 0.125, 0.25, (1, 1, 1, 1)),
    "12^4/6^4/3^4": ((12, 12, 12, 12), (6, 6, 6, 6), (3, 3, 3, 3), 0.125, 0.25, (1, 1, 1, 1)),
    "8x4x4x8/4x2x2x4/2^4 antiperiodic": ((8, 4, 4, 8), (4, 2, 2, 4), (2, 2, 2, 2), 0.125, 0.3, (1, 1, 1, -1)),
    # sub-block (0, 0, 0, 0): SSOR in even-odd site order instead of ll order
    "8^4/4^4/even-odd": ((8, 8, 8, 8), (4, 4, 4, 4), (0, 0, 0, 0), 0.120, 0.25, (1, 1, 1, 1)),
    "12^4/6^4/even-odd antiperiodic": ((12, 12, 12, 12), (6, 6, 6, 6), (0, 0, 0, 0), 0.125, 0.25, (1, 1, 1, -1)),
}


@functools.lru_cache(maxsize=None)
def fields(name, seed=7):
    L, B, S, kappa, eps, bc = GEOMS[name]
    U = synth.gauge_field(L, eps, seed)
    F = synth.clover_inverse(L, U, 1.0, kappa)
    return U, F


def relerr(a, b):
    return float(np.linalg.norm((a - b).reshape(-1)) / np.linalg.norm(b.reshape(-1)))


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    return t.cpu().numpy()
