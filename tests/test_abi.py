"""The C-ABI library loads, exports every symbol include/sapq.h declares, and validates
geometries on the host (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "sapq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sapq_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1210_7398_amd import sapq

    L = sapq.lib()
    names = declared_symbols()
    assert "sapq_solve" in names and "sapq_dslash" in names
    for n in names:
        assert hasattr(L, n), n


def _bytes(L, B, S, prec="fp32"):
    from paper_1210_7398_amd import sapq

    g = sapq.Geom((ctypes.c_int * 4)(*L), (ctypes.c_int * 4)(*B), (ctypes.c_int * 4)(*S), (ctypes.c_int * 4)(1, 1, 1, 1))
    p = sapq.Params(0.125, 1.0, 1e-2, 4, 4, 50, 100, sapq.PREC[prec], 0, 0)
    return sapq.lib().sapq_arena_bytes(ctypes.byref(g), ctypes.byref(p))


def test_geometry_validation():
    assert _bytes((8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2)) > 0
    assert _bytes((24, 24, 24, 48), (6, 6, 6, 12), (3, 3, 3, 6)) > 0
    assert _bytes((8, 8, 8, 12), (4, 4, 4, 4), (2, 2, 2, 2)) == 0  # 3 blocks in t: odd
    assert _bytes((8, 8, 8, 8), (8, 4, 4, 4), (2, 2, 2, 2)) == 0  # one block in x
    assert _bytes((8, 8, 8, 8), (4, 4, 4, 4), (1, 2, 2, 2)) == 0  # sub-block extent 1
    assert _bytes((12, 8, 8, 8), (6, 4, 4, 4), (4, 2, 2, 2)) == 0  # sub-block does not divide
    assert _bytes((8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 2), "fp64") == 0  # inner precision


def test_arena_scales_with_storage_precision():
    b32 = _bytes((16, 16, 16, 32), (4, 4, 4, 4), (2, 2, 2, 2), "fp32")
    b16 = _bytes((16, 16, 16, 32), (4, 4, 4, 4), (2, 2, 2, 2), "fp16")
    assert 0 < b16 < b32
