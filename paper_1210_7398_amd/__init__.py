"""sapq: an MI355X-native SAP/SSOR clover-Wilson quark solver (Boku et al., arXiv:1210.7398).

The compute path is the C-ABI library ``libsapq.so`` (hand-written HIP kernels
for gfx950, declared in ``include/sapq.h``); :mod:`paper_1210_7398_amd.sapq` is
its thin ctypes binding.  Importing this package loads nothing: the library is
opened on first use and raises if it is missing.
"""
__all__ = ["sapq", "synth"]
