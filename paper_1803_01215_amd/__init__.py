"""hjpd: grid-free Hamilton-Jacobi solves on MI355X.

Per-point primal-dual splitting of Lin, Chow and Osher (arXiv 1803.01215)
as hand-written HIP kernels for gfx950 behind a C ABI (include/hjpd.h).
``paper_1803_01215_amd.hjpd`` is the ctypes binding with the C names;
``paper_1803_01215_amd.solver`` wraps it for torch tensors.
"""
from . import hjpd  # noqa: F401

__all__ = ["hjpd"]
