"""MI355X (gfx950) implementation of the Euler-Lagrange bubble-column method of arXiv 1710.07073:
a fused D3Q19 BGK lattice-Boltzmann step with a per-cell Guo body force, two-way coupled to
Lagrangian bubbles through the clipped fourth-order polynomial mapping kernel.

``lbm`` is the ctypes binding of the C ABI (include/lbm.h); ``sim`` builds simulations on it
with PyTorch-owned device buffers.
"""
from . import lbm  # noqa: F401

__all__ = ["lbm"]
