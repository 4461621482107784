"""MI355X (gfx950) implementation of the RI measurement operator hot path of
Faceted HyperSARA (arXiv 2209.07604): Phi = Theta G F Z, its adjoint and the
l2-ball data-fidelity dual step, as hand-written HIP kernels behind a C ABI
(include/phi.h, libphi.so).  This package is the thin Python binding.
"""
from ._lib import PhiError, load, EXPORTS, PER_CHANNEL, GRAPH, PERSISTENT, FUSED_GH, DR  # noqa: F401
from .plan import Plan  # noqa: F401
