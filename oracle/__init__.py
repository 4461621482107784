"""FP64 CPU oracle for the RI measurement operator and the data-fidelity step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path (``paper_2209_07604_amd``):
both sides only consume the seeded inputs produced by ``synth``.

Contents (each function cites the passage it follows):
  operator  Phi = Theta G F Z and its adjoint (Section 2.1, eq. 1)
  dual      l2-ball projection and the PDFB data-fidelity dual step (Section 2.2, eq. 2)
  nudft     direct non-uniform DFT (what the NUFFT of eq. 1 approximates)
  dr        visibility-gridding dimensionality reduction (Section 3.4, eqs. 4-5)
  analysis  PSF, its peak normalisation eta_l and the residual image (the
            residual-image definition among the evaluation metrics), and
            ||Phi_l||^2 (dense definition and the power method)
  gbuild    rows of G from per-visibility tables: Kaiser-Bessel kernel
            convolved with the w-kernel and the antenna pair's DDE kernel
            (Sections 3.1-3.2)
  pdfb      regularizer-free PDFB iteration (non-negativity only, Section 2.2)
            with the adaptive l2-bound rule of the effective noise
            estimation (Section 3.3)

Everything is complex128 / float64.
"""
from .operator import (Operator, BlockG, zpad, zpad_adj, fft2_fwd, fft2_adj,
                       g_matrix, grid_fwd)
from .dual import (l2ball_project, dual_step, chi2_radius, block_radii)
from .nudft import nudft

__all__ = ["Operator", "BlockG", "zpad", "zpad_adj", "fft2_fwd", "fft2_adj",
           "g_matrix", "grid_fwd", "l2ball_project", "dual_step", "chi2_radius",
           "block_radii", "nudft"]
