"""Seeded synthetic inputs for the measurement operator Phi = Theta G F Z.

This package only *produces data*: sky images, uv/w coverages, the dense
S x S windows that make up the rows of the de-gridding matrix G, and the
deapodisation vectors that go with the Kaiser-Bessel interpolation kernel.
It never applies the operator, its adjoint or the l2-ball step: those belong
to ``oracle/`` (the FP64 CPU checker) and to the HIP library, which both
consume what is generated here and share nothing else.

Every chunk (configuration, channel, block) is regenerable on its own from
``numpy.random.SeedSequence((220907604, cfg, l, b))``.
"""
from .kb import (KB_J, KB_ALPHA, kb_beta, kb_psi, kb_psi_hat, deapodisation,
                 window_base)
from .problem import (Problem, Block, make_problem, CONFIGS, config_names)

__all__ = [
    "KB_J", "KB_ALPHA", "kb_beta", "kb_psi", "kb_psi_hat", "deapodisation",
    "window_base", "Problem", "Block", "make_problem", "CONFIGS", "config_names",
]
