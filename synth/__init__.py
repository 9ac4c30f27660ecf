"""Seeded synthetic inputs for the Maxwell parallel imaging encoding operator.

This package only draws data: phantoms, orthonormal smooth bases (dense or
Tucker-factored), coefficients, Cartesian masks, radial trajectories,
density-compensation weights and unit noise.  It holds none of the
operator's arithmetic (no DFT, no basis apply, no sampling), so that the
FP64 oracle and the HIP path can both consume its outputs without sharing
code.
"""
from .inputs import *  # noqa: F401,F403
