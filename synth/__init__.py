"""Seeded synthetic inputs shared by the solver path and the checker.

This package holds no arithmetic of the solver or of the finite element
discretisation: only workload descriptions (mesh sizes, material constants,
solver settings), a counter-free splitmix64 stream and the random numbers
drawn from it.  Both sides receive the same random numbers as inputs.
"""

from .seeds import SplitMix64, fourier_coefficients, serving_stream  # noqa: F401
from .configs import ProblemSpec, CONFIGS, config  # noqa: F401
