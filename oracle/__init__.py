"""CPU FP64 oracle for the Sternheimer hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library or its binding.
"""
from . import sternheimer_oracle  # noqa: F401
from .sternheimer_oracle import *  # noqa: F401,F403
from .driver import solve_pairs, spectral_setup  # noqa: F401
