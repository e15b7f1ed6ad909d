"""Seeded synthetic inputs for the Sternheimer solves (shared by the library's
tests/benchmarks and the CPU oracle; contains none of the method's arithmetic)."""
from . import crystal, configs  # noqa: F401
from .configs import Problem, batch, held_out, si2, si16, si64, si64nl, small  # noqa: F401
