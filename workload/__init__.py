"""Seeded synthetic DLPNO doubles-residual workloads (descriptors + inputs).

Shared by the CPU checker and the GPU path; holds none of the method's
arithmetic, only the data model (which pairs, which spin blocks are stored,
where each tensor lives) and the random draws.
"""
from .problem import Problem, build_problem, CONFIGS, BLOCK_BITS, BLOCK_NAMES  # noqa: F401
