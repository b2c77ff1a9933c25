"""Seeded synthetic inputs for the solver, its oracle and the benchmark.

This package only draws random numbers and builds test matrices; it holds
none of the solver's arithmetic (no factorization, solve or refinement), so
both the GPU path and the CPU oracle can be fed from it without sharing code.
"""
from .gen import (  # noqa: F401
    batched_systems,
    grad_problem,
    haar_orthogonal,
    integer_system,
    prescribed_cond_system,
    sigma_geometric,
    spd_system,
    uniform_system,
)
