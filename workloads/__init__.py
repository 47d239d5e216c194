"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds no arithmetic of the discretization itself: it evaluates the
push-forward map of a warped periodic box at reference node positions supplied by
the caller, smooth random initial fields, the Taylor-Green initial condition,
cotangent vectors, the neighbour table of a structured grid, and the manufactured solution of the
viscous error-vs-cost study with its forcing (``workloads.mms``).
"""
from .inputs import (  # noqa: F401
    Problem, make_problem, config, CONFIG_NAMES, batch_config,
    coords, state, neighbours, cotangent, direction, cfl_dt, mms_problem,
    channel_problem, problem_neighbours, jumped_state, mapping_jacobian,
)
from . import mms  # noqa: F401
