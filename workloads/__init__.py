"""Seeded synthetic inputs (meshes, upwind operators, right-hand sides).

This package serves both the HIP path and the CPU oracle and therefore holds
none of the multigrid method's arithmetic: only mesh generation and operator
assembly.
"""
from .configs import Problem, p0_square, dg_square, p0_cube, batch, adjoint, concat, by_name, SEEDS  # noqa: F401
