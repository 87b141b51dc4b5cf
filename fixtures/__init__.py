"""Seeded synthetic FEM inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only builds problem *inputs* (structured Q1 meshes, element matrices, coefficients
and right-hand sides).  It contains none of the solver's arithmetic: no tree, no elimination, no
substitution.  Both the CPU oracle and the HIP path consume what it produces.
"""
from .mesh import (  # noqa: F401
    Mesh, Problem, structured_q1, q1_reference_matrices, element_matrices,
    reaction_diffusion, advection_diffusion, config_problem, CONFIGS,
)
