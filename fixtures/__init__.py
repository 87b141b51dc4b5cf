"""Seeded synthetic FEM inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only builds problem *inputs* (structured Q_p meshes, element matrices, coefficients
and right-hand sides).  It contains none of the solver's arithmetic: no tree, no elimination, no
substitution.  Both the CPU oracle and the HIP path consume what it produces.
"""
from .mesh import (  # noqa: F401
    Mesh, Problem, structured_q1, q1_reference_matrices, element_matrices,
    reaction_diffusion, advection_diffusion, config_problem, CONFIGS,
    structured_qp, qp_reference_matrices, lagrange_1d, load_vector, node_coords, l2_projection,
    l2_workload, L2_SHAPES,
)
