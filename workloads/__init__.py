"""Seeded synthetic inputs (meshes, materials, boundary flags, load vectors).

This package is shared by the CPU oracle and the GPU path. It only produces
inputs; it holds none of the solver's arithmetic (no stiffness assembly, no
region tree, no V-cycle, no PCG).
"""
from .meshes import (  # noqa: F401
    Mesh, grid2d, grid3d, grid3d_box, box3d, signed_measure, load_constant, load_function_tri,
    load_function_tet, manufactured_2d, manufactured_mesh, cfg1, cfg2, cfg3, cfg4,
    small2d, small3d, request_mesh, fourier_body_force, load_fourier_tet,
)
