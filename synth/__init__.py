"""Seeded synthetic inputs for the VAG Darcy + transport path.

This package only *generates problem data* (meshes, fracture face lists,
permeabilities, boundary data).  It holds none of the discretisation's
arithmetic, so both the CPU oracle and the GPU library may consume it.
"""
from .meshes import (  # noqa: F401
    Problem,
    node_index,
    structured_hex,
    plane_faces,
    config1,
    config2,
    config3,
    config4_job,
    config5,
    cartesian_problem,
    planes_problem,
    random_problem,
    add_wells,
    e1_problem,
    e2_problem,
    CONFIGS,
    GeneralProblem,
    general_problem,
    general_from_hex,
    faces_of_cells,
    general_workload,
    grid_cells,
)
