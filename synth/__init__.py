"""Seeded synthetic inputs shared by the oracle and the GPU product path.

This package holds *inputs only*: triangle meshes (structured, Delaunay,
jittered), their uniform (quadrisection) and barycentric (Alfeld) refinements
with parent maps, and the analytic problem data (manufactured solution,
forcing functions).  It contains none of the solver's arithmetic: no finite
element basis, no quadrature, no assembly, no patches, no factorisation, no
multigrid and no Krylov method.  Those live twice, independently, in
``oracle/`` and in ``paper_2407_07253_amd/``.
"""
from .meshes import (  # noqa: F401
    Mesh,
    structured_square,
    delaunay_square,
    jitter_interior,
    refine_uniform,
    alfeld_split,
    hierarchy,
    config_mesh_hierarchy,
    structured_cube,
    cube_hierarchy,
)
from .problem_data import (  # noqa: F401
    mms_amplitude,
    mms_velocity,
    mms_pressure,
    mms_forcing,
    gaussian_bump_params,
    gaussian_bump_forcing,
    fourier_field_params,
    fourier_field,
    log_viscosity,
    gaussian_bump_params3d,
    gaussian_bump_forcing3d,
)
