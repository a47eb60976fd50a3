"""Seeded synthetic microstructure generators.

This package produces inputs only: inclusion lists, voxel images, random
rotations, request streams.  It holds none of the homogenisation method's
arithmetic (no Fourier coefficients of materials, no projections, no solver,
no quadrature), so that both the CPU oracle and the GPU path can draw the
same inputs from it without sharing any of the computation under test.
"""

from .microstructures import (  # noqa: F401
    square_inclusion,
    circle_inclusion_vf,
    cube_inclusion_aniso,
    random_circles,
    random_spd,
    grf_voxels,
    serving_requests,
    serving_requests_3d,
    poisson_arrivals,
    with_arrivals,
    grf_request,
    polycrystal,
    multiphase_aniso,
)
