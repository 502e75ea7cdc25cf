"""Seeded synthetic inputs shared by the library's tests, the oracle's tests and the benchmark.

Holds no arithmetic of the method itself: surfaces (node positions and their
parameter derivatives), coefficient values with ambient gradients, and
right-hand sides.
"""
from .surfaces import Surface, cube_sphere, torus, torus_boundary_curve, gl_nodes, real_sph_harm_cartesian  # noqa: F401
from .configs import (  # noqa: F401
    Problem, sphere_problem, ellipsoid_problem, star_problem, wobbly_torus_problem, wavy_torus_problem,
    helmholtz_sphere_problem, helmholtz_ellipsoid_problem, EdgeSamples, wavy_torus_piece_problem,
    serving_requests, random_density,
)
