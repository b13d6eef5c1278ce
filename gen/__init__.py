"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package holds no arithmetic of the distance method: it only builds meshes
(vertex and triangle arrays) and query point sets from seeded random draws.
"""
from .meshes import (uv_sphere, capped_cylinder, capped_cone, cylinder_cone,
                     icosphere, displaced_icosphere, torus, cube, tetrahedron,
                     regular_ngon_prism)
from .queries import uniform_box, near_surface, scaled_box
from .configs import (SEED_BASE, config_c0, config_c1, config_c2, config_c3,
                      config_c4, c4_plan)

__all__ = [
    "uv_sphere", "capped_cylinder", "capped_cone", "cylinder_cone", "icosphere",
    "displaced_icosphere", "torus", "cube", "tetrahedron", "regular_ngon_prism",
    "uniform_box", "near_surface", "scaled_box", "SEED_BASE", "config_c0",
    "config_c1", "config_c2", "config_c3", "config_c4", "c4_plan",
]
