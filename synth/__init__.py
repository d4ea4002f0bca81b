"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds inputs: vertex coordinates and element-to-vertex
tables of pyramid meshes, random coefficient vectors and per-element
materials, and the vertex identities of periodic meshes.  It holds none of the discretisation's arithmetic (no basis, no
cubature, no geometric factors, no face matching).
"""

from .mesh import (hex_pyramid_mesh, octahedron_mesh, periodic_pair_ids, single_pyramid,
                   warped_pyramid)
from .fields import random_state, random_materials, n_basis

__all__ = [
    "hex_pyramid_mesh",
    "octahedron_mesh",
    "periodic_pair_ids",
    "single_pyramid",
    "warped_pyramid",
    "random_state",
    "random_materials",
    "n_basis",
]
