"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws and arranges input data: periodic Voronoi grain maps,
random orientations, stiff spherical particles, material constant blocks and
the macroscopic deformation-gradient history of the cyclic test.  It performs
none of the solver's arithmetic (no projection, no constitutive law, no
Newton/CG), so the CPU oracle and the HIP library can both consume the same
inputs without sharing any of the method's code.
"""

from .micro import (voronoi_periodic, shoemake_quaternions, place_particles,
                    Microstructure, make_microstructure)
from .loading import macro_F, triangle, cyclic_history
from .configs import (RveConfig, CONFIGS, config_by_name, material_params,
                      PARAM_NAMES)

__all__ = [
    "voronoi_periodic", "shoemake_quaternions", "place_particles",
    "Microstructure", "make_microstructure", "macro_F", "triangle",
    "cyclic_history", "RveConfig", "CONFIGS", "config_by_name",
    "material_params", "PARAM_NAMES",
]
