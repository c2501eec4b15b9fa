"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark: triangular meshes, frozen Eulerian fields and the particle-count
recipe of each workload.

This package holds none of the particle method's arithmetic.  It produces what
the paper's Eulerian solvers and mesh generator would hand to the particle
step (section 3, the canyon meshes and the converged mean fields), which are
not available, so smooth synthetic stand-ins are generated instead.
"""
from .mesh import Mesh, EDGE, unit_square_mesh, canyon_mesh, doubly_periodic_box
from .fields import FIELD_NAMES, NFIELD, uniform_fields, canyon_fields
from .configs import (Workload, Ensemble, config1, config2, config3, config3w, config3b, config4, config5,
                      small_canyon,
                      tiny_canyon, square_box, apportion, SLM, GLM, PSI_ZERO, PSI_LEFT_QUARTER)

__all__ = [
    "Mesh", "EDGE", "unit_square_mesh", "canyon_mesh", "doubly_periodic_box",
    "FIELD_NAMES", "NFIELD", "uniform_fields", "canyon_fields",
    "Workload", "config1", "config2", "config3", "config3w", "config3b", "config4", "config5",
    "small_canyon", "tiny_canyon", "square_box", "apportion", "Ensemble",
    "SLM", "GLM", "PSI_ZERO", "PSI_LEFT_QUARTER",
]
