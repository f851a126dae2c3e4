"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package holds only input generators: mesh descriptions (node coordinates,
connectivity, boundary tags), case parameters and a counter-based random
generator.  It contains none of the spectral-difference arithmetic, so both
the CPU oracle and the HIP library can consume what it produces without
sharing any of the method's code.
"""
from .meshes import (FACE_INTERIOR, FACE_PERIODIC, FACE_SLIDING,  # noqa: F401
                     FACE_WALL_ISOTHERMAL, FACE_WALL_SLIP, FACE_FARFIELD,
                     GEOM_LINEAR, GEOM_CUBIC)
