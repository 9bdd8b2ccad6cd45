"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Meshes (``synth.mesh``), closed-form fields and exact cell averages
(``synth.fields``) and the named workloads (``synth.configs``).  Nothing here
computes any step of the finite-volume method.
"""
from . import configs, fields, mesh  # noqa: F401
from .mesh import HEX, KUHN6, PRISM_X, PRISM_Y, PRISM_Z, Mesh, mixed_kinds, periodic_2d, periodic_3d  # noqa: F401
