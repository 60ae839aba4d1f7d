"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This package builds meshes (uniform hexahedra, box-clipped jittered-BCC
Voronoi polyhedra) and fields (volume fractions by sub-sampling, temperature
profiles, boundary temperatures).  It contains none of the reconstruction,
gradient or mass-transfer arithmetic: those live, independently, in
``oracle/`` (the CPU checker) and in the HIP library.
"""
from .meshes import Mesh, hex_mesh, voronoi_box_mesh, voronoi_pipe_mesh  # noqa: F401
from . import fields, workloads  # noqa: F401
