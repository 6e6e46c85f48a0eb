"""Seeded synthetic inputs (meshes, scenes, candidate poses).

This package holds no part of the scoring method: it builds procedural
meshes, places them on a table, simulates the RGB-D sensor by ray casting and
draws candidate poses.  Both the GPU path and the CPU oracle consume what it
produces.
"""
from .meshes import Mesh, make_shape, SHAPES  # noqa: F401
from .scenes import Workload, Scene, ObjectQuery, make_config, camera_rig  # noqa: F401
