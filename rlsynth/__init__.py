"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds scene generation (rooms, poses, rendered RGB-D frames), the random
forest structure and parameter presets.  Nothing in here computes any step
of the relocaliser.
"""
from . import forest, presets, scene, workloads  # noqa: F401
from .forest import NODE_DTYPE, make_forest  # noqa: F401
from .scene import intrinsics, make_room, pose_error, render  # noqa: F401
