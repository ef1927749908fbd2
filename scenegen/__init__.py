"""Seeded synthetic scenes and cameras for ray-based Gaussian splatting.

This package only draws random numbers and lays them out; it holds none of the
renderer's arithmetic.  Both the CPU oracle (tests) and the HIP path consume
what it produces, so it must stay free of either side's code.
"""
from .scenes import (  # noqa: F401
    WORKLOADS,
    look_at,
    pinhole,
    make_scene,
    make_cameras,
    make_workload,
    tiny_scene,
    thin_structure_scene,
    wall_scene,
    approach_cameras,
    default_options,
    fd_subcase,
)
