"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package builds analytic street-block scenes (ground plane, walls, boxes), samples
surfel maps from virtual LiDAR scans of them, writes the spinning-LiDAR beam tables and
raycasts exact target range images.  It holds none of the surfel rendering arithmetic:
the renderer under test and the oracle both only consume what it produces.
"""
from .scene import (  # noqa: F401
    WORKLOADS,
    Scene,
    beam_tables,
    make_pose,
    make_scene,
    make_workload,
    quat_from_frame,
    ray_dirs_f64,
    raycast,
    sample_surfels,
    synthetic_frame,
    synthetic_scan,
    targets_for_pose,
)
