"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package draws point clouds, grids, robot descriptions, trajectories and
submap batches.  It holds none of the method's arithmetic: no rasterisation,
no slicing, no cost formula.  Both the HIP path and the CPU oracle consume
what it produces; neither is imported here.
"""
from .synth import (  # noqa: F401
    Scene,
    config0_scene,
    multistorey_scene,
    config1_scene,
    dense_surface_scene,
    random_walks,
    submap_batch,
    robot_profiles,
    plan_layers,
    plan_serpentine,
    plan_building,
    traj_problems,
    ROBOT_CONFIG0,
    ROBOT_TABLE1,
)
