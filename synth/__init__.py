"""Seeded synthetic LiDAR inputs (points and poses) for tests and benchmarks.

This package produces inputs only. It contains none of the mapping method's
arithmetic (no transform into the map frame, no voxelisation, no binning, no
kernels): both the HIP library and the CPU oracle consume what it writes.
"""
from .scene import (  # noqa: F401
    CONFIGS,
    Scene,
    SensorModel,
    config_grid,
    make_scene,
    make_trajectory,
    cast_rays,
    sensor_directions,
    synth_scan,
    config_scans,
    pose_from_xyz_rpy,
    config_poses,
    random_cloud,
    random_pose,
    KERNEL_DEFAULTS,
)
