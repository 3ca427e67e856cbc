"""FP64 CPU oracle for one CE-MPPI replan (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does, and this package
imports nothing from it.  The arithmetic lives in ``cemppi_oracle.c``;
this module only builds that file and marshals numpy arrays through ctypes.
"""
from .oracle import (  # noqa: F401
    build,
    load,
    philox4x32_10,
    noise_words,
    rollout_noise,
    uniform,
    box_muller,
    unicycle_step,
    arm_frames,
    arm_spheres,
    simulate,
    rotvec_quat,
    rot_quat,
    quat_angle,
    closest_obstacle,
    closest_obstacle_margin,
    select_cluster,
    obstacle_velocity,
    dbscan,
    weighted_update,
    replan,
    noise_blocks,
    UNICYCLE,
    ARM6,
    FLAG_POSE_COST,
    FLAG_OBS_CONST_VEL,
    ST_FALLBACK,
    ST_ALL_COLLIDE,
    ST_NO_CLUSTER,
    ST_DYN_STATIC,
    ST_NONFINITE,
)
