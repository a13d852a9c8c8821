"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only draws RTE parameter fields (extinction, albedo, emission per
cell) from fixed seeds.  It contains none of the P_N method's arithmetic, so
both sides of a parity test can consume exactly the same FP32 inputs.
"""
from .media import (  # noqa: F401
    value_noise, fbm, gaussian_blob, Medium,
    config_p1_homogeneous, config_p3_fbm, config_p3_train, config_p5_nebula, config_batch,
    config_uniform_periodic, config_small, checkerboard_blocks, config_checkerboard, config_point_source,
)
