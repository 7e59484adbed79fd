"""Seeded synthetic inputs for the AERO-MPPI planning step.

This package only builds inputs: obstacle scenes, simulated LiDAR sweeps,
states, goals and the parameter values of the paper's Table I.  It holds
none of the planner's arithmetic, so both the HIP path and the CPU oracle
can consume it without sharing code.
"""
from .scenes import (  # noqa: F401
    Cylinder, Box, lidar_sweep, forest_scene, verticals_scene, incline_scene,
    cylinders_surface_points, record_frame,
)
from .configs import (  # noqa: F401
    table1_params, make_plain_problem, make_ensemble_problem,
    make_batched_problems, make_loop_step, make_paper_point_problem, split_instances, hover_controls,
)
