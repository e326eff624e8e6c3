"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the oracle.

This package holds vehicle presets (plain data) and seeded random draws
(parameter multipliers, initial states, actions, waypoints).  It contains none
of the arithmetic of the dynamics: no mass matrix, no allocation matrix, no
right-hand side, no integrator.  Both the FP64 oracle and the GPU library build
those from the raw numbers given here, each on its own.
"""
from .presets import BLUEROV2, BLUEROV2_HEAVY, PARAM_NAMES, G0, vehicle_variant
from .gen import (CONFIGS, WorkloadConfig, rng_for, param_multipliers, initial_state,
                  actions, action_frames, circle_waypoints, env_classes, euler_to_quat,
                  random_states)

__all__ = [
    "BLUEROV2", "BLUEROV2_HEAVY", "PARAM_NAMES", "G0", "vehicle_variant",
    "CONFIGS", "WorkloadConfig", "rng_for", "param_multipliers", "initial_state",
    "actions", "action_frames", "circle_waypoints", "env_classes", "euler_to_quat", "random_states",
]
