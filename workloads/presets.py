"""Vehicle presets: plain data for the BlueROV2 and BlueROV2 Heavy classes.

The paper names the two vehicles (Sec. II, the UUV dynamics module; Sec. III,
the four tasks use the Heavy) but prints no parameter values.  Only the
BlueROV2 dry mass, 11.5 kg, is fixed by the workload definition; every other
number below is an illustrative round value of BlueROV2 magnitude, kept here
as data so it can be swapped without touching either implementation.

Units are SI.  Frames: body frame forward-right-down, origin (CO) at the centre
of buoyancy; world frame north-east-down.

Each preset is a dict with:
  mass, inertia (diag of I_g about the CG), r_g, r_b (CG / CB w.r.t. the CO),
  added_mass, d_lin, d_quad (diagonals, 6 each), buoyancy (N),
  thr_pos (n x 3), thr_dir (n x 3, unit direction of positive thrust),
  f_max (N), thr_map (0 linear, 1 quadratic), thr_tau (s, 0 = no lag).

Randomisable per-env parameters (order of the [23][E] multiplier arrays):
  m, Ixx, Iyy, Izz, M_A(6), D_L(6), D_Q(6), B.
"""
import copy
import math

#: gravitational acceleration used to turn mass into weight (m/s^2)
G0 = 9.81

PARAM_NAMES = (["m", "Ixx", "Iyy", "Izz"]
               + [f"MA{i}" for i in range(6)]
               + [f"DL{i}" for i in range(6)]
               + [f"DQ{i}" for i in range(6)]
               + ["B"])
assert len(PARAM_NAMES) == 23

_C = 1.0 / math.sqrt(2.0)

# four horizontal thrusters at 45 degrees, shared by both layouts
_HORIZ_POS = [(0.15, 0.10, 0.05), (0.15, -0.10, 0.05),
              (-0.15, 0.10, 0.05), (-0.15, -0.10, 0.05)]
_HORIZ_DIR = [(_C, -_C, 0.0), (_C, _C, 0.0), (_C, _C, 0.0), (_C, -_C, 0.0)]
# vertical thrusters push up (-z in a z-down body frame) for a positive command
_UP = (0.0, 0.0, -1.0)

BLUEROV2 = {
    "name": "BlueROV2",
    "mass": 11.5,
    "inertia": [0.16, 0.16, 0.16],
    "r_g": [0.0, 0.0, 0.02],
    "r_b": [0.0, 0.0, 0.0],
    "added_mass": [5.5, 12.7, 14.6, 0.12, 0.12, 0.12],
    "d_lin": [4.0, 6.0, 5.0, 0.07, 0.07, 0.07],
    "d_quad": [18.0, 21.0, 37.0, 0.45, 0.45, 0.45],
    "buoyancy": 11.5 * G0,          # neutrally buoyant at nominal mass
    "thr_pos": _HORIZ_POS + [(0.0, 0.11, -0.02), (0.0, -0.11, -0.02)],
    "thr_dir": _HORIZ_DIR + [_UP, _UP],
    "f_max": 40.0,
    "thr_map": 0,
    "thr_tau": 0.0,
}

BLUEROV2_HEAVY = {
    "name": "BlueROV2Heavy",
    "mass": 13.5,
    "inertia": [0.26, 0.23, 0.37],
    "r_g": [0.0, 0.0, 0.02],
    "r_b": [0.0, 0.0, 0.0],
    "added_mass": [5.5, 12.7, 14.6, 0.12, 0.12, 0.12],
    "d_lin": [4.0, 6.0, 5.0, 0.07, 0.07, 0.07],
    "d_quad": [18.0, 21.0, 37.0, 0.45, 0.45, 0.45],
    "buoyancy": 13.5 * G0,
    "thr_pos": _HORIZ_POS + [(0.12, 0.22, -0.02), (0.12, -0.22, -0.02),
                             (-0.12, 0.22, -0.02), (-0.12, -0.22, -0.02)],
    "thr_dir": _HORIZ_DIR + [_UP, _UP, _UP, _UP],
    "f_max": 40.0,
    "thr_map": 0,
    "thr_tau": 0.0,
}


def vehicle_variant(base, **overrides):
    """Deep copy of a preset with some fields replaced (e.g. thr_map=1, thr_tau=0.05)."""
    v = copy.deepcopy(base)
    for k, val in overrides.items():
        if k not in v:
            raise KeyError(k)
        v[k] = val
    return v
