"""Seeded synthetic inputs (FP32 arrays, SoA layout [component][env]).

Every array is drawn in FP64 by numpy's PCG64 and rounded once to FP32; the
oracle and the GPU library then consume the *same* FP32 values (the oracle
widens them to FP64 exactly).  Seeds follow ``1000 * config + stream`` with
stream 1 = parameter multipliers, 2 = initial state, 3 = actions,
4 = waypoints, 5 = env classes.

The workload shapes mirror the paper's setting (Sec. III: BlueROV2-class
vehicles, many parallel environments, per-env domain randomisation); the paper
gives no sizes, so the five configurations below are this library's own
benchmark definitions.
"""
from dataclasses import dataclass, field
import math

import numpy as np

STREAM_PARAMS, STREAM_INIT, STREAM_ACTIONS, STREAM_WAYPOINTS, STREAM_CLASSES = 1, 2, 3, 4, 5


@dataclass(frozen=True)
class WorkloadConfig:
    key: str
    seed_base: int
    n_envs: int
    classes: str          # "bluerov2", "heavy", "halves" (first half BlueROV2) or "bernoulli"
    rho: float            # +-rho uniform parameter randomisation (0 = nominal)
    thr_map: int          # 0 linear, 1 quadratic
    thr_tau: float        # first-order thruster lag (s), 0 = none
    n_ctrl: int           # control steps
    substeps: int         # RK4 substeps per control step
    dt_sub: float         # substep (s)
    extra: dict = field(default_factory=dict)


CONFIGS = {
    "c1": WorkloadConfig("c1", 1000, 64, "bluerov2", 0.0, 0, 0.0, 1000, 1, 0.01),
    "c2": WorkloadConfig("c2", 2000, 4096, "heavy", 0.2, 1, 0.05, 1000, 4, 0.005),
    "c3": WorkloadConfig("c3", 3000, 1 << 20, "halves", 0.2, 1, 0.05, 200, 16, 0.005),
    "c4": WorkloadConfig("c4", 4000, 8192, "bluerov2", 0.0, 0, 0.0, 64, 1, 0.01,
                         {"ckpt_every": 8, "lam": 1.0, "omega": 0.5}),
    "c5": WorkloadConfig("c5", 5000, 0, "bernoulli", 0.2, 1, 0.05, 64, 4, 0.005,
                         {"clients": 32, "rate": 2000.0, "env_lo": 16, "env_hi": 65536}),
}


def rng_for(seed_base, stream):
    return np.random.Generator(np.random.PCG64(seed_base + stream))


def param_multipliers(n_envs, rho, seed):
    """[23][E] FP32 multipliers, independent U[1-rho, 1+rho] per element."""
    if rho == 0.0:
        return np.ones((23, n_envs), dtype=np.float32)
    r = np.random.Generator(np.random.PCG64(seed))
    return r.uniform(1.0 - rho, 1.0 + rho, size=(23, n_envs)).astype(np.float32)


def euler_to_quat(phi, theta, psi):
    """ZYX Euler angles -> unit quaternion (w, x, y, z), body-to-NED."""
    cr, sr = np.cos(phi / 2), np.sin(phi / 2)
    cp, sp = np.cos(theta / 2), np.sin(theta / 2)
    cy, sy = np.cos(psi / 2), np.sin(psi / 2)
    w = cr * cp * cy + sr * sp * sy
    x = sr * cp * cy - cr * sp * sy
    y = cr * sp * cy + sr * cp * sy
    z = cr * cp * sy - sr * sp * cy
    return np.stack([w, x, y, z])


def initial_state(n_envs, state_dim, seed, sigma=0.1):
    """[D][E] FP32: position, ZYX Euler angles and body velocities ~ N(0, sigma^2);
    attitude stored as a quaternion; thruster states (rows 13..) start at zero."""
    r = np.random.Generator(np.random.PCG64(seed))
    z = r.normal(0.0, sigma, size=(12, n_envs))
    x = np.zeros((state_dim, n_envs), dtype=np.float64)
    x[0:3] = z[0:3]
    x[3:7] = euler_to_quat(z[3], z[4], z[5])
    x[7:13] = z[6:12]
    return x.astype(np.float32)


def random_states(n_envs, state_dim, seed, f_max=40.0):
    """[D][E] FP32 states spread over the operating envelope (for one-step checks):
    p ~ U[-10,10] m, uniformly random attitude, v ~ U[-1.5,1.5] m/s,
    omega ~ U[-2,2] rad/s, thruster states ~ U[-f_max, f_max]."""
    r = np.random.Generator(np.random.PCG64(seed))
    x = np.zeros((state_dim, n_envs), dtype=np.float64)
    x[0:3] = r.uniform(-10, 10, size=(3, n_envs))
    q = r.normal(size=(4, n_envs))
    x[3:7] = q / np.linalg.norm(q, axis=0)
    x[7:10] = r.uniform(-1.5, 1.5, size=(3, n_envs))
    x[10:13] = r.uniform(-2.0, 2.0, size=(3, n_envs))
    if state_dim > 13:
        x[13:] = r.uniform(-f_max, f_max, size=(state_dim - 13, n_envs))
    return x.astype(np.float32)


def actions(n_ctrl, n_max, n_envs, seed):
    """[T][N_max][E] FP32 throttles, i.i.d. U[-1, 1)."""
    r = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n_ctrl, n_max, n_envs), dtype=np.float32)
    for t in range(n_ctrl):
        u = r.random((n_max, n_envs), dtype=np.float32)
        out[t] = u * np.float32(2.0) - np.float32(1.0)
    return out


def action_frames(n_ctrl, n_max, n_envs, seed):
    """Same values as :func:`actions`, yielded one [N_max][E] frame at a time."""
    r = np.random.Generator(np.random.PCG64(seed))
    for _ in range(n_ctrl):
        u = r.random((n_max, n_envs), dtype=np.float32)
        yield u * np.float32(2.0) - np.float32(1.0)


def circle_waypoints(n_ctrl, n_envs, dt, seed, omega=0.5):
    """Circle-tracking references (the paper's circle task, Sec. III), one per control step
    t = 1..T: centre c ~ N(0, 0.1^2), radius ~ U[0.5, 1.5], phase ~ U[0, 2 pi),
    angular rate omega; attitude reference is yaw-only, tangent to the circle.
    Returns (p_ref [T][3][E], q_ref [T][4][E]) FP32."""
    r = np.random.Generator(np.random.PCG64(seed))
    c = r.normal(0.0, 0.1, size=(3, n_envs))
    rad = r.uniform(0.5, 1.5, size=n_envs)
    ph = r.uniform(0.0, 2 * math.pi, size=n_envs)
    t = (np.arange(1, n_ctrl + 1, dtype=np.float64) * dt)[:, None]
    ang = omega * t + ph[None, :]
    p = np.empty((n_ctrl, 3, n_envs))
    p[:, 0] = c[0] + rad * np.cos(ang)
    p[:, 1] = c[1] + rad * np.sin(ang)
    p[:, 2] = c[2]
    yaw = ang + math.pi / 2
    q = np.zeros((n_ctrl, 4, n_envs))
    q[:, 0] = np.cos(yaw / 2)
    q[:, 3] = np.sin(yaw / 2)
    return p.astype(np.float32), q.astype(np.float32)


def env_classes(n_envs, kind, seed=None):
    """[E] int32 class index: 0 = BlueROV2, 1 = BlueROV2 Heavy."""
    if kind == "bluerov2":
        return np.zeros(n_envs, dtype=np.int32)
    if kind == "heavy":
        return np.ones(n_envs, dtype=np.int32)
    if kind == "halves":
        c = np.zeros(n_envs, dtype=np.int32)
        c[n_envs // 2:] = 1
        return c
    if kind == "bernoulli":
        r = np.random.Generator(np.random.PCG64(seed))
        return (r.random(n_envs) < 0.5).astype(np.int32)
    raise ValueError(kind)


def splitmix64_throttles(seed, n_steps, n_max, n_envs):
    """[T][N_max][E] FP32 throttles of a serving request whose actions are generated from a
    seed: throttle i of env e at control step t is 2 u - 1 with u = (z >> 40) 2^-24, z the
    SplitMix64 output number (t N_max + i) E + e of the generator seeded with `seed`
    (Steele, Lea and Flood, OOPSLA 2014: output k = mix(seed + (k + 1) gamma))."""
    gamma = np.uint64(0x9E3779B97F4A7C15)
    k = np.arange(n_steps * n_max * n_envs, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (k + np.uint64(1)) * gamma
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)
    return (u * np.float32(2.0) - np.float32(1.0)).reshape(n_steps, n_max, n_envs)
