"""Pins of the oracle's Gym-style tasks (Sec. III): the reference curves against
their defining identities and a finite-difference tangent, the ZYX Euler angles
against quaternions built from elementary rotations, the observation of Eq. (2)
and the error of Eq. (4) on states placed exactly on the reference, and the
episode bookkeeping (counter, termination, truncation, automatic reset) against
a plain Python loop over single control steps.  CPU only.
"""
import math

import numpy as np
import pytest

from workloads import (BLUEROV2, BLUEROV2_HEAVY, vehicle_variant, initial_state, actions,
                       param_multipliers, env_classes)

CURVES = {"circle": 1, "helix": 2, "lemniscate": 3}


def _task(kind, **kw):
    t = {"task": kind, "lookahead": 3, "radius": 1.5, "omega": 0.4, "climb_rate": 0.05,
         "lookahead_dt": 0.0, "episode_steps": 1 << 30, "max_error": 0.0}
    t.update(kw)
    return t


def _qaxis(axis, angle):
    q = np.zeros(4)
    q[0] = math.cos(angle / 2)
    q[1 + axis] = math.sin(angle / 2)
    return q


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _q_zyx(roll, pitch, yaw):
    """q = q_z(yaw) (x) q_y(pitch) (x) q_x(roll): R = Rz Ry Rx."""
    return _qmul(_qmul(_qaxis(2, yaw), _qaxis(1, pitch)), _qaxis(0, roll))


def _angdiff(a, b):
    return abs(math.remainder(a - b, 2 * math.pi))


@pytest.mark.parametrize("omega", [0.4, -0.7])
@pytest.mark.parametrize("kind", ["circle", "helix", "lemniscate"])
def test_reference_curve_identities_and_tangent(oracle, kind, omega):
    tk = _task(kind, omega=omega)
    c = np.array([0.3, -1.2, 2.0])
    R = tk["radius"]
    for t in np.linspace(0.0, 20.0, 37):
        pr, psi = oracle.task_reference(tk, c, 0.25, 0.0, t)
        d = pr - c
        if kind in ("circle", "helix"):
            assert math.hypot(d[0], d[1]) == pytest.approx(R, abs=1e-12)
            assert d[2] == pytest.approx(tk["climb_rate"] * t if kind == "helix" else 0.0,
                                         abs=1e-12)
        else:
            r2 = d[0] ** 2 + d[1] ** 2
            assert r2 * r2 == pytest.approx(R * R * (d[0] ** 2 - d[1] ** 2), abs=1e-12)
            assert d[2] == 0.0
        h = 1e-6
        p1, _ = oracle.task_reference(tk, c, 0.25, 0.0, t + h)
        p0, _ = oracle.task_reference(tk, c, 0.25, 0.0, t - h)
        v = (p1 - p0) / (2 * h)
        assert _angdiff(psi, math.atan2(v[1], v[0])) < 1e-6


def test_lemniscate_landmarks(oracle):
    """Bernoulli's lemniscate through the centre at s = pi/2 and at +-R on the x axis."""
    tk = _task("lemniscate", omega=1.0)
    c = np.zeros(3)
    p, _ = oracle.task_reference(tk, c, 0.0, 0.0, 0.0)
    np.testing.assert_allclose(p, [1.5, 0, 0], atol=1e-15)
    p, _ = oracle.task_reference(tk, c, 0.0, 0.0, math.pi / 2)
    np.testing.assert_allclose(p, [0, 0, 0], atol=1e-15)
    p, _ = oracle.task_reference(tk, c, 0.0, 0.0, math.pi)
    np.testing.assert_allclose(p, [-1.5, 0, 0], atol=1e-15)


def test_station_reference_is_the_target(oracle):
    p, psi = oracle.task_reference(_task("station"), [1.0, 2.0, 3.0], 0.7, -2.5, 12.0)
    np.testing.assert_array_equal(p, [1.0, 2.0, 3.0])
    assert psi == -2.5


def test_euler_zyx_inverts_elementary_rotations(oracle):
    rng = np.random.default_rng(11)
    for _ in range(200):
        roll, yaw = rng.uniform(-math.pi + 1e-3, math.pi - 1e-3, 2)
        pitch = rng.uniform(-math.pi / 2 + 1e-3, math.pi / 2 - 1e-3)
        got = oracle.euler_zyx(_q_zyx(roll, pitch, yaw))
        np.testing.assert_allclose(got, [roll, pitch, yaw], atol=1e-9)


def _on_reference_state(oracle, tk, c, ph, yaw0, t, D=13):
    """A state at the reference point and attitude (level, reference heading) of time t."""
    pr, psi = oracle.task_reference(tk, c, ph, yaw0, t)
    x = np.zeros(D)
    x[:3] = pr
    x[3:7] = _q_zyx(0.0, 0.0, psi)
    x[7:13] = np.arange(1, 7) * 0.1
    return x


@pytest.mark.parametrize("kind", ["station", "circle", "helix", "lemniscate"])
def test_observation_on_the_reference(oracle, kind):
    """A state on the first look-ahead point (tracking) or on the target (station keeping)
    observes a zero first pose error; nu is copied; the width is 12 or 6 m + 6; the later
    look-ahead blocks hold p - p_r(t + i dl) exactly."""
    tk = _task(kind)
    dtc = 0.02
    c, ph, yw, k = np.array([0.5, -0.5, 1.0]), 0.3, 0.8, 7
    t_first = k * dtc if kind == "station" else (k + 1) * dtc
    x = _on_reference_state(oracle, tk, c, ph, yw, t_first)
    obs = oracle.task_observe(tk, x[:, None], c[:, None], [ph], [yw], [k], dtc)[:, 0]
    assert len(obs) == (12 if kind == "station" else 6 * tk["lookahead"] + 6)
    np.testing.assert_allclose(obs[:6], 0.0, atol=1e-12)
    np.testing.assert_array_equal(obs[-6:], x[7:13])
    if kind != "station":
        for i in range(2, tk["lookahead"] + 1):
            pr, psi = oracle.task_reference(tk, c, ph, yw, (k + i) * dtc)
            np.testing.assert_allclose(obs[6 * (i - 1):6 * (i - 1) + 3], x[:3] - pr, atol=1e-14)
            ref_psi = oracle.task_reference(tk, c, ph, yw, t_first)[1]
            assert _angdiff(obs[6 * (i - 1) + 5], ref_psi - psi) < 1e-12


def test_observation_wraps_the_heading_error(oracle):
    """Heading 3.0 against target yaw -3.0: the error is 6 - 2 pi, not 6."""
    tk = _task("station")
    x = np.zeros(13)
    x[3:7] = _q_zyx(0.0, 0.0, 3.0)
    obs = oracle.task_observe(tk, x[:, None], np.zeros((3, 1)), [0.0], [-3.0], [0], 0.02)[:, 0]
    assert obs[5] == pytest.approx(6.0 - 2 * math.pi, abs=1e-12)
    assert -math.pi < obs[5] <= math.pi


def _python_episodes(oracle, classes, cls, tk, x0, act, S, dt, center, phase, yaw, mult,
                     reset_state, reset_mult, D):
    """The bookkeeping written as a plain loop over single control steps of the oracle."""
    T, _, E = act.shape
    dtc = S * dt
    x = x0.astype(np.float64).copy()
    m = mult.astype(np.float64).copy()
    k = np.zeros(E, np.int64)
    obs = [oracle.task_observe(tk, x, center, phase, yaw, k, dtc)]
    errs, dones = [], []
    for t in range(T):
        x = oracle.rollout(classes, x, act[t:t + 1], S, dt, env_class=cls, mult=m)["x"]
        k += 1
        err = np.zeros(E)
        done = np.zeros(E, np.int32)
        for e in range(E):
            pr, _ = oracle.task_reference(tk, center[:, e], phase[e], yaw[e], k[e] * dtc)
            err[e] = np.linalg.norm(x[:3, e] - pr)
            finite = np.all(np.isfinite(x[:, e]))
            if not finite or (tk["max_error"] > 0 and not err[e] <= tk["max_error"]):
                done[e] = 1
            elif k[e] >= tk["episode_steps"]:
                done[e] = 2
            if done[e]:
                x[:, e] = reset_state[:, e]
                m[:, e] = reset_mult[:, e]
                k[e] = 0
        errs.append(err)
        dones.append(done)
        obs.append(oracle.task_observe(tk, x, center, phase, yaw, k, dtc))
    return np.array(obs), np.array(errs), np.array(dones), x, k


@pytest.mark.parametrize("kind", ["station", "circle", "helix", "lemniscate"])
def test_episode_bookkeeping_against_a_plain_loop(oracle, kind):
    """Counter, terminated / truncated flags, automatic reset of state and parameters and
    the post-reset observation equal a plain loop over single oracle control steps."""
    E, T, S, dt, D = 24, 11, 4, 0.005, 21
    classes = [vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05),
               vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)]
    cls = env_classes(E, "halves")
    x0 = initial_state(E, D, 801)
    x0[19:, cls == 0] = 0
    act = actions(T, 8, E, 802)
    mult = param_multipliers(E, 0.2, 803)
    rng = np.random.default_rng(804)
    center = rng.normal(0, 0.3, (3, E))
    phase = rng.uniform(0, 2 * math.pi, E)
    yaw = rng.uniform(-math.pi, math.pi, E)
    reset_state = initial_state(E, D, 805)
    reset_state[19:, cls == 0] = 0
    reset_mult = param_multipliers(E, 0.2, 806)
    # episode length 4; an error bound that some envs cross (the 80th percentile of the
    # errors of a run without one)
    free = oracle.task_rollout(classes, _task(kind, episode_steps=4), x0, act, S, dt, center,
                               phase, yaw, env_class=cls, mult=mult, reset_state=reset_state,
                               reset_mult=reset_mult)
    tk = _task(kind, episode_steps=4, max_error=float(np.quantile(free["err"], 0.8)))
    got = oracle.task_rollout(classes, tk, x0, act, S, dt, center, phase, yaw, env_class=cls,
                              mult=mult, reset_state=reset_state, reset_mult=reset_mult)
    obs, err, done, xT, kT = _python_episodes(oracle, classes, cls, tk, x0, act, S, dt, center,
                                              phase, yaw, mult, reset_state, reset_mult, D)
    np.testing.assert_array_equal(got["done"], done)
    assert (done == 1).any() and (done == 2).any()
    np.testing.assert_allclose(got["err"], err, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(got["obs"], obs, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(got["x"], xT, rtol=1e-13, atol=1e-13)
    np.testing.assert_array_equal(got["k"], kT)


def test_nonfinite_env_terminates_and_restarts(oracle):
    """An env whose mass matrix is not positive definite goes non-finite, is reported as
    terminated and restarts from its reset state and parameters."""
    E, T, S, dt = 3, 2, 1, 0.01
    x0 = initial_state(E, 13, 811)
    act = actions(T, 6, E, 812)
    mult = np.ones((23, E))
    mult[0, 1] = -50.0          # negative mass: M is not positive definite
    reset_state = initial_state(E, 13, 813)
    tk = _task("station", episode_steps=100)
    got = oracle.task_rollout(BLUEROV2, tk, x0, act, S, dt, np.zeros((3, E)), np.zeros(E),
                              mult=mult, reset_state=reset_state, reset_mult=np.ones((23, E)))
    assert got["done"][0, 1] == 1 and got["done"][0, 0] == 0 and got["done"][0, 2] == 0
    assert got["done"][1, 1] == 0 and np.all(np.isfinite(got["x"]))
    assert got["k"][1] == 1 and got["k"][0] == 2
