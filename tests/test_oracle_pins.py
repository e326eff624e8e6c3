"""Pins of the FP64 oracle against what the mechanics fixes, independent of the
oracle's own formulas: textbook closed forms (Fossen's Euler-angle restoring
vector, the parallel-axis theorem, elementary rotation matrices), conservation
laws, analytic steady states, the exact RK4 amplification factor of linear
modes, the RK4 global order, and finite differences for the dual-number
gradient.  A dropped term, a sign error or a transposed operand in the oracle
fails at least one of these.  CPU only.
"""
import math

import numpy as np
import pytest

from workloads import (BLUEROV2, BLUEROV2_HEAVY, G0, CONFIGS, vehicle_variant, euler_to_quat,
                       initial_state, actions, param_multipliers, circle_waypoints)


def _rest_state(D=13):
    x = np.zeros(D)
    x[3] = 1.0
    return x


def _rk4_factor(z):
    """Amplification of classical RK4 on y' = lambda y, z = lambda * dt."""
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


# --------------------------------------------------------------------------------------
# thruster allocation
# --------------------------------------------------------------------------------------

def test_allocation_columns_hand_computed(oracle):
    c = 1 / math.sqrt(2)
    B = oracle.alloc(BLUEROV2)
    # thruster 1: r = (0.15, 0.10, 0.05), d = (c, -c, 0): r x d = (0.05c, 0.05c, -0.25c)
    np.testing.assert_allclose(B[:, 0], [c, -c, 0, 0.05 * c, 0.05 * c, -0.25 * c], atol=1e-15)
    # thruster 4: r = (-0.15, -0.10, 0.05), d = (c, -c, 0): r x d = (0.05c, 0.05c, 0.25c)
    np.testing.assert_allclose(B[:, 3], [c, -c, 0, 0.05 * c, 0.05 * c, 0.25 * c], atol=1e-15)
    # vertical at (0, 0.11, -0.02), d = (0, 0, -1): r x d = (-0.11, 0, 0)
    np.testing.assert_allclose(B[:, 4], [0, 0, -1, -0.11, 0, 0], atol=1e-15)
    Bh = oracle.alloc(BLUEROV2_HEAVY)
    # Heavy vertical at (-0.12, -0.22, -0.02): r x d = (0.22, -0.12, 0)
    np.testing.assert_allclose(Bh[:, 7], [0, 0, -1, 0.22, -0.12, 0], atol=1e-15)


def test_allocation_ranks(oracle):
    # BlueROV2 cannot pitch independently (its verticals sit on the y axis): rank 5
    assert np.linalg.matrix_rank(oracle.alloc(BLUEROV2)) == 5
    assert np.linalg.matrix_rank(oracle.alloc(BLUEROV2_HEAVY)) == 6


# --------------------------------------------------------------------------------------
# mass matrix
# --------------------------------------------------------------------------------------

def _parallel_axis_mass(preset, mult):
    """Textbook construction: I_O = I_G + m (|r|^2 I - r r^T), coupling m S(r_g)."""
    m = preset["mass"] * mult[0]
    Ig = np.diag(np.array(preset["inertia"]) * mult[1:4])
    r = np.array(preset["r_g"], dtype=float)
    Io = Ig + m * (r @ r * np.eye(3) - np.outer(r, r))
    Sr = np.array([[0, -r[2], r[1]], [r[2], 0, -r[0]], [-r[1], r[0], 0]])
    M = np.zeros((6, 6))
    M[:3, :3] = m * np.eye(3)
    M[:3, 3:] = (m * Sr).T          # = -m S(r_g)
    M[3:, :3] = m * Sr
    M[3:, 3:] = Io
    return M + np.diag(np.array(preset["added_mass"]) * mult[4:10])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_mass_matrix_parallel_axis_and_spd(oracle, seed):
    rng = np.random.default_rng(seed)
    v = vehicle_variant(BLUEROV2_HEAVY, r_g=list(rng.uniform(-0.05, 0.05, 3)))
    mult = rng.uniform(0.8, 1.2, 23)
    M = oracle.mass_matrix(v, mult)
    np.testing.assert_allclose(M, _parallel_axis_mass(v, mult), rtol=0, atol=1e-14)
    np.testing.assert_array_equal(M, M.T)
    assert np.linalg.eigvalsh(M).min() > 0


def test_mass_matrix_structured_entries(oracle):
    m, zg = 11.5, 0.02
    M = oracle.mass_matrix(BLUEROV2)
    assert M[0, 4] == pytest.approx(m * zg, abs=1e-15)     # surge-pitch
    assert M[1, 3] == pytest.approx(-m * zg, abs=1e-15)    # sway-roll
    assert M[3, 3] == pytest.approx(0.16 + m * zg * zg + 0.12, abs=1e-15)
    assert M[5, 5] == pytest.approx(0.16 + 0.12, abs=1e-15)
    assert M[0, 0] == pytest.approx(m + 5.5, abs=1e-15)
    # the (u, q) block is positive definite in closed form
    det = (m + 5.5) * (0.16 + m * zg * zg + 0.12) - (m * zg) ** 2
    assert det > 0
    assert np.linalg.eigvalsh(M).min() == pytest.approx(0.28, abs=1e-3)


# --------------------------------------------------------------------------------------
# Coriolis / centripetal
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_coriolis_skew_and_kirchhoff_form(oracle, seed):
    rng = np.random.default_rng(100 + seed)
    v = vehicle_variant(BLUEROV2, r_g=list(rng.uniform(-0.05, 0.05, 3)))
    M = oracle.mass_matrix(v, rng.uniform(0.8, 1.2, 23))
    nu = rng.normal(size=6)
    C = oracle.coriolis_matrix(M, nu)
    np.testing.assert_array_equal(C + C.T, np.zeros((6, 6)))
    assert abs(nu @ C @ nu) <= 5e-15 * (1 + np.abs(nu).max() ** 2 * np.abs(M).max())
    # Kirchhoff's equations: C(nu) nu = [w x a ; v x a + w x b],  [a; b] = M nu
    ab = M @ nu
    a, b = ab[:3], ab[3:]
    vv, w = nu[:3], nu[3:]
    kir = np.concatenate([np.cross(w, a), np.cross(vv, a) + np.cross(w, b)])
    np.testing.assert_allclose(C @ nu, kir, atol=1e-14)


# --------------------------------------------------------------------------------------
# rotation and restoring forces
# --------------------------------------------------------------------------------------

def _rzyx(phi, th, psi):
    cx, sx, cy, sy, cz, sz = (math.cos(phi), math.sin(phi), math.cos(th), math.sin(th),
                              math.cos(psi), math.sin(psi))
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


@pytest.mark.parametrize("seed", range(5))
def test_rotation_equals_zyx_euler(oracle, seed):
    rng = np.random.default_rng(200 + seed)
    phi, th, psi = rng.uniform(-1.4, 1.4, 3)
    q = euler_to_quat(np.array(phi), np.array(th), np.array(psi))
    np.testing.assert_allclose(oracle.rotation(q), _rzyx(phi, th, psi), atol=1e-14)


def test_restoring_level_is_pure_heave(oracle):
    mult = np.ones(23)
    mult[22] = 0.9                      # B = 0.9 W: net weight 0.1 W pushes down (+z)
    W = 11.5 * G0
    for psi in [0.0, 0.7, -2.5, 3.1]:
        q = euler_to_quat(np.array(0.0), np.array(0.0), np.array(psi))
        g = oracle.restoring(BLUEROV2, q, mult)
        np.testing.assert_allclose(g, [0, 0, -(W - 0.9 * W), 0, 0, 0], atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_restoring_matches_fossen_euler_form(oracle, seed):
    """g(eta) against the textbook Euler-angle expression for W != B, r_g and r_b general."""
    rng = np.random.default_rng(300 + seed)
    rg = rng.uniform(-0.03, 0.03, 3)
    rb = rng.uniform(-0.03, 0.03, 3)
    v = vehicle_variant(BLUEROV2_HEAVY, r_g=list(rg), r_b=list(rb))
    mult = rng.uniform(0.8, 1.2, 23)
    W = v["mass"] * mult[0] * G0
    B = v["buoyancy"] * mult[22]
    phi, th, psi = rng.uniform(-1.3, 1.3, 3)
    q = euler_to_quat(np.array(phi), np.array(th), np.array(psi))
    g = oracle.restoring(v, q, mult)
    sph, cph, sth, cth = math.sin(phi), math.cos(phi), math.sin(th), math.cos(th)
    xg, yg, zg = rg
    xb, yb, zb = rb
    expect = [
        (W - B) * sth,
        -(W - B) * cth * sph,
        -(W - B) * cth * cph,
        -(yg * W - yb * B) * cth * cph + (zg * W - zb * B) * cth * sph,
        (zg * W - zb * B) * sth + (xg * W - xb * B) * cth * cph,
        -(xg * W - xb * B) * cth * sph - (yg * W - yb * B) * sth,
    ]
    np.testing.assert_allclose(g, expect, atol=1e-12)


# --------------------------------------------------------------------------------------
# closed-form trajectories
# --------------------------------------------------------------------------------------

def _one_env_rollout(oracle, v, x0, a, T, S, dt, mult=None, traj=False):
    act = np.repeat(np.asarray(a, dtype=float)[None, :, None], T, axis=0)
    out = oracle.rollout(v, np.asarray(x0, float)[:, None], act, S, dt,
                         mult=None if mult is None else np.asarray(mult, float)[:, None],
                         want_traj=traj)
    return out["traj"][:, :, 0] if traj else out["x"][:, 0]


def _heave_terminal(dl, dq, F):
    """Velocity where d_l w + d_q w |w| = F (F > 0 pushes down)."""
    s = math.copysign(1.0, F)
    return s * (-dl + math.sqrt(dl * dl + 4 * dq * abs(F))) / (2 * dq)


@pytest.mark.parametrize("variant", ["linear", "quadratic_lag"])
def test_heave_steady_state(oracle, variant):
    if variant == "linear":
        v, a_v = BLUEROV2, 0.5
        F = -2 * 40.0 * 0.5                 # two verticals push up (-z)
    else:
        v, a_v = vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05), 0.5
        F = -2 * 40.0 * 0.25
    D = oracle.state_dim(v)
    x = _one_env_rollout(oracle, v, _rest_state(D), [0, 0, 0, 0, a_v, a_v], 3000, 1, 0.01)
    w_star = _heave_terminal(5.0, 37.0, F)
    assert x[9] == pytest.approx(w_star, rel=1e-12, abs=1e-12)
    # no other velocity or rotation is excited
    assert np.abs(x[[7, 8, 10, 11, 12]]).max() < 1e-12
    np.testing.assert_allclose(x[3:7], [1, 0, 0, 0], atol=1e-12)


def test_sink_rate_with_net_weight(oracle):
    mult = np.ones(23)
    mult[22] = 0.95
    x = _one_env_rollout(oracle, BLUEROV2, _rest_state(), [0] * 6, 3000, 1, 0.01, mult=mult)
    W = 11.5 * G0
    assert x[9] == pytest.approx(_heave_terminal(5.0, 37.0, W - 0.95 * W), rel=1e-12)
    assert x[9] > 0                         # sinks (NED z down)


def _surge_vehicle():
    return vehicle_variant(BLUEROV2, r_g=[0, 0, 0], d_quad=[0.0] * 6,
                           thr_pos=[(0.0, 0.0, 0.0)], thr_dir=[(1.0, 0.0, 0.0)])


def test_linear_surge_exact_rk4_recursion(oracle):
    """Decoupled linear surge: each RK4 step maps u - u_inf by R(-d dt / m')."""
    v = _surge_vehicle()
    m_ = 11.5 + 5.5
    d, F, dt = 4.0, 40.0 * 0.7, 0.01
    traj = _one_env_rollout(oracle, v, _rest_state(), [0.7], 200, 1, dt, traj=True)
    u_inf = F / d
    k = _rk4_factor(-d * dt / m_)
    u_expect = u_inf + (0.0 - u_inf) * k ** np.arange(1, 201)
    np.testing.assert_allclose(traj[:, 7], u_expect, rtol=0, atol=2e-13)
    # and the continuous solution u(t) = (F/d)(1 - exp(-d t / m')) to RK4 accuracy
    t = dt * np.arange(1, 201)
    np.testing.assert_allclose(traj[:, 7], u_inf * (1 - np.exp(-d * t / m_)), atol=1e-9)
    assert np.abs(traj[:, [8, 9, 10, 11, 12]]).max() == 0.0


def test_thruster_lag_exact_rk4_recursion(oracle):
    v = vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)
    a = np.array([0.9, -0.6, 0.3, -1.0, 0.2, 0.45, -0.8, 1.0])
    dt = 0.005
    x0 = _rest_state(21)
    x0[13:] = np.linspace(-20, 20, 8)
    traj = _one_env_rollout(oracle, v, x0, a, 60, 1, dt, traj=True)
    fcmd = 40.0 * a * np.abs(a)
    k = _rk4_factor(-dt / 0.05)
    expect = fcmd[None, :] + (x0[13:] - fcmd)[None, :] * (k ** np.arange(1, 61))[:, None]
    np.testing.assert_allclose(traj[:, 13:], expect, rtol=0, atol=1e-12)
    t = dt * np.arange(1, 61)[:, None]
    exact = fcmd + (x0[13:] - fcmd) * np.exp(-t / 0.05)
    # |R^n - e^{nz}| <= n max(R, e^z)^(n-1) |R - e^z|, scaled by the initial offset
    n = np.arange(1, 61)
    bound = (np.abs(x0[13:] - fcmd).max() * (n * max(k, math.exp(-dt / 0.05)) ** (n - 1)).max()
             * abs(k - math.exp(-dt / 0.05)))
    np.testing.assert_allclose(traj[:, 13:], exact, rtol=0, atol=1.01 * bound)
    assert bound < 5e-5


def test_clamp_saturates_throttle(oracle):
    v = _surge_vehicle()
    x1 = _one_env_rollout(oracle, v, _rest_state(), [1.0], 10, 1, 0.01)
    x2 = _one_env_rollout(oracle, v, _rest_state(), [7.5], 10, 1, 0.01)
    np.testing.assert_array_equal(x1, x2)


def test_torque_free_axisymmetric_precession(oracle):
    """Euler's equations with I'_x = I'_y: omega_z constant, (omega_x, omega_y) rotates
    at Omega = (I'_z - I'_x) / I'_x * omega_z."""
    v = vehicle_variant(BLUEROV2, r_g=[0, 0, 0], inertia=[0.2, 0.2, 0.5],
                        added_mass=[5.5, 12.7, 14.6, 0.1, 0.1, 0.05], d_lin=[0.0] * 6,
                        d_quad=[0.0] * 6)
    x0 = _rest_state()
    x0[10:13] = [0.3, -0.2, 1.0]
    dt, T = 0.001, 5000
    traj = _one_env_rollout(oracle, v, x0, [0.0] * 6, T, 1, dt, traj=True)
    Om = (0.55 - 0.3) / 0.3 * 1.0
    t = dt * np.arange(1, T + 1)
    wx = 0.3 * np.cos(Om * t) + 0.2 * np.sin(Om * t)
    wy = 0.3 * np.sin(Om * t) - 0.2 * np.cos(Om * t)
    np.testing.assert_allclose(traj[:, 10], wx, atol=1e-10)
    np.testing.assert_allclose(traj[:, 11], wy, atol=1e-10)
    np.testing.assert_allclose(traj[:, 12], 1.0, atol=1e-12)
    np.testing.assert_allclose(traj[:, 7:10], 0.0, atol=1e-12)


def test_constant_rate_quaternion_exponential(oracle):
    """Spherical inertia keeps omega constant; then q(t) = q0 (x) exp(omega t / 2)."""
    v = vehicle_variant(BLUEROV2, r_g=[0, 0, 0], inertia=[0.2, 0.2, 0.2],
                        added_mass=[5.5, 12.7, 14.6, 0.1, 0.1, 0.1], d_lin=[0.0] * 6,
                        d_quad=[0.0] * 6)
    x0 = _rest_state()
    q0 = euler_to_quat(np.array(0.3), np.array(-0.4), np.array(1.1))
    x0[3:7] = q0
    om = np.array([0.4, -0.7, 0.9])
    x0[10:13] = om
    dt, T = 0.01, 500
    traj = _one_env_rollout(oracle, v, x0, [0.0] * 6, T, 1, dt, traj=True)
    n = np.linalg.norm(om)
    for i in [0, 99, 499]:
        t = dt * (i + 1)
        e = np.concatenate([[math.cos(n * t / 2)], math.sin(n * t / 2) * om / n])
        np.testing.assert_allclose(traj[i, 3:7], _qmul(q0, e), atol=1e-10)
    np.testing.assert_allclose(np.linalg.norm(traj[:, 3:7], axis=1), 1.0, atol=1e-15)


# --------------------------------------------------------------------------------------
# conservation laws (sign of the Coriolis terms)
# --------------------------------------------------------------------------------------

def _free_body():
    # CG = CB off the origin (couples M), W = B, no damping, no thrust: no external force
    r = [0.01, -0.02, 0.03]
    return vehicle_variant(BLUEROV2_HEAVY, r_g=r, r_b=r, d_lin=[0.0] * 6, d_quad=[0.0] * 6)


def _free_traj(oracle, dt, tend=10.0):
    v = _free_body()
    x0 = _rest_state()
    x0[3:7] = euler_to_quat(np.array(0.2), np.array(0.1), np.array(-0.5))
    x0[7:13] = [0.4, -0.3, 0.2, 0.5, -0.6, 0.8]
    T = int(round(tend / dt))
    traj = _one_env_rollout(oracle, v, x0, [0.0] * 8, T, 1, dt, traj=True)
    return v, x0, traj


def test_energy_conserved_with_fourth_order_drift(oracle):
    drifts = []
    for dt in [0.04, 0.02, 0.01]:
        v, x0, traj = _free_traj(oracle, dt)
        M = oracle.mass_matrix(v)
        e0 = 0.5 * x0[7:13] @ M @ x0[7:13]
        e1 = 0.5 * traj[-1, 7:13] @ M @ traj[-1, 7:13]
        drifts.append(abs(e1 - e0) / e0)
    assert drifts[-1] < 1e-7
    assert drifts[0] / drifts[1] > 12 and drifts[1] / drifts[2] > 12


def test_world_momentum_conserved(oracle):
    """Kirchhoff: with no external force the world-frame impulse R(q) a and the angular
    impulse R(q) b + p x R(q) a are constant ([a; b] = M nu).  A sign error in C breaks this."""
    v, x0, traj = _free_traj(oracle, 0.005)
    M = oracle.mass_matrix(v)

    def impulses(x):
        R = oracle.rotation(x[3:7])
        ab = M @ x[7:13]
        P = R @ ab[:3]
        return P, R @ ab[3:] + np.cross(x[:3], P)

    P0, L0 = impulses(x0)
    for i in [100, 999, len(traj) - 1]:
        P, L = impulses(traj[i])
        np.testing.assert_allclose(P, P0, atol=1e-8)
        np.testing.assert_allclose(L, L0, atol=1e-8)


# --------------------------------------------------------------------------------------
# RK4 order, renormalisation, statistics, batching
# --------------------------------------------------------------------------------------

def test_rk4_fourth_order_global_error(oracle):
    """Smooth case (no quadratic damping): halving dt divides the error by ~16."""
    v = vehicle_variant(BLUEROV2_HEAVY, d_quad=[0.0] * 6, thr_map=1, thr_tau=0.05)
    x0 = _rest_state(21)
    x0[3:7] = euler_to_quat(np.array(0.3), np.array(-0.2), np.array(0.5))
    x0[7:13] = [0.5, -0.4, 0.3, 0.8, -0.6, 1.2]
    a = [0.8, -0.5, 0.3, 0.9, -0.7, 0.6, 0.2, -0.4]

    def final(n):
        return _one_env_rollout(oracle, v, x0, a, 1, n, 1.0 / n)

    ref = final(3200)
    errs = [np.abs(final(n) - ref).max() for n in (25, 50, 100)]
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.7 < s < 4.3 for s in slopes), (errs, slopes)


def test_quaternion_unit_after_every_substep(oracle):
    c = CONFIGS["c1"]
    x0 = initial_state(16, 13, c.seed_base + 2)
    act = actions(200, 6, 16, c.seed_base + 3)
    traj = oracle.rollout(BLUEROV2, x0, act, 1, 0.01, want_traj=True)["traj"]
    np.testing.assert_allclose(np.linalg.norm(traj[:, 3:7], axis=1), 1.0, atol=2e-16 * 8)


def test_statistics_brute_force(oracle):
    v = vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)
    E, T = 40, 30
    x0 = initial_state(E, 21, 11)
    act = actions(T, 8, E, 12)
    act[5, 2, 7] = np.nan                      # env 7 goes non-finite from step 5
    mult = param_multipliers(E, 0.2, 13)
    tgt = np.random.default_rng(14).normal(size=(3, E))
    out = oracle.rollout(v, x0, act, 4, 0.005, mult=mult, target=tgt, want_traj=True,
                         want_stats=True)
    traj, st = out["traj"], out["stats"]
    for t in range(T):
        fin = np.isfinite(traj[t]).all(axis=0)
        d = np.linalg.norm(traj[t, :3] - tgt, axis=0)
        ke = np.array([0.5 * traj[t, 7:13, e] @ oracle.mass_matrix(v, mult[:, e]) @ traj[t, 7:13, e]
                       if fin[e] else 0.0 for e in range(E)])
        assert st[t, 3] == (~fin).sum() == (1 if t >= 5 else 0)
        assert st[t, 0] == pytest.approx(d[fin].sum(), rel=1e-14)
        assert st[t, 1] == pytest.approx(d[fin].max(), rel=1e-15)
        assert st[t, 2] == pytest.approx(ke.sum(), rel=1e-13)


def test_batched_classes_equal_separate_runs_and_threads(oracle):
    vb = vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05)
    vh = vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)
    E, T = 24, 20
    cls = np.array([0, 1] * 12, dtype=np.int32)
    x0 = initial_state(E, 21, 21)
    act = actions(T, 8, E, 22)
    mult = param_multipliers(E, 0.2, 23)
    mixed = oracle.rollout([vb, vh], x0, act, 2, 0.005, env_class=cls, mult=mult, nthreads=3)["x"]
    one = oracle.rollout([vb, vh], x0, act, 2, 0.005, env_class=cls, mult=mult, nthreads=1)["x"]
    np.testing.assert_array_equal(mixed, one)
    for k, v in enumerate([vb, vh]):
        sel = cls == k
        D = oracle.state_dim(v)
        sep = oracle.rollout(v, x0[:D, sel], act[:, :, sel], 2, 0.005, mult=mult[:, sel])["x"]
        np.testing.assert_array_equal(mixed[:D, sel], sep)
        assert np.all(mixed[D:, sel] == 0)


# --------------------------------------------------------------------------------------
# circle-tracking loss of the adjoint workload: sum over control steps t = 1..T of
# |p_t - p*_t|^2 + lam (1 - <q_t, q*_t>^2), x_t the state after control step t
# --------------------------------------------------------------------------------------

def _neutral_vehicle(**kw):
    """CG at the CB (r_g = r_b = 0) and B = W: no restoring wrench at any attitude."""
    return vehicle_variant(BLUEROV2, r_g=[0.0, 0.0, 0.0], **kw)


def _axis_angle_quat(axis, angle):
    n = np.asarray(axis, dtype=float)
    n = n / np.linalg.norm(n)
    return np.concatenate([[math.cos(angle / 2)], math.sin(angle / 2) * n])


def _hold(T, arr):
    """[k][E] -> the same reference at every one of T control steps, [T][k][E]."""
    return np.repeat(np.asarray(arr, dtype=float)[None], T, axis=0)


def _random_unit_quats(E, seed):
    q = np.random.default_rng(seed).normal(size=(4, E))
    return q / np.linalg.norm(q, axis=0)


def test_tracking_loss_zero_on_a_held_reference(oracle):
    """At rest with no restoring wrench and zero throttle a vehicle stays put; with the
    reference at its own pose every term vanishes.  Each term is >= 0, so a zero sum over
    the T steps means zero at every step."""
    v = _neutral_vehicle()
    E, T = 6, 7
    rng = np.random.default_rng(31)
    x0 = np.zeros((13, E))
    x0[0:3] = rng.uniform(-3, 3, size=(3, E))
    x0[3:7] = _random_unit_quats(E, 32)
    act = np.zeros((T, 6, E))
    traj = oracle.rollout(v, x0, act, 1, 0.01, want_traj=True)["traj"]
    np.testing.assert_allclose(traj, _hold(T, x0), rtol=0, atol=1e-15)   # the premise
    for lam in (1.0, 0.7):
        loss = oracle.track_loss(v, x0, act, 1, 0.01, _hold(T, x0[0:3]), _hold(T, x0[3:7]),
                                 lam=lam)
        np.testing.assert_allclose(loss, 0.0, rtol=0, atol=1e-14)


def test_tracking_loss_offsets_closed_form(oracle):
    """A held pose offset by d in position and by a rotation of angle delta about any axis
    from the reference: <q, q*> = cos(delta / 2), so each step adds
    |d|^2 + lam sin^2(delta / 2) and the loss is T times that."""
    v = _neutral_vehicle()
    T, lam = 9, 0.7
    deltas = np.array([0.0, 0.3, -1.2, 2.5, math.pi, 4.0, 0.9, -2.2])
    axes = [(0, 0, 1)] * 6 + [(1, 0, 0), (0.3, -0.5, 0.8)]    # yaw-only, roll, oblique
    E = len(deltas)
    rng = np.random.default_rng(41)
    p0 = rng.uniform(-2, 2, size=(3, E))
    d = rng.normal(0.0, 0.5, size=(3, E))
    d[:, 0] = 0.0                                               # a pure attitude offset
    qref = _random_unit_quats(E, 42)
    x0 = np.zeros((13, E))
    x0[0:3] = p0
    for e in range(E):
        # state attitude = reference rotated by delta about a body axis: q = q* (x) r
        x0[3:7, e] = _qmul(qref[:, e], _axis_angle_quat(axes[e], deltas[e]))
    act = np.zeros((T, 6, E))
    loss = oracle.track_loss(v, x0, act, 1, 0.01, _hold(T, p0 - d), _hold(T, qref), lam=lam)
    expect = T * (np.sum(d * d, axis=0) + lam * np.sin(deltas / 2) ** 2)
    np.testing.assert_allclose(loss, expect, rtol=1e-13, atol=1e-14)
    assert expect[4] == pytest.approx(T * (np.sum(d[:, 4] ** 2) + lam), rel=1e-15)


def test_tracking_loss_sign_of_quaternion_is_irrelevant(oracle):
    """q and -q are the same attitude: negating the initial quaternion negates the whole
    attitude trajectory (R(q) is quadratic, q' linear in q), and negating the reference
    quaternions changes no term, on a randomised rollout with every force acting."""
    x0, act, pref, qref, mult = _c4_small(E=6, T=10)
    base = oracle.track_loss(BLUEROV2, x0, act, 1, 0.01, pref, qref, mult=mult)
    x0n = x0.astype(np.float64).copy()
    x0n[3:7] *= -1.0
    np.testing.assert_allclose(oracle.track_loss(BLUEROV2, x0n, act, 1, 0.01, pref, qref,
                                                 mult=mult), base, rtol=1e-14)
    qn = qref.astype(np.float64).copy()
    qn[::2] *= -1.0                                  # every other step's reference
    np.testing.assert_allclose(oracle.track_loss(BLUEROV2, x0, act, 1, 0.01, pref, qn,
                                                 mult=mult), base, rtol=1e-14)
    assert np.all(base > 0)


def test_tracking_loss_counts_the_states_after_each_control_step(oracle):
    """Undamped coasting with no restoring wrench: surge u0 at yaw psi0 keeps nu constant
    (C(nu) nu = 0 for nu along one principal axis), so after control step t of S sub-steps
    p_t = p0 + t S dt u0 (cos psi0, sin psi0, 0).  Against a reference held at the origin
    the loss is sum_{t=1..T} |p0 + t c|^2, and a reference moving with the vehicle gives 0."""
    v = _neutral_vehicle(d_lin=[0.0] * 6, d_quad=[0.0] * 6)
    T, S, dt = 12, 4, 0.005
    psi0 = np.array([0.0, 0.8, -2.4])
    u0 = np.array([0.8, -1.5, 0.3])
    E = len(psi0)
    p0 = np.array([[0.5, -1.0, 2.0], [0.2, 0.3, -0.7], [-0.4, 1.1, 0.05]])
    x0 = np.zeros((13, E))
    x0[0:3] = p0
    x0[3] = np.cos(psi0 / 2)
    x0[6] = np.sin(psi0 / 2)
    x0[7] = u0
    act = np.zeros((T, 6, E))
    c = u0 * S * dt * np.stack([np.cos(psi0), np.sin(psi0), np.zeros(E)])   # [3][E] per step
    t = np.arange(1, T + 1)
    expect = (T * np.sum(p0 * p0, axis=0) + 2 * np.sum(p0 * c, axis=0) * t.sum()
              + np.sum(c * c, axis=0) * (t * t).sum())
    loss = oracle.track_loss(v, x0, act, S, dt, np.zeros((T, 3, E)), _hold(T, x0[3:7]))
    np.testing.assert_allclose(loss, expect, rtol=1e-13)
    moving = p0[None] + t[:, None, None] * c[None]
    loss = oracle.track_loss(v, x0, act, S, dt, moving, _hold(T, x0[3:7]))
    np.testing.assert_allclose(loss, 0.0, atol=1e-20)


# --------------------------------------------------------------------------------------
# reference gradient (dual numbers) vs finite differences and a closed form
# --------------------------------------------------------------------------------------

def _c4_small(E=4, T=8):
    c = CONFIGS["c4"]
    x0 = initial_state(E, 13, c.seed_base + 2)
    act = actions(T, 6, E, c.seed_base + 3)
    pref, qref = circle_waypoints(T, E, c.dt_sub, c.seed_base + 4)
    mult = param_multipliers(E, 0.2, 77)
    return x0, act, pref, qref, mult


def test_dual_gradient_matches_central_fd(oracle):
    x0, act, pref, qref, mult = _c4_small()
    E = x0.shape[1]
    loss, g_act, g_th, g_x0 = oracle.track_loss_grad(BLUEROV2, x0, act, 1, 0.01, pref, qref,
                                                     mult=mult, want_x0=True)
    np.testing.assert_allclose(loss, oracle.track_loss(BLUEROV2, x0, act, 1, 0.01, pref, qref,
                                                       mult=mult), rtol=1e-15)
    h = 1e-6
    rng = np.random.default_rng(5)
    act64 = act.astype(np.float64)
    # actions: a random subset of (t, i)
    for _ in range(12):
        t, i = rng.integers(0, act.shape[0]), rng.integers(0, 6)
        ap, am = act64.copy(), act64.copy()
        ap[t, i] += h
        am[t, i] -= h
        fd = (oracle.track_loss(BLUEROV2, x0, ap, 1, 0.01, pref, qref, mult=mult)
              - oracle.track_loss(BLUEROV2, x0, am, 1, 0.01, pref, qref, mult=mult)) / (2 * h)
        np.testing.assert_allclose(g_act[t, i], fd, rtol=1e-6, atol=1e-8)
    # hydrodynamic parameters, absolute units.  The five-point stencil
    # (f(-2s) - 8 f(-s) + 8 f(s) - f(2s)) / 12s with a step of 3e-3 of each env's own
    # parameter value has truncation error O(s^4) and rounding error ~ eps L / s, both
    # far below the tolerance: the worst env and parameter sits at 0.0074 of it (a
    # central difference with a step of 1e-6 sat at 0.87, on its rounding floor).
    nominal = np.concatenate([BLUEROV2["added_mass"], BLUEROV2["d_lin"], BLUEROV2["d_quad"],
                              [BLUEROV2["buoyancy"]]])
    m64 = mult.astype(np.float64)
    for j in range(19):
        p = nominal[j] * m64[4 + j]                  # absolute parameter, per env
        step = 3e-3 * p

        def loss_at(k):
            m = m64.copy()
            m[4 + j] = (p + k * step) / nominal[j]
            return oracle.track_loss(BLUEROV2, x0, act, 1, 0.01, pref, qref, mult=m)

        fd = (loss_at(-2) - 8 * loss_at(-1) + 8 * loss_at(1) - loss_at(2)) / (12 * step)
        np.testing.assert_allclose(g_th[j], fd, rtol=2e-6, atol=1e-9)
    # initial state
    for i in [0, 4, 9, 12]:
        xp, xm = x0.astype(np.float64).copy(), x0.astype(np.float64).copy()
        xp[i] += h
        xm[i] -= h
        fd = (oracle.track_loss(BLUEROV2, xp, act, 1, 0.01, pref, qref, mult=mult)
              - oracle.track_loss(BLUEROV2, xm, act, 1, 0.01, pref, qref, mult=mult)) / (2 * h)
        np.testing.assert_allclose(g_x0[i], fd, rtol=1e-6, atol=1e-8)


def test_steady_heave_sensitivity_closed_form(oracle):
    """dw*/dd_l = -w* / (d_l + 2 d_q |w*|) from the steady state of the heave balance."""
    T = 3000
    act = np.zeros((T, 6))
    act[:, 4:] = 0.5
    dth = np.zeros(19)
    dth[6 + 2] = 1.0                               # D_L of heave
    traj, dtraj = oracle.jvp(BLUEROV2, _rest_state(), act, 1, 0.01, dtheta=dth)
    w = _heave_terminal(5.0, 37.0, -40.0)
    assert traj[-1, 9] == pytest.approx(w, rel=1e-12)
    assert dtraj[-1, 9] == pytest.approx(-w / (5.0 + 2 * 37.0 * abs(w)), rel=1e-10)


def test_golden_regression(oracle):
    """The oracle still produces the committed C1 states (written by tests/golden/make_golden.py)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_c1_regression.json")) as f:
        g = json.load(f)
    c = CONFIGS["c1"]
    x0 = initial_state(c.n_envs, 13, c.seed_base + 2)
    act = actions(c.n_ctrl, 6, c.n_envs, c.seed_base + 3)
    out = oracle.rollout(BLUEROV2, x0, act, c.substeps, c.dt_sub, want_traj=True, want_stats=True)
    for t in g["steps"]:
        for e in g["envs"]:
            np.testing.assert_allclose(out["traj"][t - 1, :, e], g["states"][str(t)][str(e)],
                                       rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(out["stats"][t - 1], g["stats"][str(t)], rtol=1e-12)
