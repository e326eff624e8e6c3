"""Pins of the oracle's split scheme (Sec. II: the rigid body stepped by semi-implicit
Euler, the hydrodynamic wrench with the previous sub-step's added-mass acceleration acting
as an external force) against what it reduces to: a one-degree-of-freedom heave
recurrence written out by hand, the closed-form attitude of the normalised first-order
quaternion update at a constant rate, the growth factor A / m of the lagged added mass,
and first-order convergence to the coupled RK4 solution.  CPU only.
"""
import copy
import math

import numpy as np
import pytest

from workloads import BLUEROV2, G0, vehicle_variant, initial_state, actions


def _heave_vehicle(added_w, d_w=5.0, f_max=10.0):
    """Neutral, CG = CB = CO, one thruster at the CO pushing along body z, no quadratic
    damping: a throttle a gives pure heave."""
    v = copy.deepcopy(BLUEROV2)
    v["r_g"] = [0.0, 0.0, 0.0]
    v["r_b"] = [0.0, 0.0, 0.0]
    v["buoyancy"] = v["mass"] * G0
    v["added_mass"] = [5.5, 12.7, added_w, 0.12, 0.12, 0.12]
    v["d_lin"] = [4.0, 6.0, d_w, 0.07, 0.07, 0.07]
    v["d_quad"] = [0.0] * 6
    v["thr_pos"] = [[0.0, 0.0, 0.0]]
    v["thr_dir"] = [[0.0, 0.0, 1.0]]
    v["f_max"] = f_max
    v["thr_map"] = 0
    v["thr_tau"] = 0.0
    return v


def _rest(E=1, D=13):
    x = np.zeros((D, E))
    x[3] = 1.0
    return x


@pytest.mark.parametrize("added_w", [4.0, 9.0])
def test_heave_recurrence(oracle, added_w):
    """m a_n = F - d w_n - A a_(n-1), w_(n+1) = w_n + dt a_n, z_(n+1) = z_n + dt w_(n+1)."""
    v = _heave_vehicle(added_w)
    m, A, d, F, dt, n = v["mass"], added_w, 5.0, 0.6 * 10.0, 0.01, 300
    act = np.full((n, 1, 1), 0.6)
    got = oracle.split_rollout(v, _rest(), act, 1, dt, want_traj=True)
    z, w, a = 0.0, 0.0, 0.0
    for k in range(n):
        a = (F - d * w - A * a) / m
        w += dt * a
        z += dt * w
        np.testing.assert_allclose(got["traj"][k, [2, 9], 0], [z, w], rtol=1e-12, atol=1e-14)
    assert got["acc"][2, 0] == pytest.approx(a, rel=1e-12)
    np.testing.assert_allclose(got["traj"][-1, [0, 1, 7, 8, 10, 11, 12], 0], 0.0, atol=1e-15)


def test_lagged_added_mass_growth_factor(oracle):
    """Heave with the added mass above the rigid-body mass (A / m = 1.27, as in the
    BlueROV2 preset) is unstable: the acceleration alternates in sign and grows by A / m
    per sub-step; below it (A / m = 0.5) the velocity settles at F / d."""
    dt = 0.001
    for added_w, unstable in ((14.6, True), (5.75, False)):
        v = _heave_vehicle(added_w, d_w=0.0)
        act = np.zeros((200, 1, 1))
        x0 = _rest()
        acc0 = np.zeros((6, 1))
        acc0[2] = 1.0
        got = oracle.split_rollout(v, x0, act, 1, dt, acc0=acc0)
        ratio = abs(got["acc"][2, 0])
        if unstable:
            assert ratio == pytest.approx((added_w / v["mass"]) ** 200, rel=1e-6)
        else:
            # 0.5^200 lies below the rounding of the restoring terms that cancel beside it
            assert ratio < 1e-12
    v = _heave_vehicle(5.75)
    got = oracle.split_rollout(v, _rest(), np.full((20000, 1, 1), 0.6), 1, 0.01)
    assert got["x"][9, 0] == pytest.approx(6.0 / 5.0, rel=1e-9)


def test_attitude_update_at_constant_rate(oracle):
    """Spin about the body z axis of a body with no forces: each sub-step maps q to
    q (x) (1, 0, 0, w dt / 2) / |.|, a rotation by 2 atan(w dt / 2) about z."""
    v = copy.deepcopy(_heave_vehicle(5.0))
    v["added_mass"] = [0.0] * 6
    v["d_lin"] = [0.0] * 6
    w, dt, n = 0.9, 0.05, 40
    x0 = _rest()
    x0[12] = w
    got = oracle.split_rollout(v, x0, np.zeros((n, 1, 1)), 1, dt)
    ang = n * 2 * math.atan(w * dt / 2)
    np.testing.assert_allclose(got["x"][3:7, 0], [math.cos(ang / 2), 0, 0, math.sin(ang / 2)],
                               atol=1e-13)
    np.testing.assert_allclose(got["x"][7:13, 0], [0, 0, 0, 0, 0, w], atol=1e-13)
    np.testing.assert_allclose(got["x"][:3, 0], 0.0, atol=1e-15)


def test_first_order_convergence_to_the_coupled_solution(oracle):
    """With the added mass below the rigid-body mass on every axis the split scheme
    converges to the coupled RK4 solution at first order: halving dt halves the error."""
    v = vehicle_variant(BLUEROV2, thr_map=0, thr_tau=0.0)
    v = copy.deepcopy(v)
    v["added_mass"] = [a * 0.4 for a in v["added_mass"]]
    E, t_end = 8, 1.0
    x0 = initial_state(E, 13, 901)
    act1 = actions(1, 6, E, 902)
    ref = oracle.rollout(v, x0, act1, 4000, t_end / 4000)["x"]
    errs = []
    for n in (100, 200, 400):
        x = oracle.split_rollout(v, x0, act1, n, t_end / n)["x"]
        errs.append(np.max(np.abs(x - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.7 < r1 < 2.3 and 1.8 < r2 < 2.2
