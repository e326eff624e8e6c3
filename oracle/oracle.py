"""ctypes shim over the FP64 oracle (fossen_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and
by the benchmark's CPU-baseline leg.  The GPU library and its binding never
import this module.  Parity unpinned: fidelity to a physical BlueROV2 (the
paper prints no parameters or trajectories), see the oracle's header.

All inputs are widened to FP64 before the call, so the oracle consumes the very
FP32 values the GPU library consumes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fossen_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_THR = 8
NUM_THETA = 19

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class OrVehicle(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("inertia", ctypes.c_double * 3),
        ("r_g", ctypes.c_double * 3), ("r_b", ctypes.c_double * 3),
        ("added_mass", ctypes.c_double * 6), ("d_lin", ctypes.c_double * 6),
        ("d_quad", ctypes.c_double * 6), ("buoyancy", ctypes.c_double),
        ("thr_pos", (ctypes.c_double * 3) * MAX_THR), ("thr_dir", (ctypes.c_double * 3) * MAX_THR),
        ("f_max", ctypes.c_double), ("thr_tau", ctypes.c_double),
        ("n_thr", ctypes.c_int32), ("thr_map", ctypes.c_int32),
    ]


class OrTask(ctypes.Structure):
    _fields_ = [
        ("task", ctypes.c_int32), ("lookahead", ctypes.c_int32),
        ("radius", ctypes.c_double), ("omega", ctypes.c_double),
        ("climb_rate", ctypes.c_double), ("lookahead_dt", ctypes.c_double),
        ("episode_steps", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("max_error", ctypes.c_double),
    ]


TASKS = {"station": 0, "circle": 1, "helix": 2, "lemniscate": 3}


def task_struct(task):
    """Fill the oracle's task struct from a dict: task (name or 0..3), lookahead, radius,
    omega, climb_rate, lookahead_dt, episode_steps, max_error."""
    t = OrTask()
    kind = task["task"]
    t.task = TASKS[kind] if isinstance(kind, str) else int(kind)
    t.lookahead = int(task.get("lookahead", 1))
    t.radius = float(task.get("radius", 0.0))
    t.omega = float(task.get("omega", 0.0))
    t.climb_rate = float(task.get("climb_rate", 0.0))
    t.lookahead_dt = float(task.get("lookahead_dt", 0.0))
    t.episode_steps = int(task.get("episode_steps", 1 << 30))
    t.max_error = float(task.get("max_error", 0.0))
    return t


def build(force=False):
    """Compile the oracle with g++ (OpenMP, FP64, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp = ctypes.POINTER(OrVehicle)
        L.or_version.restype = ctypes.c_int
        L.or_max_threads.restype = ctypes.c_int
        L.or_alloc.argtypes = [vp, _dp]
        L.or_mass_matrix.argtypes = [vp, _dp, _dp]
        L.or_coriolis_matrix.argtypes = [_dp, _dp, _dp]
        L.or_restoring.argtypes = [vp, _dp, _dp, _dp]
        L.or_rotation.argtypes = [_dp, _dp]
        L.or_rhs.argtypes = [vp, _dp, _dp, _dp, _dp]
        L.or_rollout.argtypes = [vp, ctypes.c_int, _ip, ctypes.c_int64, _dp, _dp, ctypes.c_int,
                                 _dp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, _dp, _dp, _dp, ctypes.c_int]
        L.or_kinetic_energy.argtypes = [vp, _dp, _dp]
        L.or_kinetic_energy.restype = ctypes.c_double
        L.or_track_loss.argtypes = [vp, ctypes.c_int64, _dp, _dp, ctypes.c_int, _dp, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp,
                                    ctypes.c_double, _dp, ctypes.c_int]
        L.or_track_loss_grad.argtypes = [vp, ctypes.c_int64, _dp, _dp, ctypes.c_int, _dp,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, _dp, _dp, ctypes.c_double, _dp, _dp,
                                         _dp, _dp, ctypes.c_int]
        L.or_jvp.argtypes = [vp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_double, _dp, _dp, _dp, _dp, _dp]
        tp = ctypes.POINTER(OrTask)
        L.or_task_reference.argtypes = [tp, _dp, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, _dp, _dp]
        L.or_euler_zyx.argtypes = [_dp, _dp]
        L.or_task_obs_dim.argtypes = [tp]
        L.or_task_observe.argtypes = [tp, ctypes.c_int64, _dp, ctypes.c_int, _dp, _dp, _dp, _ip,
                                      ctypes.c_double, _dp]
        L.or_task_rollout.argtypes = [vp, ctypes.c_int, _ip, ctypes.c_int64, _dp, _dp,
                                      ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, tp, _dp, _dp, _dp, _ip, _dp, _dp, _dp,
                                      _dp, _ip, _dp, _ip, ctypes.c_int]
        L.or_split_rollout.argtypes = [vp, ctypes.c_int, _ip, ctypes.c_int64, _dp, _dp, _dp,
                                       ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_double, _dp, _dp, _dp,
                                       ctypes.c_int]
        L.or_split_rollout.restype = ctypes.c_int
        for name in ("or_alloc", "or_mass_matrix", "or_coriolis_matrix", "or_restoring",
                     "or_rotation", "or_rhs", "or_rollout", "or_track_loss",
                     "or_track_loss_grad", "or_jvp", "or_task_reference", "or_euler_zyx",
                     "or_task_obs_dim", "or_task_observe", "or_task_rollout"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a):
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def vehicle(preset):
    """Fill the oracle's own vehicle struct from a preset dict (raw numbers only)."""
    v = OrVehicle()
    v.mass = preset["mass"]
    for i in range(3):
        v.inertia[i] = preset["inertia"][i]
        v.r_g[i] = preset["r_g"][i]
        v.r_b[i] = preset["r_b"][i]
    for i in range(6):
        v.added_mass[i] = preset["added_mass"][i]
        v.d_lin[i] = preset["d_lin"][i]
        v.d_quad[i] = preset["d_quad"][i]
    v.buoyancy = preset["buoyancy"]
    n = len(preset["thr_pos"])
    assert 1 <= n <= MAX_THR and len(preset["thr_dir"]) == n
    for i in range(n):
        for j in range(3):
            v.thr_pos[i][j] = preset["thr_pos"][i][j]
            v.thr_dir[i][j] = preset["thr_dir"][i][j]
    v.n_thr = n
    v.f_max = preset["f_max"]
    v.thr_map = int(preset["thr_map"])
    v.thr_tau = float(preset["thr_tau"])
    return v


def state_dim(preset):
    return 13 + (len(preset["thr_pos"]) if preset["thr_tau"] > 0 else 0)


def alloc(preset):
    out = np.zeros((6, MAX_THR))
    lib().or_alloc(ctypes.byref(vehicle(preset)), _ptr(out))
    return out[:, :len(preset["thr_pos"])]


def mass_matrix(preset, mult=None):
    out = np.zeros((6, 6))
    m = _f64(mult)
    lib().or_mass_matrix(ctypes.byref(vehicle(preset)), _ptr(m), _ptr(out))
    return out


def coriolis_matrix(M, nu):
    out = np.zeros((6, 6))
    lib().or_coriolis_matrix(_ptr(_f64(M)), _ptr(_f64(nu)), _ptr(out))
    return out


def restoring(preset, q, mult=None):
    out = np.zeros(6)
    lib().or_restoring(ctypes.byref(vehicle(preset)), _ptr(_f64(mult)), _ptr(_f64(q)), _ptr(out))
    return out


def rotation(q):
    out = np.zeros((3, 3))
    lib().or_rotation(_ptr(_f64(q)), _ptr(out))
    return out


def rhs(preset, x, a, mult=None):
    x = _f64(x)
    out = np.zeros_like(x)
    lib().or_rhs(ctypes.byref(vehicle(preset)), _ptr(_f64(mult)), _ptr(x), _ptr(_f64(a)),
                 _ptr(out))
    return out


def kinetic_energy(preset, nu, mult=None):
    return lib().or_kinetic_energy(ctypes.byref(vehicle(preset)), _ptr(_f64(mult)),
                                   _ptr(_f64(nu)))


def rollout(presets, x0, act, n_substeps, dt, env_class=None, mult=None, target=None,
            want_traj=False, want_stats=False, nthreads=0):
    """Batched FP64 rollout.  x0 [D][E], act [T][nmax][E]; returns dict with
    'x' [D][E] (final), optionally 'traj' [T][D][E] and 'stats' [T][4]."""
    if isinstance(presets, dict):
        presets = [presets]
    x0 = _f64(x0)
    act = _f64(act)
    D, E = x0.shape
    T, nmax, E2 = act.shape
    assert E2 == E
    vs = (OrVehicle * len(presets))(*[vehicle(p) for p in presets])
    ec = None
    if env_class is not None:
        ec = np.ascontiguousarray(np.asarray(env_class, dtype=np.int32))
        assert ec.shape == (E,)
    m = _f64(mult)
    if m is not None:
        assert m.shape == (23, E)
    tg = _f64(target)
    if tg is not None:
        assert tg.shape == (3, E)
    xT = np.zeros((D, E))
    traj = np.zeros((T, D, E)) if want_traj else None
    stats = np.zeros((T, 4)) if want_stats else None
    rc = lib().or_rollout(vs, len(presets), ec.ctypes.data_as(_ip) if ec is not None else None,
                          E, _ptr(m), _ptr(x0), D, _ptr(act), nmax, _ptr(tg), T,
                          int(n_substeps), float(dt), _ptr(traj), _ptr(xT), _ptr(stats),
                          int(nthreads))
    if rc != 0:
        raise ValueError("or_rollout rejected its arguments")
    out = {"x": xT}
    if want_traj:
        out["traj"] = traj
    if want_stats:
        out["stats"] = stats
    return out


def track_loss(preset, x0, act, n_substeps, dt, pref, qref, lam=1.0, mult=None, nthreads=0):
    x0 = _f64(x0)
    act = _f64(act)
    D, E = x0.shape
    T, nmax, _ = act.shape
    loss = np.zeros(E)
    rc = lib().or_track_loss(ctypes.byref(vehicle(preset)), E, _ptr(_f64(mult)), _ptr(x0), D,
                             _ptr(act), nmax, T, int(n_substeps), float(dt), _ptr(_f64(pref)),
                             _ptr(_f64(qref)), float(lam), _ptr(loss), int(nthreads))
    if rc != 0:
        raise ValueError("or_track_loss rejected its arguments")
    return loss


def track_loss_grad(preset, x0, act, n_substeps, dt, pref, qref, lam=1.0, mult=None,
                    want_x0=False, nthreads=0):
    """Forward-mode (dual number) gradient of :func:`track_loss`.
    Returns (loss [E], g_act [T][nmax][E], g_theta [19][E], g_x0 [D][E] or None)."""
    x0 = _f64(x0)
    act = _f64(act)
    D, E = x0.shape
    T, nmax, _ = act.shape
    loss = np.zeros(E)
    g_act = np.zeros((T, nmax, E))
    g_th = np.zeros((NUM_THETA, E))
    g_x0 = np.zeros((D, E)) if want_x0 else None
    rc = lib().or_track_loss_grad(ctypes.byref(vehicle(preset)), E, _ptr(_f64(mult)), _ptr(x0),
                                  D, _ptr(act), nmax, T, int(n_substeps), float(dt),
                                  _ptr(_f64(pref)), _ptr(_f64(qref)), float(lam), _ptr(loss),
                                  _ptr(g_act), _ptr(g_th), _ptr(g_x0), int(nthreads))
    if rc != 0:
        raise ValueError("or_track_loss_grad rejected its arguments")
    return loss, g_act, g_th, g_x0


def jvp(preset, x0, act, n_substeps, dt, mult=None, dact=None, dtheta=None, dx0=None):
    """Tangent of one env's trajectory.  x0 [Dc], act [T][nmax]."""
    x0 = _f64(x0)
    act = _f64(act)
    T, nmax = act.shape
    Dc = state_dim(preset)
    traj = np.zeros((T, Dc))
    dtraj = np.zeros((T, Dc))
    rc = lib().or_jvp(ctypes.byref(vehicle(preset)), _ptr(_f64(mult)), _ptr(x0), _ptr(act), nmax,
                      T, int(n_substeps), float(dt), _ptr(_f64(dact)), _ptr(_f64(dtheta)),
                      _ptr(_f64(dx0)), _ptr(traj), _ptr(dtraj))
    if rc != 0:
        raise ValueError("or_jvp rejected its arguments")
    return traj, dtraj


# -- tasks of Sec. III ---------------------------------------------------------------------

def _i32(a):
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def task_reference(task, center, phase, yaw, t):
    """Reference point (3,) and heading of one env at episode time t."""
    pr = np.zeros(3)
    psi = ctypes.c_double()
    c = _f64(center)
    rc = lib().or_task_reference(ctypes.byref(task_struct(task)), _ptr(c), float(phase),
                                 float(yaw), float(t), _ptr(pr), ctypes.byref(psi))
    if rc != 0:
        raise ValueError("or_task_reference rejected its arguments")
    return pr, psi.value


def euler_zyx(q):
    rpy = np.zeros(3)
    lib().or_euler_zyx(_ptr(_f64(q)), _ptr(rpy))
    return rpy


def task_obs_dim(task):
    return lib().or_task_obs_dim(ctypes.byref(task_struct(task)))


def task_observe(task, x, center, phase, yaw, k, dt_ctrl):
    """Observations [obs_dim][E] of states x [D][E] at episode steps k [E]."""
    x = _f64(x)
    D, E = x.shape
    obs = np.zeros((task_obs_dim(task), E))
    c, ph, yw, kk = _f64(center), _f64(phase), _f64(yaw), _i32(k)
    rc = lib().or_task_observe(ctypes.byref(task_struct(task)), E, _ptr(x), D, _ptr(c), _ptr(ph),
                               _ptr(yw), kk.ctypes.data_as(_ip) if kk is not None else None,
                               float(dt_ctrl), _ptr(obs))
    if rc != 0:
        raise ValueError("or_task_observe rejected its arguments")
    return obs


def task_rollout(presets, task, x0, act, n_substeps, dt, center, phase, yaw=None, env_class=None,
                 mult=None, k0=None, reset_state=None, reset_mult=None, nthreads=0):
    """T Gym-style steps with the task epilogue and automatic reset; returns dict with
    'obs' [T+1][obs_dim][E], 'err' [T][E], 'done' [T][E], 'x' [D][E], 'k' [E]."""
    if isinstance(presets, dict):
        presets = [presets]
    x0 = _f64(x0)
    act = _f64(act)
    D, E = x0.shape
    T, nmax, E2 = act.shape
    assert E2 == E
    vs = (OrVehicle * len(presets))(*[vehicle(p) for p in presets])
    ec = _i32(env_class)
    tk = task_struct(task)
    od = lib().or_task_obs_dim(ctypes.byref(tk))
    obs = np.zeros((T + 1, od, E))
    err = np.zeros((T, E))
    done = np.zeros((T, E), np.int32)
    xT = np.zeros((D, E))
    kT = np.zeros(E, np.int32)
    k0a = _i32(k0)
    m, c, ph, yw, rs, rm = (_f64(mult), _f64(center), _f64(phase), _f64(yaw), _f64(reset_state),
                            _f64(reset_mult))
    rc = lib().or_task_rollout(vs, len(presets), ec.ctypes.data_as(_ip) if ec is not None else None,
                               E, _ptr(m), _ptr(x0), D, _ptr(act), nmax, T, int(n_substeps),
                               float(dt), ctypes.byref(tk), _ptr(c), _ptr(ph), _ptr(yw),
                               k0a.ctypes.data_as(_ip) if k0a is not None else None, _ptr(rs),
                               _ptr(rm), _ptr(obs), _ptr(err), done.ctypes.data_as(_ip), _ptr(xT),
                               kT.ctypes.data_as(_ip), int(nthreads))
    if rc != 0:
        raise ValueError("or_task_rollout rejected its arguments")
    return {"obs": obs, "err": err, "done": done, "x": xT, "k": kT}


# -- split scheme of Sec. II -----------------------------------------------------------------

def split_rollout(presets, x0, act, n_substeps, dt, env_class=None, mult=None, acc0=None,
                  want_traj=False, nthreads=0):
    """The split scheme (rigid body by semi-implicit Euler, hydrodynamic wrench with the
    added-mass term of the previous sub-step as an external force).  Returns dict with
    'x' [D][E], 'acc' [6][E] and optionally 'traj' [T][D][E]."""
    if isinstance(presets, dict):
        presets = [presets]
    x0 = _f64(x0)
    act = _f64(act)
    D, E = x0.shape
    T, nmax, E2 = act.shape
    assert E2 == E
    vs = (OrVehicle * len(presets))(*[vehicle(p) for p in presets])
    ec = _i32(env_class)
    xT = np.zeros((D, E))
    accT = np.zeros((6, E))
    traj = np.zeros((T, D, E)) if want_traj else None
    m, a0 = _f64(mult), _f64(acc0)
    rc = lib().or_split_rollout(vs, len(presets), ec.ctypes.data_as(_ip) if ec is not None else None,
                                E, _ptr(m), _ptr(x0), _ptr(a0), D, _ptr(act), nmax, T,
                                int(n_substeps), float(dt), _ptr(traj), _ptr(xT), _ptr(accT),
                                int(nthreads))
    if rc != 0:
        raise ValueError("or_split_rollout rejected its arguments")
    out = {"x": xT, "acc": accT}
    if want_traj:
        out["traj"] = traj
    return out
