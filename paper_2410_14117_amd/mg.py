"""Python binding of libmg (include/mg.h): argument marshalling only.

Every computation runs in the HIP kernels of libmg.so; torch tensors serve as
device memory and torch's current HIP stream as the stream.  If the library
is missing the binding raises instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MG_LIBRARY") or os.path.join(HERE, "libmg.so")
# the bounds-checked build (python -m paper_2410_14117_amd.build --debug); select it with
# MG_LIBRARY=<its path> before this module is imported
DEBUG_LIB_PATH = os.path.join(HERE, "libmg_debug.so")
# failed-check bits of the debug build (include/mg.h)
MG_DBG_SEGMENT, MG_DBG_COLUMN, MG_DBG_INTERNAL, MG_DBG_LIST, MG_DBG_PAGE = 1, 2, 4, 8, 16

MG_ABI_VERSION = 4
MAX_THR = 8
NUM_PARAMS = 23
NUM_THETA = 19
NUM_STATS = 4

(MG_OK, MG_ERR_INVALID, MG_ERR_OOM, MG_ERR_DEVICE, MG_ERR_UNSUPPORTED, MG_ERR_BUSY,
 MG_ERR_CANCELLED) = range(7)


class MgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mg status {status}: {msg}")
        self.status = status


class MgVehicle(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("inertia", ctypes.c_double * 3),
        ("r_g", ctypes.c_double * 3), ("r_b", ctypes.c_double * 3),
        ("added_mass", ctypes.c_double * 6), ("d_lin", ctypes.c_double * 6),
        ("d_quad", ctypes.c_double * 6), ("buoyancy", ctypes.c_double),
        ("thr_pos", (ctypes.c_double * 3) * MAX_THR), ("thr_dir", (ctypes.c_double * 3) * MAX_THR),
        ("f_max", ctypes.c_double), ("thr_tau", ctypes.c_double),
        ("n_thr", ctypes.c_int32), ("thr_map", ctypes.c_int32),
    ]


class MgConfig(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32), ("n_classes", ctypes.c_int32),
        ("n_envs", ctypes.c_int64), ("classes", ctypes.POINTER(MgVehicle)),
        ("env_class", ctypes.POINTER(ctypes.c_int32)), ("dt_sub", ctypes.c_double),
        ("substeps", ctypes.c_int32), ("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
    ]


class MgServerConfig(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32), ("n_classes", ctypes.c_int32),
        ("classes", ctypes.POINTER(MgVehicle)), ("dt_sub", ctypes.c_double),
        ("substeps", ctypes.c_int32), ("device", ctypes.c_int32),
        ("mem_cap_bytes", ctypes.c_int64), ("mem_fraction", ctypes.c_double),
        ("fifo_plain", ctypes.c_int32), ("max_queue", ctypes.c_int32),
        ("reserve_bytes", ctypes.c_int64),
        ("steps_per_tick", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class MgTask(ctypes.Structure):
    _fields_ = [
        ("task", ctypes.c_int32), ("lookahead", ctypes.c_int32),
        ("radius", ctypes.c_double), ("omega", ctypes.c_double),
        ("climb_rate", ctypes.c_double), ("lookahead_dt", ctypes.c_double),
        ("episode_steps", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("max_error", ctypes.c_double),
    ]


TASKS = {"station": 0, "circle": 1, "helix": 2, "lemniscate": 3}


def task_struct(task):
    """mg_task from a dict: task (name or 0..3), lookahead, radius, omega, climb_rate,
    lookahead_dt, episode_steps, max_error."""
    t = MgTask()
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


class MgRequest(ctypes.Structure):
    _fields_ = [
        ("n_envs", ctypes.c_int64), ("n_steps", ctypes.c_int32),
        ("actions_from_seed", ctypes.c_int32),
        ("env_class", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("param_mult", ctypes.c_void_p),
        ("actions", ctypes.c_void_p), ("ld", ctypes.c_int64), ("out", ctypes.c_void_p),
        ("arrival_ns", ctypes.c_uint64), ("action_seed", ctypes.c_uint64),
    ]


class MgServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("completed", "rejected", "ticks", "env_steps", "active_envs", "max_active_envs",
                 "queued", "cap_pages", "created_pages", "issue_ns", "wait_ns", "mean_queue_ns",
                 "max_queue_ns", "max_issue_ns", "grow_events", "held_joins",
                 "deferred_retires")]


_vp = ctypes.c_void_p
_SIGS = {
    "mg_abi_version": (ctypes.c_uint32, []),
    "mg_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "mg_last_error": (ctypes.c_char_p, [_vp]),
    "mg_create": (ctypes.c_int32, [ctypes.POINTER(MgConfig), ctypes.POINTER(_vp)]),
    "mg_destroy": (None, [_vp]),
    "mg_set_stream": (ctypes.c_int32, [_vp, _vp]),
    "mg_state_dim": (ctypes.c_int32, [_vp]),
    "mg_action_dim": (ctypes.c_int32, [_vp]),
    "mg_num_envs": (ctypes.c_int64, [_vp]),
    "mg_reset": (ctypes.c_int32, [_vp, _vp, ctypes.c_int64, _vp, _vp]),
    "mg_set_params": (ctypes.c_int32, [_vp, _vp]),
    "mg_set_state": (ctypes.c_int32, [_vp, _vp]),
    "mg_step": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "mg_step_plain": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "mg_rollout": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32]),
    "mg_get_state": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32]),
    "mg_get_params": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32]),
    "mg_synchronize": (ctypes.c_int32, [_vp]),
    "mg_get_flags": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32]),
    "mg_debug_build": (ctypes.c_int32, []),
    "mg_debug_word": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int32]),
    "mg_server_debug_word": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_uint32),
                                              ctypes.c_int32]),
    "mg_clock_ns": (ctypes.c_uint64, []),
    "mg_server_create": (ctypes.c_int32, [ctypes.POINTER(MgServerConfig), ctypes.POINTER(_vp)]),
    "mg_server_submit": (ctypes.c_int32, [_vp, ctypes.POINTER(MgRequest),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "mg_server_wait": (ctypes.c_int32, [_vp, ctypes.c_uint64, ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_double)]),
    "mg_server_get_stats": (ctypes.c_int32, [_vp, ctypes.POINTER(MgServerStats)]),
    "mg_server_cancel": (ctypes.c_int32, [_vp, ctypes.c_uint64]),
    "mg_server_last_error": (ctypes.c_char_p, [_vp]),
    "mg_server_destroy": (None, [_vp]),
    "mg_step_split": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp]),
    "mg_task_configure": (ctypes.c_int32, [_vp, ctypes.POINTER(MgTask), _vp, _vp, _vp]),
    "mg_task_obs_dim": (ctypes.c_int32, [_vp]),
    "mg_task_observe": (ctypes.c_int32, [_vp, _vp]),
    "mg_task_step": (ctypes.c_int32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mg_task_counters": (ctypes.c_int32, [_vp, _vp]),
    "mg_adj_forward": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp]),
    "mg_adj_backward": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                         _vp, _vp, _vp, _vp]),
    "mg_adj_backward_noalloc": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int32,
                                                 ctypes.c_int32, _vp, _vp, _vp, _vp]),
}

_lib = None


def lib():
    """Load libmg.so (built by ``python -m paper_2410_14117_amd.build``); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2410_14117_amd.build` (there is no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.mg_abi_version() != MG_ABI_VERSION:
            raise ImportError("libmg ABI version mismatch")
        _lib = L
    return _lib


_clients = None


def clients_lib():
    """The serving client driver, libmg_clients.so (built beside libmg.so)."""
    global _clients
    if _clients is None:
        lib()
        path = os.path.join(os.path.dirname(LIB_PATH), "libmg_clients.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_2410_14117_amd.build`")
        L = ctypes.CDLL(path)
        L.mgc_replay.restype = ctypes.c_int
        L.mgc_replay.argtypes = [_vp, ctypes.c_int32, ctypes.c_int64, _vp, _vp,
                                 ctypes.POINTER(MgRequest), ctypes.c_uint64, _vp, _vp, _vp]
        _clients = L
    return _clients


def vehicle_struct(preset):
    v = MgVehicle()
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
    if not 1 <= n <= MAX_THR or len(preset["thr_dir"]) != n:
        raise ValueError("a vehicle needs 1..8 thrusters with a position and a direction each")
    for i in range(n):
        for k in range(3):
            v.thr_pos[i][k] = preset["thr_pos"][i][k]
            v.thr_dir[i][k] = preset["thr_dir"][i][k]
    v.n_thr = n
    v.f_max = preset["f_max"]
    v.thr_map = int(preset["thr_map"])
    v.thr_tau = float(preset["thr_tau"])
    return v


def _ptr(t, dtype, shape, name):
    """Device pointer of a contiguous CUDA tensor with the given dtype/shape (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Sim:
    """A batch of environments on one GPU (wraps an ``mg_sim``)."""

    def __init__(self, classes, n_envs, dt_sub, substeps, env_class=None, device=0):
        L = lib()
        if isinstance(classes, dict):
            classes = [classes]
        self._classes = (MgVehicle * len(classes))(*[vehicle_struct(c) for c in classes])
        cfg = MgConfig()
        cfg.abi_version = MG_ABI_VERSION
        cfg.n_classes = len(classes)
        cfg.n_envs = int(n_envs)
        cfg.classes = self._classes
        ec = None
        if env_class is not None:
            ec = np.ascontiguousarray(np.asarray(env_class, dtype=np.int32))
            if ec.shape != (n_envs,):
                raise ValueError("env_class must have shape [n_envs]")
            cfg.env_class = ec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        cfg.dt_sub = float(dt_sub)
        cfg.substeps = int(substeps)
        cfg.device = int(device)
        cfg.stream = _current_stream()
        h = _vp()
        st = L.mg_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != MG_OK:
            raise MgError(st, L.mg_last_error(None).decode())
        self._h = h
        self.device = int(device)
        self.n_envs = int(n_envs)
        self.state_dim = L.mg_state_dim(h)
        self.action_dim = L.mg_action_dim(h)
        self.dt_sub = float(dt_sub)
        self.substeps = int(substeps)

    # -- plumbing --------------------------------------------------------------------------
    def _check(self, st):
        if st != MG_OK:
            raise MgError(st, lib().mg_last_error(self._h).decode())

    def _bind_stream(self):
        self._check(lib().mg_set_stream(self._h, _current_stream()))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls -----------------------------------------------------------------------------
    def reset(self, env_ids=None, state=None, param_mult=None):
        import torch
        n = self.n_envs if env_ids is None else int(env_ids.numel())
        ids = _ptr(env_ids, torch.int64, (n,), "env_ids")
        s = _ptr(state, torch.float32, (self.state_dim, n), "state")
        m = _ptr(param_mult, torch.float32, (NUM_PARAMS, n), "param_mult")
        self._bind_stream()
        self._check(lib().mg_reset(self._h, ids, n if env_ids is not None else 0, s, m))

    def set_params(self, params):
        import torch
        p = _ptr(params, torch.float32, (NUM_PARAMS, self.n_envs), "params")
        self._bind_stream()
        self._check(lib().mg_set_params(self._h, p))

    def set_state(self, state):
        import torch
        s = _ptr(state, torch.float32, (self.state_dim, self.n_envs), "state")
        self._bind_stream()
        self._check(lib().mg_set_state(self._h, s))

    def _step_args(self, actions, n_ctrl, targets, traj, stats):
        import torch
        E, D, N = self.n_envs, self.state_dim, self.action_dim
        a = _ptr(actions, torch.float32, (n_ctrl, N, E), "actions")
        tg = _ptr(targets, torch.float32, (3, E), "targets")
        tr = _ptr(traj, torch.float32, (n_ctrl, D, E), "traj")
        stt = _ptr(stats, torch.float64, (n_ctrl, NUM_STATS), "stats")
        return a, tg, tr, stt

    def step_split(self, actions, traj=None):
        """actions [n_ctrl][N_max][E]: n_ctrl control steps of the split scheme of Sec. II
        in one launch per class (see mg_step_split)."""
        import torch
        n_ctrl = int(actions.shape[0])
        E, D, N = self.n_envs, self.state_dim, self.action_dim
        a = _ptr(actions, torch.float32, (n_ctrl, N, E), "actions")
        tr = _ptr(traj, torch.float32, (n_ctrl, D, E), "traj")
        self._bind_stream()
        self._check(lib().mg_step_split(self._h, a, n_ctrl, tr))

    # -- Gym-style tasks ---------------------------------------------------------------------
    def task_configure(self, task, center, phase, yaw=None):
        """task: dict (see task_struct); center [3][E], phase [E], yaw [E] device tensors."""
        import torch
        E = self.n_envs
        self._task = task_struct(task)
        self._bind_stream()
        self._check(lib().mg_task_configure(
            self._h, ctypes.byref(self._task), _ptr(center, torch.float32, (3, E), "center"),
            _ptr(phase, torch.float32, (E,), "phase"), _ptr(yaw, torch.float32, (E,), "yaw")))
        self.obs_dim = lib().mg_task_obs_dim(self._h)

    def task_observe(self, obs=None):
        import torch
        if obs is None:
            obs = torch.empty((self.obs_dim, self.n_envs), dtype=torch.float32,
                              device=f"cuda:{self.device}")
        p = _ptr(obs, torch.float32, (self.obs_dim, self.n_envs), "obs")
        self._bind_stream()
        self._check(lib().mg_task_observe(self._h, p))
        return obs

    def task_step(self, actions, obs=None, err=None, done=None, reset_state=None,
                  reset_mult=None):
        """actions [N_max][E]; returns (obs [obs_dim][E], err [E], done [E] int32)."""
        import torch
        E, dev = self.n_envs, f"cuda:{self.device}"
        if obs is None:
            obs = torch.empty((self.obs_dim, E), dtype=torch.float32, device=dev)
        if err is None:
            err = torch.empty((E,), dtype=torch.float32, device=dev)
        if done is None:
            done = torch.empty((E,), dtype=torch.int32, device=dev)
        args = (_ptr(actions, torch.float32, (self.action_dim, E), "actions"),
                _ptr(obs, torch.float32, (self.obs_dim, E), "obs"),
                _ptr(err, torch.float32, (E,), "err"),
                _ptr(done, torch.int32, (E,), "done"),
                _ptr(reset_state, torch.float32, (self.state_dim, E), "reset_state"),
                _ptr(reset_mult, torch.float32, (NUM_PARAMS, E), "reset_mult"))
        self._bind_stream()
        self._check(lib().mg_task_step(self._h, *args))
        return obs, err, done

    def task_counters(self, out=None):
        import torch
        if out is None:
            out = torch.empty((self.n_envs,), dtype=torch.int32, device=f"cuda:{self.device}")
        p = _ptr(out, torch.int32, (self.n_envs,), "out")
        self._bind_stream()
        self._check(lib().mg_task_counters(self._h, p))
        return out

    def step(self, actions, targets=None, traj=None, stats=None, plain=False):
        """actions [n_ctrl][N_max][E]: n_ctrl control steps fused in one launch per class."""
        n_ctrl = int(actions.shape[0])
        a, tg, tr, st = self._step_args(actions, n_ctrl, targets, traj, stats)
        self._bind_stream()
        fn = lib().mg_step_plain if plain else lib().mg_step
        self._check(fn(self._h, a, n_ctrl, tg, tr, st))

    def rollout(self, actions, targets=None, traj=None, stats=None, plain=False):
        """actions [T][N_max][E]: T launches per class replayed from a cached HIP graph."""
        T = int(actions.shape[0])
        a, tg, tr, st = self._step_args(actions, T, targets, traj, stats)
        self._bind_stream()
        self._check(lib().mg_rollout(self._h, a, T, tg, tr, st, 1 if plain else 0))

    def get_state(self, out=None):
        import torch
        if out is None:
            out = torch.empty((self.state_dim, self.n_envs), dtype=torch.float32,
                              device=f"cuda:{self.device}")
        p = _ptr(out, torch.float32, (self.state_dim, self.n_envs), "out")
        self._bind_stream()
        self._check(lib().mg_get_state(self._h, p, 1))
        return out

    def get_params(self, out=None):
        import torch
        if out is None:
            out = torch.empty((NUM_PARAMS, self.n_envs), dtype=torch.float32,
                              device=f"cuda:{self.device}")
        p = _ptr(out, torch.float32, (NUM_PARAMS, self.n_envs), "out")
        self._bind_stream()
        self._check(lib().mg_get_params(self._h, p, 1))
        return out

    def synchronize(self):
        self._check(lib().mg_synchronize(self._h))

    def get_flags(self):
        """Per-env status flags (int32 [E] device tensor): 1 = state went non-finite, 2 = mass
        matrix not positive definite; a flagged env is frozen."""
        import torch
        out = torch.empty((self.n_envs,), dtype=torch.int32, device=f"cuda:{self.device}")
        self._bind_stream()
        self._check(lib().mg_get_flags(self._h, out.data_ptr(), 1))
        return out

    def debug_word(self, clear=True):
        """Failed-check bits of the debug build's kernels (MG_DBG_*; always 0 in the release
        build); waits for the sim's stream."""
        w = ctypes.c_uint32(0)
        self._bind_stream()
        self._check(lib().mg_debug_word(self._h, ctypes.byref(w), 1 if clear else 0))
        return w.value

    # -- adjoint ---------------------------------------------------------------------------
    def adj_forward(self, actions, ckpt_every, ckpt=None, traj=None):
        """Rollout of T = actions.shape[0] control steps from the current state, saving a
        checkpoint before every ckpt_every-th step.  Returns (ckpt, traj)."""
        import torch
        T, E, D, N = int(actions.shape[0]), self.n_envs, self.state_dim, self.action_dim
        K = int(ckpt_every)
        if K < 1:
            raise ValueError("ckpt_every must be >= 1")
        nseg = (T + K - 1) // K
        dev = f"cuda:{self.device}"
        if ckpt is None:
            ckpt = torch.empty((nseg, D, E), dtype=torch.float32, device=dev)
        a = _ptr(actions, torch.float32, (T, N, E), "actions")
        ck = _ptr(ckpt, torch.float32, (nseg, D, E), "ckpt")
        tr = _ptr(traj, torch.float32, (T, D, E), "traj")
        self._bind_stream()
        self._check(lib().mg_adj_forward(self._h, a, T, K, ck, tr))
        return ckpt, traj

    def adj_backward(self, ckpt, actions, ckpt_every, dL_dtraj, want_x0=True, out=None,
                     noalloc=False, traj=None):
        """Returns (dL/d actions [T][N_max][E], dL/d theta [19][E], dL/d x0 [D][E] or None).
        out: optional (dL_dact, dL_dtheta, dL_dx0 or None) tensors to write into;
        noalloc: call mg_adj_backward_noalloc (static scratch, no device allocation);
        traj: the trajectory adj_forward wrote (with one sub-step per control step the
        backward then reads its inputs from it instead of recomputing them)."""
        import torch
        T, E, D, N = int(actions.shape[0]), self.n_envs, self.state_dim, self.action_dim
        K = int(ckpt_every)
        nseg = (T + K - 1) // K
        dev = f"cuda:{self.device}"
        if out is None:
            gact = torch.empty((T, N, E), dtype=torch.float32, device=dev)
            gth = torch.empty((NUM_THETA, E), dtype=torch.float32, device=dev)
            gx0 = torch.empty((D, E), dtype=torch.float32, device=dev) if want_x0 else None
        else:
            gact, gth, gx0 = out
        ga = _ptr(gact, torch.float32, (T, N, E), "dL_dact")
        gt = _ptr(gth, torch.float32, (NUM_THETA, E), "dL_dtheta")
        gx = _ptr(gx0, torch.float32, (D, E), "dL_dx0")
        ck = _ptr(ckpt, torch.float32, (nseg, D, E), "ckpt")
        a = _ptr(actions, torch.float32, (T, N, E), "actions")
        g = _ptr(dL_dtraj, torch.float32, (T, D, E), "dL_dtraj")
        tr = _ptr(traj, torch.float32, (T, D, E), "traj")
        self._bind_stream()
        fn = lib().mg_adj_backward_noalloc if noalloc else lib().mg_adj_backward
        self._check(fn(self._h, ck, tr, a, T, K, g, ga, gt, gx))
        return gact, gth, gx0


def page_bytes(state_dim):
    """Device bytes of one 64-env serving page (state + derived constants + column map)."""
    return (state_dim + 30) * 64 * 4 + 64 * 4


class Server:
    """Continuous-batching serving loop on one GPU (wraps an ``mg_server``)."""

    def __init__(self, classes, dt_sub, substeps, device=0, mem_cap_bytes=0, mem_fraction=0.0,
                 fifo_plain=False, max_queue=0, reserve_bytes=0, steps_per_tick=1):
        import threading
        L = lib()
        if isinstance(classes, dict):
            classes = [classes]
        self._classes = (MgVehicle * len(classes))(*[vehicle_struct(c) for c in classes])
        cfg = MgServerConfig()
        cfg.abi_version = MG_ABI_VERSION
        cfg.n_classes = len(classes)
        cfg.classes = self._classes
        cfg.dt_sub = float(dt_sub)
        cfg.substeps = int(substeps)
        cfg.device = int(device)
        cfg.mem_cap_bytes = int(mem_cap_bytes)
        cfg.mem_fraction = float(mem_fraction)
        cfg.fifo_plain = 1 if fifo_plain else 0
        cfg.max_queue = int(max_queue)
        cfg.reserve_bytes = int(reserve_bytes)
        cfg.steps_per_tick = int(steps_per_tick)
        h = _vp()
        st = L.mg_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != MG_OK:
            raise MgError(st, L.mg_server_last_error(None).decode())
        self._h = h
        self.state_dim = 13 + max([len(c["thr_pos"]) for c in classes if c["thr_tau"] > 0] or [0])
        self.action_dim = max(len(c["thr_pos"]) for c in classes)
        self._keep = {}
        self._lock = threading.Lock()

    @staticmethod
    def clock_ns():
        return lib().mg_clock_ns()

    def submit(self, n_envs, n_steps, x0_ptr, actions_ptr, ld, out, env_class=None,
               mult_ptr=None, arrival_ns=0, action_seed=None):
        """Device pointers x0 [D][ld], actions [n_steps][N_max][ld], mult [23][ld] (optional);
        out: host float32 array [D][n_envs] that receives the final states.  With
        action_seed (an unsigned 64-bit int) the throttles are generated on the device from
        it and actions_ptr is ignored.  Returns (status, ticket)."""
        if out.dtype != np.float32 or out.shape != (self.state_dim, n_envs) or \
                not out.flags["C_CONTIGUOUS"]:
            raise ValueError("out must be a contiguous float32 [D][n_envs] host array")
        ec = None
        if env_class is not None:
            ec = np.ascontiguousarray(np.asarray(env_class, dtype=np.int32))
            if ec.shape != (n_envs,):
                raise ValueError("env_class must have shape [n_envs]")
        r = MgRequest()
        r.n_envs = int(n_envs)
        r.n_steps = int(n_steps)
        r.env_class = ec.ctypes.data if ec is not None else None
        r.x0 = int(x0_ptr)
        r.param_mult = int(mult_ptr) if mult_ptr else None
        if action_seed is None:
            r.actions = int(actions_ptr)
        else:
            r.actions_from_seed = 1
            r.action_seed = int(action_seed) & 0xFFFFFFFFFFFFFFFF
        r.ld = int(ld)
        r.out = out.ctypes.data
        r.arrival_ns = int(arrival_ns)
        t = ctypes.c_uint64()
        st = lib().mg_server_submit(self._h, ctypes.byref(r), ctypes.byref(t))
        if st == MG_OK:
            with self._lock:
                self._keep[t.value] = out
        return st, t.value

    def wait(self, ticket, timeout_us=-1):
        """Returns (status, latency_s)."""
        lat = ctypes.c_double(0.0)
        st = lib().mg_server_wait(self._h, ctypes.c_uint64(ticket), int(timeout_us),
                                  ctypes.byref(lat))
        if st != MG_ERR_BUSY:
            with self._lock:
                self._keep.pop(ticket, None)
        return st, lat.value

    def replay(self, requests, n_clients, start_delay_ns=20_000_000):
        """Replays an arrival trace from n_clients native client threads (libmg_clients.so,
        mgc_replay): request i is submitted by client requests[i]["client"] at
        t0 + requests[i]["at_ns"], stamped with that arrival, and waited for by the same
        thread; t0 is start_delay_ns after the requests have been marshalled.  Each request
        is a dict with client, at_ns, n_envs, n_steps, x0_ptr, ld, out (host [D][n_envs]
        float32), and optionally env_class, mult_ptr, actions_ptr or action_seed.  Returns
        (status [n] int32, latency_s [n], submit lag ns [n], t0 on mg_clock_ns)."""
        n = len(requests)
        reqs = (MgRequest * max(1, n))()
        client = np.zeros(max(1, n), np.int32)
        at = np.zeros(max(1, n), np.uint64)
        keep = []
        for i, q in enumerate(requests):
            out = q["out"]
            if out.dtype != np.float32 or out.shape != (self.state_dim, q["n_envs"]) or \
                    not out.flags["C_CONTIGUOUS"]:
                raise ValueError("out must be a contiguous float32 [D][n_envs] host array")
            r = reqs[i]
            r.n_envs = int(q["n_envs"])
            r.n_steps = int(q["n_steps"])
            ec = q.get("env_class")
            if ec is not None:
                ec = np.ascontiguousarray(np.asarray(ec, dtype=np.int32))
                keep.append(ec)
                r.env_class = ec.ctypes.data
            r.x0 = int(q["x0_ptr"])
            r.param_mult = int(q["mult_ptr"]) if q.get("mult_ptr") else None
            if q.get("action_seed") is not None:
                r.actions_from_seed = 1
                r.action_seed = int(q["action_seed"]) & 0xFFFFFFFFFFFFFFFF
            else:
                r.actions = int(q["actions_ptr"])
            r.ld = int(q["ld"])
            r.out = out.ctypes.data
            client[i] = int(q["client"])
            at[i] = int(q["at_ns"])
        status = np.zeros(max(1, n), np.int32)
        lat = np.zeros(max(1, n), np.float64)
        lag = np.zeros(max(1, n), np.int64)
        L = clients_lib()
        t0 = int(Server.clock_ns()) + int(start_delay_ns)
        rc = L.mgc_replay(self._h, int(n_clients), n, client.ctypes.data, at.ctypes.data, reqs,
                          t0, status.ctypes.data, lat.ctypes.data, lag.ctypes.data)
        if rc != 0:
            raise ValueError("mgc_replay rejected its arguments")
        return status[:n], lat[:n], lag[:n], t0

    def cancel(self, ticket):
        """Cancels a request that has not completed (mg_server_cancel); returns the status."""
        return lib().mg_server_cancel(self._h, int(ticket))

    def last_error(self):
        return (lib().mg_server_last_error(self._h) or b"").decode()

    def debug_word(self, clear=True):
        """The server's failed-check bits (debug build; 0 in the release build)."""
        w = ctypes.c_uint32(0)
        st = lib().mg_server_debug_word(self._h, ctypes.byref(w), 1 if clear else 0)
        if st:
            raise RuntimeError(f"mg_server_debug_word failed: {st}")
        return w.value

    def stats(self):
        s = MgServerStats()
        lib().mg_server_get_stats(self._h, ctypes.byref(s))
        return {n: getattr(s, n) for n, _ in MgServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().mg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
