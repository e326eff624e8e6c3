"""C-ABI contract tests that need no GPU: the library loads, exports every
function include/mg.h declares, and rejects bad arguments without side effects."""
import ctypes
import os
import re

import pytest

from paper_2410_14117_amd import mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = mg.lib()
    names = _declared("mg.h")
    assert "mg_create" in names and "mg_step" in names and "mg_rollout" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_debug_build_exports_the_same_symbols_and_says_so():
    """libmg_debug.so (the bounds-checked build of the same sources) exports every symbol
    include/mg.h declares; mg_debug_build tells the two builds apart."""
    if not os.path.exists(mg.DEBUG_LIB_PATH):
        pytest.skip("libmg_debug.so not built (python -m paper_2410_14117_amd.build --debug)")
    D = ctypes.CDLL(mg.DEBUG_LIB_PATH)
    missing = [n for n in _declared("mg.h") if not hasattr(D, n)]
    assert not missing, missing
    assert D.mg_debug_build() == 1 and mg.lib().mg_debug_build() == 0
    assert D.mg_abi_version() == mg.MG_ABI_VERSION
    w = ctypes.c_uint32(7)
    assert mg.lib().mg_debug_word(None, ctypes.byref(w), 0) == mg.MG_ERR_INVALID
    assert mg.lib().mg_server_debug_word(None, ctypes.byref(w), 0) == mg.MG_ERR_INVALID


def test_client_driver_exports_every_declared_symbol():
    text = open(os.path.join(ROOT, "include", "mg_clients.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(mgc_[a-z_]+)\s*\(", text)))
    assert names == ["mgc_replay"]
    L = mg.clients_lib()
    assert all(hasattr(L, n) for n in names)
    # bad arguments are refused before anything is submitted
    assert L.mgc_replay(None, 1, 0, None, None, None, 0, None, None, None) == -1


def test_abi_version_and_status_strings():
    L = mg.lib()
    assert L.mg_abi_version() == mg.MG_ABI_VERSION
    for s in range(7):
        assert L.mg_status_str(s)
    assert L.mg_status_str(99) == b"unknown status"


def _cfg(preset, n_envs=64, **kw):
    v = (mg.MgVehicle * 1)(mg.vehicle_struct(preset))
    c = mg.MgConfig()
    c.abi_version = kw.get("abi_version", mg.MG_ABI_VERSION)
    c.n_classes = kw.get("n_classes", 1)
    c.n_envs = n_envs
    c.classes = v
    c.dt_sub = kw.get("dt_sub", 0.01)
    c.substeps = kw.get("substeps", 1)
    c.device = kw.get("device", 0)
    c.stream = None
    return c, v


def test_create_rejects_bad_arguments():
    from workloads import BLUEROV2, vehicle_variant
    L = mg.lib()
    h = ctypes.c_void_p()
    assert L.mg_create(None, ctypes.byref(h)) == mg.MG_ERR_INVALID
    assert L.mg_create(ctypes.byref(_cfg(BLUEROV2)[0]), None) == mg.MG_ERR_INVALID
    for kw in [dict(abi_version=99), dict(n_classes=0), dict(dt_sub=0.0), dict(dt_sub=float("nan")),
               dict(substeps=0)]:
        c, _keep = _cfg(BLUEROV2, **kw)
        assert L.mg_create(ctypes.byref(c), ctypes.byref(h)) == mg.MG_ERR_INVALID
        assert h.value is None
    c, _keep = _cfg(BLUEROV2, n_envs=0)
    assert L.mg_create(ctypes.byref(c), ctypes.byref(h)) == mg.MG_ERR_INVALID
    # rows of at most 2^30 floats: the step kernel addresses them with 32-bit offsets
    c, _keep = _cfg(BLUEROV2, n_envs=(1 << 30) - 1023)
    assert L.mg_create(ctypes.byref(c), ctypes.byref(h)) == mg.MG_ERR_INVALID
    assert b"2^30" in L.mg_last_error(None)
    bad = vehicle_variant(BLUEROV2, thr_map=3)
    c, _keep = _cfg(bad)
    assert L.mg_create(ctypes.byref(c), ctypes.byref(h)) == mg.MG_ERR_INVALID
    assert b"thr_map" in L.mg_last_error(None)
    off_axis = vehicle_variant(BLUEROV2, r_g=[0.01, 0.0, 0.02])
    c, _keep = _cfg(off_axis)
    assert L.mg_create(ctypes.byref(c), ctypes.byref(h)) == mg.MG_ERR_UNSUPPORTED


def test_null_sim_calls_are_safe():
    L = mg.lib()
    L.mg_destroy(None)
    assert L.mg_state_dim(None) == -1
    assert L.mg_num_envs(None) == -1
    assert L.mg_step(None, None, 1, None, None, None) == mg.MG_ERR_INVALID
    assert L.mg_reset(None, None, 0, None, None) == mg.MG_ERR_INVALID
    assert L.mg_synchronize(None) == mg.MG_ERR_INVALID
    assert L.mg_step_split(None, None, 1, None) == mg.MG_ERR_INVALID
    assert L.mg_task_obs_dim(None) == 0
    assert L.mg_task_configure(None, None, None, None, None) == mg.MG_ERR_INVALID
    assert L.mg_task_observe(None, None) == mg.MG_ERR_INVALID
    assert L.mg_task_step(None, None, None, None, None, None, None) == mg.MG_ERR_INVALID
    assert L.mg_task_counters(None, None) == mg.MG_ERR_INVALID


def test_create_without_device_reports_device_error():
    """On a host with no GPU mg_create fails with MG_ERR_DEVICE (never a CPU fallback)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from workloads import BLUEROV2
    L = mg.lib()
    h = ctypes.c_void_p()
    c, _keep = _cfg(BLUEROV2)
    assert L.mg_create(ctypes.byref(c), ctypes.byref(h)) == mg.MG_ERR_DEVICE
    assert h.value is None


def _server_cfg(preset, **kw):
    v = (mg.MgVehicle * 1)(mg.vehicle_struct(preset))
    c = mg.MgServerConfig()
    c.abi_version = kw.get("abi_version", mg.MG_ABI_VERSION)
    c.n_classes = 1
    c.classes = v
    c.dt_sub = 0.005
    c.substeps = kw.get("substeps", 4)
    c.device = 0
    c.fifo_plain = kw.get("fifo_plain", 0)
    c.reserve_bytes = kw.get("reserve_bytes", 0)
    c.steps_per_tick = kw.get("steps_per_tick", 1)
    return c, v


def test_server_create_rejects_bad_config():
    """Malformed server configurations fail with MG_ERR_INVALID before any device work."""
    from workloads import BLUEROV2
    L = mg.lib()
    h = ctypes.c_void_p()
    assert L.mg_server_create(None, ctypes.byref(h)) == mg.MG_ERR_INVALID
    for kw in [dict(abi_version=2), dict(substeps=0), dict(reserve_bytes=-1),
               dict(steps_per_tick=-1), dict(steps_per_tick=65),
               dict(fifo_plain=1, steps_per_tick=2)]:
        c, _keep = _server_cfg(BLUEROV2, **kw)
        assert L.mg_server_create(ctypes.byref(c), ctypes.byref(h)) == mg.MG_ERR_INVALID, kw
        assert h.value is None
