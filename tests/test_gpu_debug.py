"""The bounds-checked debug build (libmg_debug.so: the same sources built with
-DMG_DEBUG) on the GPU.  tests/debug_workload.py runs every kernel family once; here
it runs in the test's process with the release library and in a child process with
the debug library (MG_LIBRARY), and:

* the debug build's results equal the release build's, bitwise, and none of its checks
  fires (the debug word of every sim and of the server reads 0);
* with MG_DEBUG_SHRINK=100 (read by the debug build when a sim is created) the kernels
  treat caller columns >= n_envs - 100 as out of bounds: MG_DBG_COLUMN is set, those
  envs are left untouched, and the other envs' results still equal the release
  build's.  The shrunk bound is below the real one, so every access stays in bounds
  whether or not a check fires (a failed check only makes its lane skip its work)."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from tests.gpu_util import say

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests"))


@pytest.fixture(scope="module")
def release():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import debug_workload
    from paper_2410_14117_amd import mg
    if mg.lib().mg_debug_build() != 0:
        pytest.fail("the test process must load the release library")
    say("debug build: release pass of the workload")
    return debug_workload.run()


def _debug_pass(tmp_path, extra_env=None):
    from paper_2410_14117_amd import mg
    if not os.path.exists(mg.DEBUG_LIB_PATH):
        pytest.fail(f"{mg.DEBUG_LIB_PATH} is missing: python -m paper_2410_14117_amd.build --debug")
    out = str(tmp_path / "debug.npz")
    env = dict(os.environ, MG_LIBRARY=mg.DEBUG_LIB_PATH, **(extra_env or {}))
    say(f"debug build: child process, {extra_env or 'no test hook'}")
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "debug_workload.py"),
                        out], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    return dict(np.load(out))


def test_debug_build_equals_release_and_no_check_fires(release, tmp_path):
    rel, words = release
    assert words == {"sim": 0, "adjoint": 0, "server": 0}
    dbg = _debug_pass(tmp_path)
    for w in ("sim", "adjoint", "server"):
        assert int(dbg[f"word_{w}"]) == 0, (w, int(dbg[f"word_{w}"]))
    for k, v in rel.items():
        assert np.array_equal(dbg[k], v, equal_nan=True), k


def test_checks_fire_on_a_shrunk_bound_and_skip_only_those_envs(release, tmp_path):
    from paper_2410_14117_amd import mg
    rel, _ = release
    dbg = _debug_pass(tmp_path, {"MG_DEBUG_SHRINK": "100"})
    assert int(dbg["word_sim"]) & mg.MG_DBG_COLUMN
    assert int(dbg["word_adjoint"]) & mg.MG_DBG_COLUMN
    assert int(dbg["word_server"]) == 0          # the server takes no shrunk bound
    E, Ea = 3000, 2000
    for k in ("fused_traj", "plain_state", "rollout_state", "split_state", "task_obs0",
              "task_obs2", "task_err1", "task_done2"):
        assert np.array_equal(dbg[k][..., :E - 100], rel[k][..., :E - 100], equal_nan=True), k
    # the skipped envs were never reset either: still the zeros the sim was created with
    for k in ("plain_state", "rollout_state", "split_state"):
        assert (dbg[k][..., E - 100:] == 0).all(), k
    for k in ("adj_traj_act", "adj_traj_theta", "adj_traj_x0", "adj_recompute_act",
              "adj_recompute_theta", "adj_recompute_x0", "adj_traj"):
        assert np.array_equal(dbg[k][..., :Ea - 100], rel[k][..., :Ea - 100], equal_nan=True), k
    assert np.array_equal(dbg["serve_ptr"], rel["serve_ptr"])
    assert np.array_equal(dbg["serve_seed"], rel["serve_seed"])
