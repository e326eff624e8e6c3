"""CPU run of the FP32 adjoint backward's own source (fossen_adjoint.h: adj_bwd_env and
recompute_segment, host and device code): tests/adj_host_check.hip runs the backward of
every env of small rollouts (8 thrusters with and without lag, 6 with and without, 1 with
lag; one and several segments) in four forms -- its own recomputation loop, that loop
factored into recompute_segment, the whole-rollout recomputation then the sweep, and the
sweep that loads each next sub-step's inputs one step ahead -- which must agree bitwise, built for the host with AddressSanitizer and
UndefinedBehaviorSanitizer (GPU code is not instrumented)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_adjoint_backward_source_on_the_host(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "adj_host_check")
    subprocess.check_call([hipcc, "-O0", "-std=c++17", "--offload-arch=gfx950",
                           "-fsanitize=address,undefined", "-fno-gpu-sanitize",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2410_14117_amd", "csrc"),
                           os.path.join(ROOT, "tests", "adj_host_check.hip"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout, r.stderr[-3000:])
    assert r.returncode == 0, r.stderr[-3000:]
    assert "0 failures" in r.stdout and "runtime error" not in r.stderr
