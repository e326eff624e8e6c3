"""CPU check of the kernels' reverse-mode code: tests/vjp_check.hip compiles the
device headers for the host and compares every vector-Jacobian product (state,
throttle, the 19 hydrodynamic parameters; 1 to 4 sub-steps; with and without
thruster lag) with central finite differences in FP64."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_vjp_matches_finite_differences(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "vjp_check")
    subprocess.check_call([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950",
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2410_14117_amd", "csrc"),
                           os.path.join(ROOT, "tests", "vjp_check.hip"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 failures" in r.stdout
