"""CPU check of the fused step kernel's machine code (built here for gfx950): the
properties its speed rests on.  Three waves per SIMD (at most 168 VGPRs, no scratch),
457 VALU instructions in the sub-step loop, and the per-launch loads and stores
addressed as an SGPR row base plus a 32-bit lane offset (global_load / global_store
with an SGPR base) rather than with 64-bit index arithmetic per access."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

KERNELS = {
    6: "_ZN2mg6k_stepILi6ELb1ELb0EEEvNS_8StepArgsENS_10ClassConstE",
    8: "_ZN2mg6k_stepILi8ELb1ELb0EEEvNS_8StepArgsENS_10ClassConstE",
}


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_2410_14117_amd import build
    out = str(tmp_path_factory.mktemp("asm") / "kernels_step.s")
    subprocess.check_call([hipcc, "-S", "--cuda-device-only", *build.CFLAGS,
                           os.path.join(build.CSRC, "kernels_step.hip"), "-o", out],
                          stderr=subprocess.DEVNULL)
    return open(out).read()


def _body(s, name):
    i = s.index(name + ":")
    return s[i:s.index(".Lfunc_end", i)]


def _meta(s, name):
    meta = s[s.index("amdhsa.kernels:"):]
    e = [x for x in meta.split("\n  - ") if (".name:           " + name) in x][0]
    return (int(re.search(r"\.vgpr_count:\s+(\d+)", e).group(1)),
            int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", e).group(1)))


def _ops(lines):
    return [l.split()[0] for l in lines
            if l.strip() and not l.strip().startswith((".", ";")) and not re.match(r"^\S+:", l)]


@pytest.mark.parametrize("n_thr", [6, 8])
def test_three_waves_per_simd_without_scratch(asm, n_thr):
    vgpr, scratch = _meta(asm, KERNELS[n_thr])
    assert vgpr <= 168, vgpr
    assert scratch == 0, scratch


@pytest.mark.parametrize("n_thr", [6, 8])
def test_substep_loop_instruction_count(asm, n_thr):
    lines = _body(asm, KERNELS[n_thr]).split("\n")
    k = [n for n, l in enumerate(lines) if "v_rsq_f32" in l][0]      # renormalisation
    start = max(n for n in range(k) if re.match(r"^\.LBB\w+:", lines[n]))
    end = min(n for n in range(k, len(lines)) if re.match(r"\s*s_cbranch", lines[n]))
    valu = [o for o in _ops(lines[start + 1:end]) if o.startswith("v_")]
    assert len(valu) <= 460, len(valu)
    assert not any(o.startswith(("global_", "buffer_", "scratch_")) for o in _ops(lines[start + 1:end]))


@pytest.mark.parametrize("n_thr", [6, 8])
def test_loads_and_stores_use_an_sgpr_base(asm, n_thr):
    lines = _body(asm, KERNELS[n_thr]).split("\n")
    mem = [l for l in lines if re.search(r"\bglobal_(load|store)", l)]
    saddr = [l for l in mem if re.search(r", s\[\d+:\d+\]", l)]
    # state, constants, throttles, statistics inputs and the state write-back
    assert len(saddr) >= 60, (len(saddr), len(mem))
    assert not any(re.search(r"\bflat_(load|store)", l) for l in lines)
    assert "v_mad_u64_u32" not in _ops(lines)
