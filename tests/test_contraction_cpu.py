"""CPU check of the device code's floating-point contraction (gfx950 IR built here).

Kernels compiled from the same source must round alike: the tests require bitwise
equality between the fused and per-sub-step step kernels, the serving kernels and the
step, the adjoint's forward, recomputation and its one-wave, two-wave and
trajectory-reading sweeps.  HIP compiles with contraction allowed per operation, and
the backend fuses a multiply into an FMA with the sum it feeds when it can.  For a
product that has a single use that is always the case; for a product with several uses,
one of them a sum, the choice depends on the rest of the kernel, so two kernels with the
same source line can round it differently (it happened: a two-wave build came out with
four fewer FMAs and different low bits).  Such products are written with mul_nc (a
multiply compiled with contraction off).  This test scans the device IR of every kernel
source for a contractable multiply with several uses of which one is a contractable add
or subtract, and requires none; a planted instance in a small kernel checks that the
scan finds it, and that mul_nc removes it."""
import collections
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

SOURCES = ("kernels_step.hip", "kernels_task.hip", "kernels_split.hip", "kernels_serve.hip",
           "kernels_adjoint.hip")

PLANTED = r'''
#include "fossen_device.h"
__global__ void planted(const float* x, float* y) {
  const float p = x[0] * x[1];          // product with a sum and a multiply among its uses
  y[0] = p + x[2];
  y[1] = p * x[3];
}
__global__ void fixed(const float* x, float* y) {
  const float p = mg::mul_nc(x[0], x[1]);
  y[0] = p + x[2];
  y[1] = p * x[3];
}
'''


def ambiguous_products(ir):
    """{kernel: count} of contractable fmuls with more than one use, one of which is a
    contractable fadd / fsub."""
    out = {}
    for name, body in re.findall(r"define [^@]*@(\S+?)\((.*?)\n}\n", ir, re.S):
        defs, order = {}, []
        for line in body.split("\n"):
            d = re.match(r"\s+(%\S+) = (.*)", line)
            if d:
                defs[d.group(1)] = d.group(2).split("!dbg")[0]
                order.append(d.group(1))
        uses = collections.defaultdict(list)
        for u in order:
            for v in re.findall(r"(%[\w.]+)", defs[u]):
                uses[v].append(u)
        n = sum(1 for v in order
                if defs[v].startswith("fmul contract") and len(uses[v]) > 1
                and any(defs[u].split()[0] in ("fadd", "fsub") and "contract" in defs[u]
                        for u in uses[v]))
        if n:
            out[name] = n
    return out


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        pytest.skip("hipcc not available")
    return h


def _ir_cmd(src, out):
    from paper_2410_14117_amd import build
    return [_hipcc(), "-S", "-emit-llvm", "--cuda-device-only", *build.CFLAGS, src, "-o", out]


@pytest.fixture(scope="module")
def kernel_ir(tmp_path_factory):
    from paper_2410_14117_amd import build
    d = tmp_path_factory.mktemp("ir")
    procs = {}
    for s in SOURCES:
        out = str(d / (s + ".ll"))
        procs[s] = (subprocess.Popen(_ir_cmd(os.path.join(build.CSRC, s), out),
                                     stderr=subprocess.DEVNULL), out)
    ir = {}
    for s, (p, out) in procs.items():
        assert p.wait(timeout=600) == 0, s
        ir[s] = open(out).read()
    return ir


@pytest.mark.parametrize("src", SOURCES)
def test_no_ambiguous_contraction(kernel_ir, src):
    found = ambiguous_products(kernel_ir[src])
    assert "define" in kernel_ir[src] and not found, found


def test_scan_finds_a_planted_instance(tmp_path):
    from paper_2410_14117_amd import build
    src = tmp_path / "planted.hip"
    src.write_text(PLANTED)
    out = str(tmp_path / "planted.ll")
    subprocess.check_call(_ir_cmd(str(src), out) + ["-I", build.CSRC],
                          stderr=subprocess.DEVNULL)
    found = ambiguous_products(open(out).read())
    assert any("planted" in k for k in found), found
    assert not any("fixed" in k for k in found), found
