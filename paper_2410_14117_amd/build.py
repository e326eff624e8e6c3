"""Builds libmg.so in-tree with hipcc for gfx950.

    python -m paper_2410_14117_amd.build

Every .hip file under csrc/ is compiled to an object under _build/ and the
objects are linked into paper_2410_14117_amd/libmg.so; the serving client
driver (clients/replay.cpp, host code) becomes libmg_clients.so beside it.  Packed FP32 math is
switched off (-packed-fp32-ops) for all device code.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmg.so")
DEBUG_LIB = os.path.join(HERE, "libmg_debug.so")   # bounds-checked build (-DMG_DEBUG)
CLIENTS_LIB = os.path.join(HERE, "libmg_clients.so")
ARCH = os.environ.get("MG_OFFLOAD_ARCH", "gfx950")

CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function"]


def _hipcc():
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if p and (os.path.sep not in p or os.path.exists(p)):
            return p
    return "hipcc"


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src, extra=(), build_dir=BUILD):
    obj = os.path.join(build_dir, os.path.basename(src)[:-4] + ".o")
    cmd = [_hipcc(), "-c", *CFLAGS, *extra, src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=True, out=None, build_dir=None, defines=()):
    """Compile and link; `out`/`build_dir`/`defines` allow side builds of tuning variants."""
    bdir = build_dir or BUILD
    os.makedirs(bdir, exist_ok=True)
    extra = [f"-D{d}" for d in defines]
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, extra, bdir), srcs))
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib} from {len(srcs)} sources")
    if out is None:
        build_clients(verbose)
    return lib


def build_clients(verbose=True):
    """The serving client driver (clients/replay.cpp) as libmg_clients.so, a host-only
    library linked against libmg.so (found beside it at run time)."""
    src = os.path.join(HERE, "clients", "replay.cpp")
    tmp = CLIENTS_LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-Wall", "-I",
           os.path.join(ROOT, "include"), src, "-o", tmp, "-L", HERE, "-lmg",
           "-Wl,-rpath,$ORIGIN", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"client driver build failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, CLIENTS_LIB)
    if verbose:
        print(f"built {CLIENTS_LIB}")


def build_debug(verbose=True):
    """The bounds-checked build of the same sources (-DMG_DEBUG) as libmg_debug.so: same
    entry points and results, kernels that check every lane's indices (include/mg.h)."""
    return build(verbose, out=DEBUG_LIB, build_dir=BUILD + "_debug", defines=("MG_DEBUG",))


if __name__ == "__main__":
    if "--debug" in sys.argv[1:]:
        build_debug()
    else:
        build()
    sys.exit(0)
