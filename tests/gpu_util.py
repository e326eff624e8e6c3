"""Helpers for the GPU tests (device upload, the error norm of the tolerances)."""
import sys

import numpy as np

DEV = "cuda:0"


def say(*a):
    """Name the case before a GPU step, flushed, so a failure can be placed."""
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def rel_err(x_gpu, x_ref):
    """max over envs and components of |x_gpu - x_ref| / max(1, |x_ref|)."""
    x_gpu = np.asarray(x_gpu, dtype=np.float64)
    x_ref = np.asarray(x_ref, dtype=np.float64)
    return float(np.max(np.abs(x_gpu - x_ref) / np.maximum(1.0, np.abs(x_ref))))


# tolerances of the FP32 GPU path against the FP64 oracle
TOL_ONE_STEP = 1e-5      # one control step from identical inputs
TOL_TRAJ = 1e-3          # whole trajectory (1000 control steps)
