"""GPU check of mg_adj_backward_noalloc, the adjoint backward for callers that cannot
allocate device memory: its recomputation scratch is a static device array, and its
gradients must equal mg_adj_backward's bitwise (the same kernels run on the same inputs).
Two calls in a row, the second with fewer envs, fewer control steps and one segment;
then a call whose segment does not fit the static scratch is refused with nothing
written."""
import numpy as np
import pytest

from workloads import (BLUEROV2, BLUEROV2_HEAVY, vehicle_variant, initial_state, actions,
                       param_multipliers, env_classes)
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mgmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_14117_amd import mg
    mg.lib()
    return mg


def _both(mgmod, classes, E, T, K, S, seed, cls=None):
    """Gradients of one rollout from mg_adj_backward and from mg_adj_backward_noalloc,
    the latter written into buffers pre-filled with NaN (so that an element it does not
    write shows up)."""
    sim = mgmod.Sim(classes, E, 0.005, S, env_class=cls)
    D, N = sim.state_dim, sim.action_dim
    x0 = initial_state(E, D, seed)
    a = dev(actions(T, N, E, seed + 1) * np.float32(1.1))
    g = torch.empty((T, D, E), device="cuda").normal_(
        0.0, 1.0, generator=torch.Generator(device="cuda").manual_seed(seed + 2))
    sim.reset(state=dev(x0), param_mult=dev(param_multipliers(E, 0.2, seed + 3)))
    ckpt, _ = sim.adj_forward(a, K)
    ref = sim.adj_backward(ckpt, a, K, g)
    out = (torch.full((T, N, E), float("nan"), device="cuda"),
           torch.full((19, E), float("nan"), device="cuda"),
           torch.full((D, E), float("nan"), device="cuda"))
    got = sim.adj_backward(ckpt, a, K, g, out=out, noalloc=True)
    torch.cuda.synchronize()
    sim.close()
    return ref, got


def test_noalloc_backward_matches_allocating_backward(mgmod):
    """Call 1: 5000 mixed BlueROV2 / Heavy (lag, quadratic map) envs, 12 control steps
    of 4 sub-steps, checkpoint every 3 (whole-rollout recomputation, 4.9 MB per class
    segment).  Call 2, smaller: 700 Heavy envs, 5 control steps, checkpoint every 8 (one
    segment recomputed by the sweep kernel itself)."""
    classes = [vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05),
               vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)]
    cls = env_classes(5000, "bernoulli", 6101)
    say("noalloc backward call 1: E=5000 mixed, T=12, K=3, S=4")
    ref, got = _both(mgmod, classes, 5000, 12, 3, 4, 6110, cls)
    for r, o in zip(ref, got):
        assert torch.equal(r, o)
    say("noalloc backward call 2: E=700 Heavy, T=5, K=8, S=4")
    ref, got = _both(mgmod, classes[1], 700, 5, 8, 4, 6120)
    for r, o in zip(ref, got):
        assert torch.equal(r, o)


def test_noalloc_backward_refuses_a_segment_beyond_its_scratch(mgmod):
    """2^17 BlueROV2 envs, checkpoint every 16 of 1 sub-step: one segment's states are
    16 x 13 x 2^17 x 4 B = 109 MB > 64 MiB, so the call is refused before any launch and
    its outputs keep their contents."""
    from paper_2410_14117_amd.mg import MgError, MG_ERR_INVALID
    E, T, K = 1 << 17, 16, 16
    sim = mgmod.Sim(BLUEROV2, E, 0.01, 1)
    a = dev(actions(T, 6, E, 6130))
    g = torch.zeros((T, 13, E), device="cuda")
    ckpt, _ = sim.adj_forward(a, K)
    out = (torch.full((T, 6, E), 7.0, device="cuda"), torch.full((19, E), 7.0, device="cuda"),
           None)
    say("noalloc backward: segment beyond the static scratch (refused on the host)")
    with pytest.raises(MgError) as ei:
        sim.adj_backward(ckpt, a, K, g, want_x0=False, out=out, noalloc=True)
    assert ei.value.status == MG_ERR_INVALID
    torch.cuda.synchronize()
    assert bool((out[0] == 7.0).all()) and bool((out[1] == 7.0).all())
    sim.close()
