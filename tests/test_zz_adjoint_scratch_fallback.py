"""GPU check of mg_adj_backward's fallback when device memory has no room for the
whole rollout's recomputation buffer.  Collected last: it fills device memory with one
large allocation (released before it returns, whatever happens)."""
import pytest

from workloads import BLUEROV2_HEAVY, vehicle_variant, initial_state, actions
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


def test_segment_scratch_when_whole_rollout_does_not_fit(mgmod):
    """When device memory leaves no room for the whole rollout's recomputation buffer,
    mg_adj_backward recomputes segment by segment in a segment-sized buffer instead of
    failing, with the same gradients, bitwise.  The memory is taken by one large torch
    allocation, leaving the segment buffer plus 1.5 GB for the gradients and the runtime."""
    v = vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)
    E, T, K, S, D = 1 << 17, 64, 8, 4, 21
    whole_bytes = T * S * D * E * 4
    seg_bytes = K * S * D * E * 4
    x0 = dev(initial_state(E, D, 351))
    a = dev(actions(T, 8, E, 352))
    g = torch.empty((T, D, E), device="cuda").normal_(
        0.0, 1.0, generator=torch.Generator(device="cuda").manual_seed(353))

    def grads(sim, fill=False):
        sim.reset(state=x0)
        ckpt, _ = sim.adj_forward(a, K)
        filler = None
        try:
            if fill:
                torch.cuda.synchronize()
                free = torch.cuda.mem_get_info()[0]
                filler = torch.empty(free - seg_bytes - (3 << 29), dtype=torch.uint8,
                                     device="cuda")
                assert torch.cuda.mem_get_info()[0] < whole_bytes
            out = sim.adj_backward(ckpt, a, K, g)
            torch.cuda.synchronize()
        finally:
            del filler      # released whatever happens, so later tests have the memory
        return out

    say(f"adjoint scratch E={E}: whole-rollout buffer")
    sim1 = mgmod.Sim(v, E, 0.005, S)
    ref = grads(sim1)
    sim1.close()
    say(f"adjoint scratch E={E}: device memory filled, segment buffer")
    sim2 = mgmod.Sim(v, E, 0.005, S)
    try:
        got = grads(sim2, fill=True)
    finally:
        sim2.close()
        torch.cuda.empty_cache()
    for r, o in zip(ref, got):
        assert torch.equal(r, o)
