"""A small pass over every kernel family (fused and per-sub-step step, reset, Gym task,
split scheme, adjoint forward and both backward paths, serving join / tick / leave),
run with whichever libmg the binding loads (MG_LIBRARY selects libmg_debug.so).  Used
by tests/test_gpu_debug.py: in its own process for the debug build, in the test's
process for the release build.  Returns numpy arrays and the debug words.

    python tests/debug_workload.py OUT.npz     (writes the arrays and the words)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def run(E=3000):
    import torch
    from paper_2410_14117_amd import mg
    from workloads import (BLUEROV2, BLUEROV2_HEAVY, vehicle_variant, initial_state, actions,
                           param_multipliers)
    dev = "cuda:0"
    heavy = vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)
    out, words = {}, {}

    # mixed classes, interleaved (a non-identity internal order), 4 sub-steps of 5 ms
    cls = (np.arange(E) % 3 == 0).astype(np.int32)
    sim = mg.Sim([BLUEROV2, heavy], E, 0.005, 4, env_class=cls)
    D, N = sim.state_dim, sim.action_dim
    x0 = torch.from_numpy(initial_state(E, D, 901)).to(dev)
    mult = torch.from_numpy(param_multipliers(E, 0.2, 902)).to(dev)
    act = torch.from_numpy(actions(6, N, E, 903)).to(dev)
    sim.reset(state=x0, param_mult=mult)
    traj = torch.empty((5, D, E), device=dev)
    stats = torch.empty((5, 4), dtype=torch.float64, device=dev)
    sim.step(act[:5], traj=traj, stats=stats)
    out["fused_traj"], out["fused_stats"] = traj.cpu().numpy(), stats.cpu().numpy()
    sim.step(act[5:6], plain=True)
    out["plain_state"] = sim.get_state().cpu().numpy()
    sim.reset(env_ids=torch.arange(0, E, 7, device=dev), state=x0[:, ::7].contiguous())
    sim.rollout(act[:3])
    out["rollout_state"] = sim.get_state().cpu().numpy()
    sim.task_configure({"task": "circle", "lookahead": 4, "radius": 2.0, "omega": 0.5,
                        "episode_steps": 2},
                       center=torch.zeros(3, E, device=dev),
                       phase=torch.linspace(0, 6.0, E, device=dev))
    for k in range(3):
        obs, err, done = sim.task_step(act[k], reset_state=x0)
        out[f"task_obs{k}"], out[f"task_err{k}"] = obs.cpu().numpy(), err.cpu().numpy()
        out[f"task_done{k}"] = done.cpu().numpy()
    sim.reset(state=x0, param_mult=mult)
    sim.step_split(act[:2])
    out["split_state"] = sim.get_state().cpu().numpy()
    words["sim"] = sim.debug_word()
    sim.close()

    # adjoint: one sub-step per control step, trajectory-reading and recomputing backward
    Ea, T, K = 2000, 8, 4
    sa = mg.Sim(BLUEROV2, Ea, 0.01, 1)
    xa = torch.from_numpy(initial_state(Ea, 13, 904)).to(dev)
    aa = torch.from_numpy(actions(T, 6, Ea, 905)).to(dev)
    g = torch.from_numpy(np.random.default_rng(906).standard_normal((T, 13, Ea))
                         .astype(np.float32)).to(dev)
    sa.reset(state=xa)
    tra = torch.empty((T, 13, Ea), device=dev)
    ck, _ = sa.adj_forward(aa, K, traj=tra)
    for name, kw in (("traj", {"traj": tra}), ("recompute", {})):
        ga, gt, gx = sa.adj_backward(ck, aa, K, g, **kw)
        out[f"adj_{name}_act"], out[f"adj_{name}_theta"] = ga.cpu().numpy(), gt.cpu().numpy()
        out[f"adj_{name}_x0"] = gx.cpu().numpy()
    out["adj_traj"] = tra.cpu().numpy()
    words["adjoint"] = sa.debug_word()
    sa.close()

    # serving: a pointer-mode and a seed-mode request
    srv = mg.Server([BLUEROV2, heavy], 0.005, 4, steps_per_tick=2)
    Ds = srv.state_dim
    n1, n2, L = 300, 200, 3
    xs = torch.from_numpy(initial_state(n1, Ds, 907)).to(dev)
    acs = torch.from_numpy(actions(L, srv.action_dim, n1, 908)).to(dev)
    o1 = np.zeros((Ds, n1), np.float32)
    o2 = np.zeros((Ds, n2), np.float32)
    st1, t1 = srv.submit(n1, L, xs.data_ptr(), acs.data_ptr(), n1, o1,
                         env_class=np.arange(n1) % 2)
    st2, t2 = srv.submit(n2, L, xs.data_ptr(), 0, n1, o2, action_seed=909)
    assert st1 == 0 and st2 == 0
    assert srv.wait(t1)[0] == 0 and srv.wait(t2)[0] == 0
    out["serve_ptr"], out["serve_seed"] = o1, o2
    words["server"] = srv.debug_word()
    srv.close()
    torch.cuda.synchronize()
    return out, words


if __name__ == "__main__":
    res, w = run()
    np.savez(sys.argv[1], **res, **{f"word_{k}": np.uint32(v) for k, v in w.items()})
    print("debug workload done:", {k: int(v) for k, v in w.items()}, flush=True)
