"""torch.autograd.Function over the library's hand-written RK4 adjoint.

``rollout(sim, x0, actions, hydro, rigid, ckpt_every)`` returns the trajectory
[T][D][E] (state after each control step) and differentiates, through the
exact discrete map of the fused step kernel, with respect to the initial state
x0 [D][E], the throttles [T][N_max][E] and the hydrodynamic parameters
``hydro`` [19][E] = (M_A(6), D_L(6), D_Q(6), B) in absolute units.  ``rigid``
[4][E] = (m, Ixx, Iyy, Izz) is an input without gradient.  Both passes run in
libmg's kernels (mg_adj_forward / mg_adj_backward); torch only owns memory.
"""
import torch


class FossenRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, actions, hydro, rigid, sim, ckpt_every):
        params = torch.cat([rigid.detach(), hydro.detach()], dim=0).contiguous()
        actions = actions.detach().contiguous()
        sim.set_params(params)
        sim.set_state(x0.detach().contiguous())
        T = actions.shape[0]
        traj = torch.empty((T, sim.state_dim, sim.n_envs), dtype=torch.float32,
                           device=actions.device)
        ckpt, _ = sim.adj_forward(actions, ckpt_every, traj=traj)
        ctx.save_for_backward(ckpt, actions, params, traj)
        ctx.sim = sim
        ctx.ckpt_every = int(ckpt_every)
        return traj

    @staticmethod
    def backward(ctx, g_traj):
        ckpt, actions, params, traj = ctx.saved_tensors
        sim = ctx.sim
        sim.set_params(params)      # the sim may have been used in between
        # with one sub-step per control step the backward reads each step's input
        # from the trajectory instead of recomputing it
        gact, gth, gx0 = sim.adj_backward(ckpt, actions, ctx.ckpt_every,
                                          g_traj.to(torch.float32).contiguous(), traj=traj)
        return gx0, gact, gth, None, None, None


def rollout(sim, x0, actions, hydro, rigid, ckpt_every=8):
    return FossenRollout.apply(x0, actions, hydro, rigid, sim, ckpt_every)
