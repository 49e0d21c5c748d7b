"""torch.autograd.Function over a taped rollout: forward runs sim_rollout with
a tape, backward runs sim_backward (the discrete adjoint kernels)."""
from __future__ import annotations

import torch


class RolloutFn(torch.autograd.Function):
    """(actor [13828], theta [8][N]) -> (states [T+1][17][N], rewards [T][N]).

    The rollout starts from the simulator's current state, which is held
    fixed (no gradient flows to it).  theta is written into the simulator
    before the rollout."""

    @staticmethod
    def forward(ctx, actor, theta, sim, T):
        a = actor.detach().contiguous()
        sim.set_params(theta.detach())
        out = sim.rollout(a, T, rewards=True, dones=False, states=True, record_tape=True)
        ctx.sim = sim
        ctx.T = T
        ctx.tape_gen = sim.tape_gen
        ctx.save_for_backward(a)
        return out["states"], out["rewards"]

    @staticmethod
    def backward(ctx, d_states, d_rewards):
        (a,) = ctx.saved_tensors
        sim = ctx.sim
        # the handle holds one tape: refuse to differentiate another rollout's
        if sim.tape_gen != ctx.tape_gen or sim.tape_T != ctx.T:
            raise RuntimeError("the simulator's tape no longer belongs to this rollout (another "
                               "taped rollout, or a call that drops the tape, came in between); "
                               "run the backward before the next rollout on the same handle")
        # a NULL reward cotangent means "all ones" at the C ABI, so an absent
        # one is passed as explicit zeros
        if d_rewards is None:
            d_rewards = torch.zeros(ctx.T, sim.N, dtype=torch.float32, device=a.device)
        dS = None if d_states is None else d_states.contiguous().float()
        ga, gp = sim.backward(a, d_rewards=d_rewards.contiguous().float(), d_states=dS)
        return ga, gp, None, None


def rollout(sim, actor, theta, T):
    """Differentiable rollout: returns (states, rewards)."""
    return RolloutFn.apply(actor, theta, sim, T)
