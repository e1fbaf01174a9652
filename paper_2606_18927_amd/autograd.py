"""Gradients through the RK rollout: torch.autograd.Function over the C ABI.

``RKRollout.apply(U0, solver, dt, nsteps, checkpoint_every)`` advances U0 by
``nsteps`` RK steps with ``dg_rk_step`` and returns U_T.  Its backward pass
applies ``dg_rk_step_vjp`` step by step in reverse.  States are checkpointed
every ``checkpoint_every`` steps during the forward pass; the backward pass
recomputes the states of one segment at a time from its checkpoint, so the
memory held is (nsteps / K) checkpoints plus K states of one segment, and each
step's five stage states live only inside ``dg_rk_step_vjp``.

``kinetic_energy_gradient`` is the flow functional used for the adjoint: the
volume-averaged kinetic energy of U_T and its gradient with respect to the
nodal initial state.
"""

from __future__ import annotations

import torch

from .dgsem import Solver

__all__ = ["RKRollout", "rollout", "kinetic_energy_gradient"]


def _forward_states(solver: Solver, U0: torch.Tensor, dt: float, nsteps: int, K: int):
    """Run the rollout; return U_T and the checkpoints {step: state}."""
    ckpts = {0: U0.detach().clone()}
    solver.set_state(U0)
    done = 0
    while done < nsteps:
        n = min(K, nsteps - done)
        solver.rk_step(dt, n)
        done += n
        if done < nsteps:
            ckpts[done] = solver.get_state()
    UT = solver.get_state()
    solver.sync()
    return UT, ckpts


def _backward_states(solver: Solver, ckpts: dict, dt: float, nsteps: int, K: int,
                     lam_T: torch.Tensor) -> torch.Tensor:
    lam = lam_T.detach().clone().contiguous()
    starts = sorted(ckpts)
    for s0 in reversed(starts):
        s1 = min(s0 + K, nsteps)
        # recompute the states of the segment [s0, s1)
        states = [ckpts[s0]]
        solver.set_state(ckpts[s0])
        for _ in range(s0 + 1, s1):
            solver.rk_step(dt, 1)
            states.append(solver.get_state())
        for n in range(s1 - 1, s0 - 1, -1):
            lam = solver.rk_step_vjp(states[n - s0], dt, lam)
        del states
    solver.sync()
    return lam


class RKRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dt, nsteps, checkpoint_every):
        K = max(1, int(checkpoint_every) if checkpoint_every else nsteps)
        UT, ckpts = _forward_states(solver, U0.contiguous(), dt, nsteps, K)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.K, ctx.ckpts = solver, dt, nsteps, K, ckpts
        return UT

    @staticmethod
    def backward(ctx, gUT):
        lam0 = _backward_states(ctx.solver, ctx.ckpts, ctx.dt, ctx.nsteps, ctx.K, gUT)
        ctx.ckpts = None
        return lam0, None, None, None, None


def rollout(U0: torch.Tensor, solver: Solver, dt: float, nsteps: int, checkpoint_every: int = 0):
    return RKRollout.apply(U0, solver, dt, nsteps, checkpoint_every)


def kinetic_energy_gradient(solver: Solver, U0: torch.Tensor, dt: float, nsteps: int,
                            checkpoint_every: int = 0):
    """(J(U_T), dJ/dU0) for the volume-averaged kinetic energy J after nsteps."""
    K = max(1, checkpoint_every or nsteps)
    UT, ckpts = _forward_states(solver, U0.contiguous(), dt, nsteps, K)
    J = solver.kinetic_energy(UT)
    lam_T = solver.kinetic_energy_grad(UT)
    lam0 = _backward_states(solver, ckpts, dt, nsteps, K, lam_T)
    return J, lam0
