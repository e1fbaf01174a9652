"""Gradients through the RK rollout: torch.autograd.Function over the C ABI.

``RKRollout.apply(U0, solver, dt, nsteps, checkpoint_every)`` advances U0 by
``nsteps`` RK steps with ``dg_rk_step`` and returns U_T.  Its backward pass
goes back step by step with the RK step's vector-Jacobian product.  States
are checkpointed every ``checkpoint_every`` (K) steps during the forward pass;
the backward pass recomputes one segment at a time from its checkpoint.  By
default (``record_stages``) the recompute writes the five stage states of every
step of the segment (``dg_rk_record_stages``, 25 n_dof doubles per step) and
the reverse steps read them (``dg_rk_step_vjp_stages``): one forward pass per
segment, memory (nsteps / K) checkpoints + 5 K states.  The last segment,
reversed first, is recorded already during the forward pass into the same
buffer, so it is never recomputed (the buffer is then held from the forward
to the backward pass).  Without it the segment
keeps its K step states and ``dg_rk_step_vjp`` recomputes each step's stages:
K states, one more forward pass.

``kinetic_energy_gradient`` is the flow functional used for the adjoint: the
volume-averaged kinetic energy of U_T and its gradient with respect to the
nodal initial state.
"""

from __future__ import annotations

import torch

from .dgsem import Solver

__all__ = ["RKRollout", "rollout", "kinetic_energy_gradient"]


def _forward_states(solver: Solver, U0: torch.Tensor, dt: float, nsteps: int, K: int,
                    record_stages: bool = True):
    """Run the rollout; return U_T, the checkpoints {step: state} and, with
    record_stages, the stage-state buffer (K, 5, 5 n_dof) holding the last
    segment's stages: that segment is recorded during the forward pass, so
    the backward pass does not recompute it (same kernels, same states)."""
    ckpts = {0: U0.detach().clone()}
    solver.set_state(U0)
    buf = None
    done = 0
    while done < nsteps:
        n = min(K, nsteps - done)
        if record_stages and done + n == nsteps:
            buf = torch.empty((K, 5, 5 * solver.n_dof), dtype=torch.float64, device=U0.device)
            solver.rk_record_stages(ckpts[done], dt, n, out=buf)
        else:
            solver.rk_step(dt, n)
        done += n
        if done < nsteps:
            ckpts[done] = solver.get_state()
    UT = solver.get_state()
    solver.sync()
    return UT, ckpts, buf


def _backward_states(solver: Solver, ckpts: dict, dt: float, nsteps: int, K: int,
                     lam_T: torch.Tensor, record_stages: bool = True, buf=None) -> torch.Tensor:
    """lam_0 from lam_T; `buf`, if given, holds the last segment's recorded
    stage states (from the forward pass)."""
    lam = lam_T.detach().clone().contiguous()
    spare = torch.empty_like(lam)
    starts = sorted(ckpts)
    last = starts[-1]
    for s0 in reversed(starts):
        s1 = min(s0 + K, nsteps)
        if record_stages:
            if s0 == last and buf is not None:
                stages = buf[: s1 - s0]
            else:
                if buf is None:
                    buf = torch.empty((K, 5, 5 * solver.n_dof), dtype=torch.float64, device=lam.device)
                stages = solver.rk_record_stages(ckpts[s0], dt, s1 - s0, out=buf)
            for n in range(s1 - 1, s0 - 1, -1):
                solver.rk_step_vjp_stages(stages[n - s0], dt, lam, out=spare)
                lam, spare = spare, lam
            continue
        # recompute the step states of the segment [s0, s1)
        states = [ckpts[s0]]
        solver.set_state(ckpts[s0])
        for _ in range(s0 + 1, s1):
            solver.rk_step(dt, 1)
            states.append(solver.get_state())
        for n in range(s1 - 1, s0 - 1, -1):
            solver.rk_step_vjp(states[n - s0], dt, lam, out=spare)
            lam, spare = spare, lam
        del states
    solver.sync()
    return lam


class RKRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dt, nsteps, checkpoint_every, record_stages=True):
        K = max(1, int(checkpoint_every) if checkpoint_every else nsteps)
        UT, ckpts, buf = _forward_states(solver, U0.contiguous(), dt, nsteps, K, bool(record_stages))
        ctx.solver, ctx.dt, ctx.nsteps, ctx.K, ctx.ckpts, ctx.buf = solver, dt, nsteps, K, ckpts, buf
        ctx.record_stages = bool(record_stages)
        return UT

    @staticmethod
    def backward(ctx, gUT):
        lam0 = _backward_states(ctx.solver, ctx.ckpts, ctx.dt, ctx.nsteps, ctx.K, gUT,
                                ctx.record_stages, ctx.buf)
        ctx.ckpts = ctx.buf = None
        return lam0, None, None, None, None, None


def rollout(U0: torch.Tensor, solver: Solver, dt: float, nsteps: int, checkpoint_every: int = 0,
            record_stages: bool = True):
    return RKRollout.apply(U0, solver, dt, nsteps, checkpoint_every, record_stages)


def kinetic_energy_gradient(solver: Solver, U0: torch.Tensor, dt: float, nsteps: int,
                            checkpoint_every: int = 0, record_stages: bool = True):
    """(J(U_T), dJ/dU0) for the volume-averaged kinetic energy J after nsteps."""
    K = max(1, checkpoint_every or nsteps)
    UT, ckpts, buf = _forward_states(solver, U0.contiguous(), dt, nsteps, K, record_stages)
    J = solver.kinetic_energy(UT)
    lam_T = solver.kinetic_energy_grad(UT)
    lam0 = _backward_states(solver, ckpts, dt, nsteps, K, lam_T, record_stages, buf)
    return J, lam0
