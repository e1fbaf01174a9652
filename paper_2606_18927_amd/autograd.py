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


def _segments_to_record(solver: Solver, nsteps: int, K: int, stage_memory_bytes) -> int:
    """How many trailing segments record their stages in the forward pass:
    those whose (K, 5, 5 n_dof) buffers fit in stage_memory_bytes (None: one,
    the buffer the backward pass needs anyway)."""
    nseg = -(-nsteps // K)
    if stage_memory_bytes is None:
        return 1
    per = K * 25 * solver.n_dof * 8
    return max(1, min(nseg, int(stage_memory_bytes // per)))


def _forward_states(solver: Solver, U0: torch.Tensor, dt: float, nsteps: int, K: int,
                    record_stages: bool = True, stage_memory_bytes=None):
    """Run the rollout; return U_T, the checkpoints {step: state} and, with
    record_stages, {segment start: stage-state buffer (K, 5, 5 n_dof)} of the
    trailing segments recorded during the forward pass, which the backward
    pass then does not recompute (same kernels, same states)."""
    ckpts = {0: U0.detach().clone()}
    solver.set_state(U0)
    nrec = _segments_to_record(solver, nsteps, K, stage_memory_bytes) if record_stages else 0
    first_rec = (-(-nsteps // K) - nrec) * K  # start of the first recorded segment
    bufs = {}
    done = 0
    while done < nsteps:
        n = min(K, nsteps - done)
        if record_stages and done >= first_rec:
            bufs[done] = torch.empty((K, 5, 5 * solver.n_dof), dtype=torch.float64, device=U0.device)
            solver.rk_record_stages(ckpts[done], dt, n, out=bufs[done])
        else:
            solver.rk_step(dt, n)
        done += n
        if done < nsteps:
            ckpts[done] = solver.get_state()
    UT = solver.get_state()
    solver.sync()
    return UT, ckpts, bufs


def _backward_states(solver: Solver, ckpts: dict, dt: float, nsteps: int, K: int,
                     lam_T: torch.Tensor, record_stages: bool = True, bufs=None) -> torch.Tensor:
    """lam_0 from lam_T; `bufs` holds the stage states recorded in the forward
    pass ({segment start: buffer}); other segments are recomputed into one of
    those buffers once it has been consumed."""
    lam = lam_T.detach().clone().contiguous()
    spare = torch.empty_like(lam)
    starts = sorted(ckpts)
    bufs = dict(bufs or {})
    buf = None
    for s0 in reversed(starts):
        s1 = min(s0 + K, nsteps)
        if record_stages:
            if s0 in bufs:
                buf = bufs.pop(s0)
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
    def forward(ctx, U0, solver, dt, nsteps, checkpoint_every, record_stages=True, stage_memory_bytes=None):
        K = max(1, int(checkpoint_every) if checkpoint_every else nsteps)
        UT, ckpts, bufs = _forward_states(solver, U0.contiguous(), dt, nsteps, K, bool(record_stages),
                                          stage_memory_bytes)
        ctx.solver, ctx.dt, ctx.nsteps, ctx.K, ctx.ckpts, ctx.bufs = solver, dt, nsteps, K, ckpts, bufs
        ctx.record_stages = bool(record_stages)
        return UT

    @staticmethod
    def backward(ctx, gUT):
        lam0 = _backward_states(ctx.solver, ctx.ckpts, ctx.dt, ctx.nsteps, ctx.K, gUT,
                                ctx.record_stages, ctx.bufs)
        ctx.ckpts = ctx.bufs = None
        return lam0, None, None, None, None, None, None


def rollout(U0: torch.Tensor, solver: Solver, dt: float, nsteps: int, checkpoint_every: int = 0,
            record_stages: bool = True, stage_memory_bytes=None):
    """U_T of the rollout with the checkpointed backward pass.  stage_memory_bytes
    lets the forward pass record the stages of as many trailing segments as fit
    (K 25 n_dof doubles each; default: one), which are then not recomputed."""
    return RKRollout.apply(U0, solver, dt, nsteps, checkpoint_every, record_stages, stage_memory_bytes)


def kinetic_energy_gradient(solver: Solver, U0: torch.Tensor, dt: float, nsteps: int,
                            checkpoint_every: int = 0, record_stages: bool = True, stage_memory_bytes=None):
    """(J(U_T), dJ/dU0) for the volume-averaged kinetic energy J after nsteps
    (stage_memory_bytes as in ``rollout``)."""
    K = max(1, checkpoint_every or nsteps)
    UT, ckpts, bufs = _forward_states(solver, U0.contiguous(), dt, nsteps, K, record_stages,
                                      stage_memory_bytes)
    J = solver.kinetic_energy(UT)
    lam_T = solver.kinetic_energy_grad(UT)
    lam0 = _backward_states(solver, ckpts, dt, nsteps, K, lam_T, record_stages, bufs)
    return J, lam0
