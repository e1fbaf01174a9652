"""Adjoint of the entropy-conserving / Roe pair (Chandrashekar volume flux,
Roe surface flux with the Harten-Hyman correction) on the GPU against the
oracle (FP64).

* dg_eval_rhs_vjp vs the oracle's reverse mode, per variable rel L2 <= 1e-11,
  with density and pressure spreads of 20 % (most logarithmic means take the
  atanh form) and of 0.4 % (all take the series), periodic and wall ends,
  N = 3, 5, 7, with and without viscosity and Roe dissipation;
* <Ubar, v> vs <lam, (dL/dU) v> with the oracle's complex-step JVP;
* dg_rk_step_vjp through one RK step, and the kinetic-energy gradient of a
  checkpointed rollout, vs the oracle's reverse mode.
"""

import numpy as np
import pytest
import torch

from oracle.adjoint import rhs_jvp_cs, rhs_vjp, rollout_grad
from oracle.dgsem import rk_step
from oracle.mesh import Mesh
from oracle.physics import Gas
from paper_2606_18927_amd import dgsem, workloads
from paper_2606_18927_amd.autograd import kinetic_energy_gradient

from _cases import random_faces, random_state
from _gpu import custom, need_gpu, oracle_gas, oracle_mesh, rel_l2, say, state, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-11
EC = dict(flux="ec_roe")
P3 = ("periodic",) * 3
WY = ("periodic", "wall", "periodic")


def _case(N, n, bc, seed, amp=0.2, mu=0.01):
    rng = np.random.default_rng(seed)
    faces = [random_faces(n[d], -1.0, 1.0, rng) if bc[d] == "wall" else random_faces(n[d], 0.0, 2.0 + d, rng)
             for d in range(3)]
    mesh = Mesh(N, tuple(faces), bc=bc, T_wall=1.1)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=mu, Pr=0.72)
    U = random_state(mesh, g.gamma, g.R, rng, vel_amp=1.0, p_mean=1.0 / (1.4 * 0.01), p_amp=amp, rho_amp=amp)
    lam = rng.standard_normal(U.shape)
    return mesh, g, U.numpy(), lam


def _solver(mesh, g, **kw):
    spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall)
    return dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, flux="ec_roe", with_adjoint=True, **kw)


@pytest.mark.parametrize("N,n,bc,amp", [
    (3, (3, 2, 3), P3, 0.2),
    (3, (2, 3, 2), WY, 0.2),
    (5, (2, 3, 2), WY, 0.2),
    (5, (2, 2, 3), P3, 0.004),
    (7, (2, 2, 2), ("wall", "periodic", "periodic"), 0.2),
])
def test_ec_rhs_vjp_against_oracle(N, n, bc, amp):
    need_gpu()
    say("ec vjp case", N, n, bc, amp)
    mesh, g, U, lam = _case(N, n, bc, seed=61 + N, amp=amp)
    S = _solver(mesh, g)
    got = S.eval_rhs_vjp(to_dev(U), to_dev(lam)).cpu().numpy()
    S.sync()
    ref = rhs_vjp(torch.as_tensor(U), torch.as_tensor(lam), mesh, g, **EC).numpy()
    e = rel_l2(got, ref)
    say("  rel L2", e)
    assert np.all(e < TOL)
    # the pair's derivative matters: the Kennedy-Gruber / Lax-Friedrichs VJP differs
    ref_kg = rhs_vjp(torch.as_tensor(U), torch.as_tensor(lam), mesh, g).numpy()
    assert np.max(rel_l2(ref_kg, ref)) > 1e3 * TOL


@pytest.mark.parametrize("viscous,central", [(False, False), (False, True), (True, True)])
def test_ec_rhs_vjp_switches(viscous, central):
    need_gpu()
    mesh, g, U, lam = _case(3, (2, 3, 2), WY, seed=8)
    S = _solver(mesh, g, viscous=viscous, central_only=central)
    got = S.eval_rhs_vjp(to_dev(U), to_dev(lam)).cpu().numpy()
    S.sync()
    ref = rhs_vjp(torch.as_tensor(U), torch.as_tensor(lam), mesh, g, viscous=viscous,
                  central_only=central, **EC).numpy()
    e = rel_l2(got, ref)
    say("ec switches", viscous, central, e)
    assert np.all(e < TOL)


def test_ec_vjp_dot_product_with_complex_step_jvp():
    need_gpu()
    mesh, g, U, lam = _case(5, (2, 2, 2), ("periodic", "periodic", "wall"), seed=29)
    rng = np.random.default_rng(30)
    S = _solver(mesh, g)
    Ubar = S.eval_rhs_vjp(to_dev(U), to_dev(lam)).cpu().numpy()
    S.sync()
    for _ in range(3):
        v = rng.standard_normal(U.shape)
        jv = rhs_jvp_cs(torch.as_tensor(U), torch.as_tensor(v), mesh, g, **EC).numpy()
        lhs, rhs_ = float((lam * jv).sum()), float((Ubar.reshape(U.shape) * v).sum())
        say("ec dot", lhs, rhs_)
        assert abs(lhs - rhs_) < 1e-11 * (abs(lhs) + 1.0)


def test_ec_rk_step_vjp_against_oracle():
    need_gpu()
    wl = custom("tgv", 3, (3, 3, 2), noise=0.01, seed=3, flux="ec_roe")
    U, dt = state(wl)
    mesh, g = oracle_mesh(wl), oracle_gas(wl)
    lam = np.random.default_rng(33).standard_normal(U.shape)
    Ut = torch.as_tensor(U).requires_grad_(True)
    (ref,) = torch.autograd.grad(rk_step(Ut, mesh, g, dt, 1, **EC), Ut, grad_outputs=torch.as_tensor(lam))
    S = dgsem.solver_for(wl, with_adjoint=True)
    got = S.rk_step_vjp(to_dev(U), dt, to_dev(lam)).cpu().numpy()
    S.sync()
    e = rel_l2(got, ref.numpy())
    d = rel_l2(got - lam.reshape(got.shape), ref.numpy() - lam)
    say("ec rk vjp rel L2", e, "minus identity", d)
    assert np.all(e < TOL)
    assert np.all(d < 1e-9)


def test_ec_rollout_kinetic_energy_gradient_against_oracle():
    need_gpu()
    wl = custom("channel", 3, (2, 3, 2), seed=workloads.CHANNEL_SEED, flux="ec_roe")
    U, dt = state(wl)
    mesh, g = oracle_mesh(wl), oracle_gas(wl)
    nsteps = 6
    Jref, gref = rollout_grad(torch.as_tensor(U), mesh, g, dt, nsteps, **EC)
    S = dgsem.solver_for(wl, with_adjoint=True)
    J, grad = kinetic_energy_gradient(S, to_dev(U), dt, nsteps, checkpoint_every=4)
    J = J.item()
    say("ec J", J, Jref.item())
    assert abs(J - Jref.item()) < 1e-13 * abs(Jref.item())
    e = rel_l2(grad.cpu().numpy(), gref.numpy())
    say("ec rollout gradient rel L2", e)
    assert np.all(e < 1e-10)
