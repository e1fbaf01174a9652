"""Sutherland's viscosity law on the GPU against the oracle (FP64).

mu(T) = mu (T / T_ref)^(3/2) (T_ref + S) / (T + S) at every node (the paper's
law for its working fluid, Sec. 4), with air's S / T_ref = 110.4 K / 288.15 K.
Right-hand side: relative L2 <= 1e-12 per variable on random states (T varies
by about 40 % across nodes) at N = 3, 5, 7, periodic and between isothermal
walls, with both flux pairs; five RK steps; the wall-model stress and the
operator with wall-model ends (mu at the wall temperature); the rejected
constants.
"""

import numpy as np
import pytest
import torch

from oracle.dgsem import rhs, rk_step
from oracle.mesh import Mesh, tanh_faces, uniform_faces
from oracle.physics import Gas
from oracle.wallmodel import wall_stress_field
from paper_2606_18927_amd import dgsem

from _cases import random_faces, random_state
from _gpu import need_gpu, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12
T_REF, S_AIR = 1.0, 110.4 / 288.15
R_GAS = 1.0 / (1.4 * 0.01)  # Ma = 0.1 units, T ~ 1


def _gas(mu=2e-3):
    return Gas(gamma=1.4, R=R_GAS, mu=mu, Pr=0.72, sutherland=True, T_ref=T_REF, S=S_AIR)


def _solver(mesh, g, **kw):
    spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall, mesh.wm_node)
    return dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, sutherland=(g.T_ref, g.S), **kw)


def _state(mesh, rng):
    return random_state(mesh, 1.4, R_GAS, rng, vel_amp=1.0, p_mean=R_GAS, p_amp=0.2, rho_amp=0.2).numpy()


@pytest.mark.parametrize("N,n,bc,flux", [
    (3, (2, 3, 2), ("periodic",) * 3, "kg_llf"),
    (5, (2, 2, 3), ("periodic", "wall", "periodic"), "kg_llf"),
    (7, (2, 2, 2), ("wall", "periodic", "wall"), "kg_llf"),
    (3, (3, 2, 2), ("periodic", "wall", "periodic"), "ec_roe"),
    (5, (2, 2, 2), ("periodic",) * 3, "ec_roe"),
])
def test_sutherland_rhs_against_oracle(N, n, bc, flux):
    need_gpu()
    say("sutherland rhs", N, n, bc, flux)
    rng = np.random.default_rng(70 + N)
    lo = [-1.0 if b != "periodic" else 0.0 for b in bc]
    mesh = Mesh(N, tuple(random_faces(n[d], lo[d], lo[d] + 2.0, rng) for d in range(3)), bc=bc, T_wall=1.2)
    g = _gas()
    U = _state(mesh, rng)
    S = _solver(mesh, g, flux=flux)
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = rhs(torch.as_tensor(U), mesh, g, flux=flux).numpy()
    e = rel_l2(got, ref)
    say("  rel L2", e)
    assert np.all(e < TOL)
    # the law matters for this state: the constant-viscosity operator differs
    ref0 = rhs(torch.as_tensor(U), mesh, Gas(gamma=1.4, R=R_GAS, mu=g.mu, Pr=0.72), flux=flux).numpy()
    assert np.all(rel_l2(ref0, ref)[1:] > 1e3 * TOL)


def test_sutherland_rk_steps():
    need_gpu()
    rng = np.random.default_rng(5)
    mesh = Mesh(3, (uniform_faces(3, 0, 2 * np.pi), tanh_faces(3, 2.0), uniform_faces(2, 0, np.pi)),
                bc=("periodic", "wall", "periodic"), T_wall=1.0)
    g = _gas()
    X, Y, Z = [c.numpy() for c in mesh.coords()]
    rho = 1.0 + 0.1 * np.sin(X) * np.cos(2 * Z)
    u = 1.2 * (1 - Y * Y) * (1 + 0.05 * np.sin(Z))
    v = 0.05 * np.sin(X) * (1 - Y * Y)
    w = 0.05 * np.cos(2 * Z) * (1 - Y * Y)
    p = R_GAS * (1.0 + 0.05 * np.cos(X + Y))
    E = p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)
    U = np.stack([rho, rho * u, rho * v, rho * w, E])
    dt, nsteps = 2e-4, 5
    S = _solver(mesh, g)
    S.set_state(to_dev(U))
    S.rk_step(dt, nsteps)
    S.sync()
    got = S.get_state().cpu().numpy().reshape(U.shape)
    ref = rk_step(torch.as_tensor(U), mesh, g, dt, nsteps).numpy()
    e, e2 = rel_l2(got, ref), rel_l2(got - U, ref - U)
    say("sutherland 5 RK steps rel L2", e, "increment", e2)
    assert np.all(e < TOL) and np.all(e2 < 1e-9)


def test_sutherland_wall_model():
    need_gpu()
    rng = np.random.default_rng(11)
    mesh = Mesh(5, (uniform_faces(2, 0, 2 * np.pi), tanh_faces(4, 2.0), uniform_faces(2, 0, np.pi)),
                bc=("periodic", "wallmodel", "periodic"), T_wall=1.0, wm_node=2)
    g = _gas(mu=1e-4)
    U = _state(mesh, rng)
    S = _solver(mesh, g)
    tau = S.wall_stress(to_dev(U), 2).cpu().numpy()
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    tref = wall_stress_field(torch.as_tensor(U), mesh, g, 2, g.mu_of)
    err = np.abs(tau - tref).max() / np.abs(tref).max()
    say("sutherland wall stress rel err", err)
    assert err < 1e-13
    e = rel_l2(got, rhs(torch.as_tensor(U), mesh, g).numpy())
    say("sutherland wall-model rhs rel L2", e)
    assert np.all(e < TOL)


def test_sutherland_rejected_combinations():
    need_gpu()
    mesh = Mesh(3, (uniform_faces(2, 0, 1),) * 3)
    g = _gas()
    # (mixed precision covers Sutherland's law: tests/test_gpu_mixed_physics.py;
    # the adjoint: tests/test_gpu_adjoint.py)
    for T_ref, Sg in ((0.0, 0.3), (1.0, -0.1), (float("nan"), 0.3)):
        spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall, mesh.wm_node)
        with pytest.raises(dgsem.DgsemError) as ei:
            dgsem.Solver(spec, 1.4, R_GAS, 1e-3, 0.72, sutherland=(T_ref, Sg))
        assert ei.value.status == dgsem.DG_EINVAL
