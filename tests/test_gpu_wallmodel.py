"""The algebraic wall-stress model (dg_wall_stress, one lane per wall-face node)
against the oracle (GPU).

The paper validates its GPU wall model by CPU-GPU agreement at machine
precision; here every wall-face node is compared with the oracle's model
(Brent's method instead of the kernel's Newton iteration): relative error of
the stress vectors <= 1e-13 of the largest stress.  Cases: the paper's
wall-modelled channel mesh (N = 5, 5 x 30 x 3 elements, tanh-stretched
wall-normal spacing) with a turbulent-like mean profile plus sine
perturbations, several interface nodes; walls on all three axes (N = 3); the
N = 5, 16^3 stretched channel.
"""

import numpy as np
import pytest
import torch

from oracle.mesh import Mesh, tanh_faces, uniform_faces
from oracle.physics import Gas
from oracle.wallmodel import wall_stress_field
from paper_2606_18927_amd import dgsem, workloads

from _cases import random_faces, random_state
from _gpu import need_gpu, oracle_gas, oracle_mesh, say, state, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-13


def _solver(mesh, g):
    spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall)
    return dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr)


def _compare(mesh, g, U, n_wm):
    S = _solver(mesh, g)
    got = S.wall_stress(to_dev(U), n_wm).cpu().numpy()
    S.sync()
    ref = wall_stress_field(torch.as_tensor(U), mesh, g, n_wm, lambda T: g.mu)
    assert got.shape == ref.shape
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    say(f"  n_wm={n_wm}: {ref.shape[0]} faces, max |tau| {scale:.3e}, rel err {err:.2e}")
    assert err < TOL
    return ref


def _channel_state(mesh, g, rng, u_b=1.0, amp=0.05):
    X, Y, Z = [c.numpy() for c in mesh.coords()]
    # turbulent-like mean profile (flat core, steep near the walls) plus sine perturbations
    u = u_b * 1.14 * (1.0 - np.abs(Y) ** 8)
    u = u * (1.0 + amp * np.sin(2 * X) * np.cos(3 * Z))
    v = amp * np.sin(X + 0.3) * (1.0 - Y * Y)
    w = amp * np.cos(2 * Z) * (1.0 - Y * Y)
    rho = np.ones_like(u) * (1.0 + 0.01 * rng.standard_normal(u.shape))
    p = rho * g.R * 1.0
    E = p / (g.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


def test_wall_model_paper_channel_mesh():
    """N = 5, (5, 30, 3) elements on [0, 2pi] x [-1, 1] x [0, pi], Ma = 0.1, Re_tau = 180."""
    need_gpu()
    mesh = Mesh(5, (uniform_faces(5, 0, 2 * np.pi), tanh_faces(30, 2.0), uniform_faces(3, 0, np.pi)),
                bc=("periodic", "wall", "periodic"), T_wall=1.0)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=1.0 / 180.0 / 18.0, Pr=0.72)
    U = _channel_state(mesh, g, np.random.default_rng(5))
    say("paper channel mesh", mesh.nelem, mesh.n_dof, "DOF")
    for n_wm in (1, 2, 3, 5):
        _compare(mesh, g, U, n_wm)


def test_wall_model_walls_on_every_axis():
    need_gpu()
    rng = np.random.default_rng(9)
    mesh = Mesh(3, tuple(random_faces(n, -1.0, 1.0, rng) for n in (2, 3, 2)), bc=("wall",) * 3, T_wall=1.0)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=1e-3, Pr=0.72)
    U = random_state(mesh, g.gamma, g.R, rng, vel_amp=1.0, p_mean=1.0 / (1.4 * 0.01), p_amp=0.05).numpy()
    for n_wm in (1, 3):
        ref = _compare(mesh, g, U, n_wm)
        assert ref.shape[0] == 2 * (3 * 2 + 2 * 2 + 2 * 3)


def test_wall_model_channel_16():
    need_gpu()
    wl = workloads.WORKLOADS["channel_n5_16x16x16"]
    U, _ = state(wl)
    _compare(oracle_mesh(wl), oracle_gas(wl), U, 2)


def test_wall_model_no_walls_and_errors():
    need_gpu()
    mesh = Mesh(3, (uniform_faces(2, 0, 1),) * 3)
    g = Gas(gamma=1.4, R=1.0, mu=1e-3, Pr=0.72)
    S = _solver(mesh, g)
    assert S.wall_faces() == 0
    U = to_dev(np.ones((5,) + mesh.shape))
    assert S.wall_stress(U, 1).numel() == 0
    mesh = Mesh(3, (uniform_faces(2, 0, 1),) * 3, bc=("periodic", "wall", "periodic"), T_wall=1.0)
    S = _solver(mesh, g)
    with pytest.raises(dgsem.DgsemError) as ei:
        S.wall_stress(U, 0)
    assert ei.value.status == dgsem.DG_EINVAL
    with pytest.raises(dgsem.DgsemError) as ei:
        S.wall_stress(U, 4)
    assert ei.value.status == dgsem.DG_EINVAL


# ------------------------------------------- the wall model in the operator

def _wm_solver(mesh, g, **kw):
    spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall, mesh.wm_node)
    return dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, **kw)


def _rel_l2(got, ref):
    g = np.asarray(got).reshape(5, -1)
    r = np.asarray(ref).reshape(5, -1)
    return np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)


@pytest.mark.parametrize("N,n,bc,wm_node", [
    (3, (2, 3, 2), ("periodic", "wallmodel", "periodic"), 1),
    (5, (2, 3, 2), ("periodic", "wallmodel", "periodic"), 3),
    (3, (2, 2, 3), ("periodic", "wall", "wallmodel"), 2),
    (3, (2, 2, 2), ("wallmodel", "periodic", "wallmodel"), 3),
])
def test_wall_model_rhs_against_oracle(N, n, bc, wm_node):
    from oracle.dgsem import rhs
    need_gpu()
    say("wall-model rhs", N, n, bc, wm_node)
    rng = np.random.default_rng(40 + N + wm_node)
    faces = [random_faces(n[d], -1.0, 1.0, rng) if bc[d] != "periodic" else random_faces(n[d], 0.0, 2.0, rng)
             for d in range(3)]
    mesh = Mesh(N, tuple(faces), bc=bc, T_wall=1.1, wm_node=wm_node)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=1e-3, Pr=0.72)
    U = random_state(mesh, g.gamma, g.R, rng, vel_amp=1.0, p_mean=1.0 / (1.4 * 0.01), p_amp=0.05).numpy()
    S = _wm_solver(mesh, g)
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = rhs(torch.as_tensor(U), mesh, g).numpy()
    e = _rel_l2(got, ref)
    say("  rel L2", e)
    assert np.all(e < 1e-12)


def test_wall_model_paper_channel_rhs_and_steps():
    """The paper's wall-modelled channel: N = 5, (5, 30, 3) elements (97200 DOF);
    right-hand side against the oracle at every node, five RK steps against the
    oracle, and the exact conservation of mass and total energy over the run."""
    from oracle.dgsem import rhs, rk_step
    need_gpu()
    mesh = Mesh(5, (uniform_faces(5, 0, 2 * np.pi), tanh_faces(30, 2.0), uniform_faces(3, 0, np.pi)),
                bc=("periodic", "wallmodel", "periodic"), T_wall=1.0, wm_node=2)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=1.0 / 180.0 / 18.0, Pr=0.72)
    U = _channel_state(mesh, g, np.random.default_rng(7))
    S = _wm_solver(mesh, g)
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = rhs(torch.as_tensor(U), mesh, g).numpy()
    e = _rel_l2(got, ref)
    say("paper channel rhs rel L2", e, mesh.n_dof, "DOF")
    assert np.all(e < 1e-12)
    dt, nsteps = 2e-5, 5  # acoustic CFL about 0.15 at the smallest LGL spacing
    S.set_state(to_dev(U))
    S.rk_step(dt, nsteps)
    S.sync()
    Un = S.get_state().cpu().numpy().reshape(U.shape)
    Uref = rk_step(torch.as_tensor(U), mesh, g, dt, nsteps).numpy()
    e = _rel_l2(Un, Uref)
    e2 = _rel_l2(Un - U, Uref - U)
    say("paper channel 5 steps rel L2", e, "increment", e2)
    assert np.all(e < 1e-12) and np.all(e2 < 1e-9)
    wq = mesh.quadrature_weights().numpy()
    for v in (0, 4):
        i0, i1 = (wq * U[v]).sum(), (wq * Un[v]).sum()
        assert abs(i1 - i0) < 1e-13 * (wq * np.abs(U[v])).sum()
    assert (wq * Un[1]).sum() < (wq * U[1]).sum()  # the walls drag the flow


def test_wall_model_unsupported_combinations():
    need_gpu()
    mesh = Mesh(3, (uniform_faces(2, 0, 1), uniform_faces(2, -1, 1), uniform_faces(2, 0, 1)),
                bc=("periodic", "wallmodel", "periodic"), wm_node=1)
    g = Gas(gamma=1.4, R=1.0, mu=1e-3, Pr=0.72)
    # (mixed precision covers the wall model: tests/test_gpu_mixed_physics.py)
    S = _wm_solver(mesh, g, with_adjoint=True)
    U = to_dev(np.ones((5,) + mesh.shape) * np.array([1, 0.1, 0, 0, 3.0])[:, None, None, None, None, None, None])
    with pytest.raises(dgsem.DgsemError) as ei:
        S.eval_rhs_vjp(U, U)
    assert ei.value.status == dgsem.DG_EUNSUPPORTED
    bad = Mesh(3, mesh.faces, bc=mesh.bc, wm_node=4)
    with pytest.raises(dgsem.DgsemError) as ei:
        _wm_solver(bad, g)
    assert ei.value.status == dgsem.DG_EINVAL


def test_production_physics_paper_channel():
    """The paper's production combination on its wall-modelled channel mesh:
    the entropy-conserving volume flux with Roe's surface flux, Sutherland's
    law and the wall model (FP64): right-hand side at every node and five RK
    steps against the oracle, mass and energy conserved."""
    from oracle.dgsem import rhs, rk_step
    need_gpu()
    mesh = Mesh(5, (uniform_faces(5, 0, 2 * np.pi), tanh_faces(30, 2.0), uniform_faces(3, 0, np.pi)),
                bc=("periodic", "wallmodel", "periodic"), T_wall=1.0, wm_node=2)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=1.0 / 180.0 / 18.0, Pr=0.72, sutherland=True,
            T_ref=1.0, S=110.4 / 288.15)
    U = _channel_state(mesh, g, np.random.default_rng(9))
    spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall, mesh.wm_node)
    S = dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, flux="ec_roe", sutherland=(g.T_ref, g.S))
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = rhs(torch.as_tensor(U), mesh, g, flux="ec_roe").numpy()
    e = _rel_l2(got, ref)
    say("production physics rhs rel L2", e)
    assert np.all(e < 1e-12)
    dt, nsteps = 2e-5, 5
    S.set_state(to_dev(U))
    S.rk_step(dt, nsteps)
    S.sync()
    Un = S.get_state().cpu().numpy().reshape(U.shape)
    Uref = rk_step(torch.as_tensor(U), mesh, g, dt, nsteps, flux="ec_roe").numpy()
    e, e2 = _rel_l2(Un, Uref), _rel_l2(Un - U, Uref - U)
    say("production physics 5 steps rel L2", e, "increment", e2)
    assert np.all(e < 1e-12) and np.all(e2 < 1e-9)
    wq = mesh.quadrature_weights().numpy()
    for v in (0, 4):
        assert abs((wq * Un[v]).sum() - (wq * U[v]).sum()) < 1e-13 * (wq * np.abs(U[v])).sum()
