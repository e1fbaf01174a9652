"""The entropy-conserving volume flux with the Roe surface flux (DG_FLUX_EC_ROE)
against the FP64 oracle (GPU).

Criterion as for the default fluxes: per conserved variable, relative L2 error
<= 1e-12.  Small cases compare every node (periodic and wall boundaries,
N = 3, 5, 7, with and without viscosity and surface dissipation); the full
N = 7, 32^3-element Taylor-Green case compares sampled elements against the
oracle on periodic patches, and checks a property that holds at any size: the
Euler split form with the entropy-conserving surface flux conserves the
discrete entropy, sum_nodes w J v . Ut = 0, v the entropy variables.
"""

import numpy as np
import pytest
import torch

from oracle.dgsem import rhs, rk_step
from oracle.mesh import Mesh
from oracle.physics import Gas
from paper_2606_18927_amd import dgsem, workloads

from _cases import random_faces, random_state
from _gpu import need_gpu, oracle_gas, oracle_mesh, periodic_patch, rel_l2, say, state, to_dev, uniform_patch_mesh

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _case(N, n, bc, seed, mu=0.01):
    rng = np.random.default_rng(seed)
    faces = [random_faces(n[d], -1.0, 1.0, rng) if bc[d] == "wall" else random_faces(n[d], 0.0, 2.0 + d, rng)
             for d in range(3)]
    mesh = Mesh(N, tuple(faces), bc=bc, T_wall=1.1)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=mu, Pr=0.72)
    U = random_state(mesh, g.gamma, g.R, rng, vel_amp=1.0, p_mean=1.0 / (1.4 * 0.01), p_amp=0.05)
    return mesh, g, U.numpy()


def _solver(mesh, g, **kw):
    spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall)
    return dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, flux="ec_roe", **kw)


P3 = ("periodic",) * 3


@pytest.mark.parametrize("N,n,bc,viscous,central", [
    (3, (3, 2, 3), P3, True, False),
    (3, (2, 3, 2), ("periodic", "wall", "periodic"), True, False),
    (5, (2, 3, 2), ("periodic", "wall", "periodic"), True, False),
    (7, (2, 2, 3), P3, True, False),
    (7, (2, 3, 2), ("periodic", "periodic", "wall"), False, False),
    (5, (3, 2, 2), P3, False, True),
])
def test_ec_rhs_against_oracle(N, n, bc, viscous, central):
    need_gpu()
    say("ec case", N, n, bc, "viscous" if viscous else "euler", "central" if central else "roe")
    mesh, g, U = _case(N, n, bc, seed=70 + N)
    S = _solver(mesh, g, viscous=viscous, central_only=central)
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = rhs(torch.as_tensor(U), mesh, g, viscous=viscous, central_only=central, flux="ec_roe").numpy()
    e = rel_l2(got, ref)
    say("  rel L2", e)
    assert np.all(e < TOL)


def test_ec_tgv_n3_rk_against_oracle():
    need_gpu()
    base = workloads.WORKLOADS["tgv_n3_4x4x4"]
    wl = workloads.Workload("tgv_n3_4x4x4_ec", "tgv", 3, (4, 4, 4), nsteps=base.nsteps, flux="ec_roe")
    U, dt = state(wl)
    S = dgsem.solver_for(wl)
    S.set_state(to_dev(U))
    S.rk_step(dt, wl.nsteps)
    S.sync()
    got = S.get_state().cpu().numpy()
    ref = rk_step(torch.as_tensor(U), oracle_mesh(wl), oracle_gas(wl), dt, wl.nsteps, flux="ec_roe").numpy()
    e = rel_l2(got, ref)
    e2 = rel_l2(got - U.reshape(got.shape), ref - U)
    say("ec tgv n3, 10 steps: rel L2", e, "increment", e2)
    assert np.all(e < TOL)
    assert np.all(e2 < 1e-10)


def test_ec_unsupported_combinations():
    need_gpu()
    mesh, g, _ = _case(3, (2, 2, 2), P3, seed=1)
    spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall)
    with pytest.raises(dgsem.DgsemError) as ei:
        dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, flux="ec_roe", precision="mixed_noref")
    assert ei.value.status == dgsem.DG_EUNSUPPORTED
    # (the adjoint covers this pair: tests/test_gpu_adjoint_ec.py)


# --------------------------------------------------- full N=7, 32^3 workload

@pytest.fixture(scope="module")
def big_ec():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = workloads.WORKLOADS["tgv_n7_32x32x32_ec"]
    say("building", wl.name)
    U, dt = state(wl)
    return wl, U, dt


def test_ec_full_size_eval_rhs_sampled(big_ec):
    wl, U, dt = big_ec
    S = dgsem.solver_for(wl)
    Ut = S.eval_rhs(to_dev(U)).cpu().numpy().reshape(U.shape)
    S.sync()
    h = [2 * np.pi / 32] * 3
    pm = uniform_patch_mesh(wl.N, h, 1, wl)
    g = oracle_gas(wl)
    for c in [(0, 0, 0), (31, 17, 5), (13, 31, 30)]:
        say("ec sample", c)
        P = periodic_patch(U, c, 1)
        ref = rhs(torch.as_tensor(np.ascontiguousarray(P)), pm, g, flux="ec_roe").numpy()[:, 1, 1, 1]
        e = rel_l2(Ut[:, c[2], c[1], c[0]], ref)
        say("  rel L2", e)
        assert np.all(e < TOL)


def test_ec_full_size_entropy_conservation(big_ec):
    """Euler, entropy-conserving surface flux, periodic: d/dt sum w J S(U) = 0."""
    wl, U, dt = big_ec
    S = dgsem.solver_for(wl, viscous=False, central_only=True)
    Ut = S.eval_rhs(to_dev(U)).cpu().numpy().reshape(U.shape)
    S.sync()
    g = oracle_gas(wl)
    rho, u, v, w, E = U
    p = (g.gamma - 1.0) * (E - 0.5 * (u * u + v * v + w * w) / rho)
    s = np.log(p) - g.gamma * np.log(rho)
    beta = rho / (2.0 * p)
    q2 = (u * u + v * v + w * w) / (rho * rho)
    ent = [(g.gamma - s) / (g.gamma - 1.0) - beta * q2, 2.0 * beta * u / rho, 2.0 * beta * v / rho,
           2.0 * beta * w / rho, -2.0 * beta]
    wq = oracle_mesh(wl).quadrature_weights().numpy()
    terms = sum(ent[k] * Ut[k] for k in range(5)) * wq
    rate = terms.sum() / np.abs(terms).sum()
    say("relative entropy rate", rate)
    assert abs(rate) < 1e-12
