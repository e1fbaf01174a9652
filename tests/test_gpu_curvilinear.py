"""Curved hexahedra on the GPU against the oracle (FP64).

Right-hand side: relative L2 <= 1e-12 per variable on periodic warped boxes
(N = 3, 5, 7; Navier-Stokes, Euler, central flux, Sutherland's law); an
axis-aligned box given by its node coordinates reproduces the Cartesian
kernels; free streams are preserved on a warped mesh; ten RK steps of the
curved N = 3 Taylor-Green case; at the full N = 7, 32^3 curved workload (the
launch configuration the bench times) sampled elements against the oracle on
their 3^3 patch (a well-conditioned state at 1e-12; the Ma = 0.1 Taylor-Green
state within 20x the oracle's own summation-order spread) and
conservation of the five integrals over 20 steps; the rejected combinations.
"""

import numpy as np
import pytest
import torch

from oracle import curvilinear as cv
from oracle.mesh import Mesh
from oracle.physics import Gas
from paper_2606_18927_amd import dgsem, workloads

from _cases import random_faces, random_state
from _gpu import need_gpu, oracle_gas, periodic_patch, rel_l2, say, state, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12
GAS = Gas(gamma=1.4, R=1.0, mu=0.02, Pr=0.72)


def _solver(N, X, g, bc=("periodic",) * 3, T_wall=1.0, **kw):
    spec = dgsem.MeshSpec(N, None, bc, T_wall, nodes=X)
    suth = (g.T_ref, g.S) if g.sutherland else None
    return dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, sutherland=suth, **kw)


def _rel_l2_momentum(got, ref):
    """Relative L2 of rho and E, and of each momentum component against the
    norm of the whole momentum field: this Taylor-Green state starts with
    w = 0, so rho w stays small and its own norm would only measure rounding
    of the other components."""
    g = np.asarray(got).reshape(5, -1)
    r = np.asarray(ref).reshape(5, -1)
    num = np.linalg.norm(g - r, axis=1)
    den = np.linalg.norm(r, axis=1)
    den[1:4] = np.linalg.norm(r[1:4])
    return num / den


def _warped(N, n, amp):
    xi, _ = dgsem.lgl(N)
    return workloads.warped_nodes(xi, n, amp=amp)


@pytest.mark.parametrize("N,n,amp,viscous,central,suth,flux", [
    (3, (2, 3, 2), 0.08, True, False, False, "kg_llf"),
    (5, (2, 2, 3), 0.05, True, False, False, "kg_llf"),
    (7, (2, 2, 2), 0.05, True, False, False, "kg_llf"),
    (3, (3, 2, 2), 0.08, False, False, False, "kg_llf"),
    (5, (2, 2, 2), 0.08, True, True, False, "kg_llf"),
    (3, (2, 2, 2), 0.08, True, False, True, "kg_llf"),
    (3, (2, 3, 2), 0.08, True, False, False, "ec_roe"),
    (5, (2, 2, 3), 0.05, False, False, False, "ec_roe"),
    (7, (2, 2, 2), 0.05, True, False, True, "ec_roe"),
    (5, (2, 2, 2), 0.08, False, True, False, "ec_roe"),
])
def test_curved_rhs_against_oracle(N, n, amp, viscous, central, suth, flux):
    need_gpu()
    say("curved rhs", N, n, amp, viscous, central, suth, flux)
    X = _warped(N, n, amp)
    mesh = cv.CurvMesh(N, torch.as_tensor(X))
    g = Gas(gamma=1.4, R=1.0, mu=0.02, Pr=0.72, sutherland=True, T_ref=1.0, S=0.4) if suth else GAS
    U = random_state(mesh, g.gamma, g.R, np.random.default_rng(90 + N)).numpy()
    S = _solver(N, X, g, viscous=viscous, central_only=central, flux=flux)
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = cv.rhs(torch.as_tensor(U), mesh, g, viscous=viscous, central_only=central, flux=flux).numpy()
    e = rel_l2(got, ref)
    say("  rel L2", e)
    assert np.all(e < TOL)


def test_affine_nodes_match_cartesian_kernels():
    need_gpu()
    rng = np.random.default_rng(12)
    box = Mesh(5, tuple(random_faces(k, 0.0, 2 * np.pi, rng) for k in (2, 3, 2)))
    X = torch.stack(box.coords()).numpy()
    U = random_state(box, GAS.gamma, GAS.R, rng).numpy()
    Sc = dgsem.Solver(dgsem.MeshSpec(5, box.faces), GAS.gamma, GAS.R, GAS.mu, GAS.Pr)
    a = Sc.eval_rhs(to_dev(U)).cpu().numpy()
    Sc.sync()
    Sv = _solver(5, X, GAS)
    b = Sv.eval_rhs(to_dev(U)).cpu().numpy()
    Sv.sync()
    e = rel_l2(b, a)
    say("affine curved vs Cartesian kernels", e)
    assert np.all(e < 1e-13)


def test_free_stream_preserved_on_warped_mesh():
    need_gpu()
    N = 5
    X = _warped(N, (3, 2, 2), 0.08)
    shape = X.shape[1:]
    rho, u, v, w, p = 1.3, 0.4, -0.25, 0.15, 2.0
    E = p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)
    U = np.stack([np.full(shape, x) for x in (rho, rho * u, rho * v, rho * w, E)])
    S = _solver(N, X, GAS)
    out = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    scale = (abs(rho * u) + p + E) * 2 * N * N
    say("free stream max |Ut|", np.abs(out).max(), "scale", scale)
    assert np.abs(out).max() < 1e-12 * scale


def test_curved_ec_entropy_conservation():
    """The GPU's Euler central entropy-conserving operator on a warped mesh:
    the total entropy rate sum w J v . Ut vanishes to rounding (J from the
    oracle's metric terms, v the entropy variables of the state)."""
    from oracle.physics import entropy_variables, primitives
    need_gpu()
    N = 5
    X = _warped(N, (2, 2, 3), 0.08)
    mesh = cv.CurvMesh(N, torch.as_tensor(X))
    U = random_state(mesh, GAS.gamma, GAS.R, np.random.default_rng(31)).numpy()
    S = _solver(N, X, GAS, viscous=False, central_only=True, flux="ec_roe")
    out = S.eval_rhs(to_dev(U)).cpu().numpy().reshape(U.shape)
    S.sync()
    v = entropy_variables(primitives(torch.as_tensor(U), GAS), GAS)
    wq = mesh.quadrature_weights().numpy()
    terms = sum(wq * v[k].numpy() * out[k] for k in range(5))
    say("entropy rate", terms.sum(), "of", np.abs(terms).sum())
    assert abs(terms.sum()) < 1e-12 * np.abs(terms).sum()


def test_curved_rk_steps():
    need_gpu()
    wl = workloads.WORKLOADS["tgv_n3_4x4x4_curved"]
    U, dt = state(wl)
    X = wl.nodes(dgsem.lgl(wl.N)[0])
    S = dgsem.solver_for(wl)
    S.set_state(to_dev(U))
    S.rk_step(dt, wl.nsteps)
    S.sync()
    got = S.get_state().cpu().numpy().reshape(U.shape)
    ref = cv.rk_step(torch.as_tensor(U), cv.CurvMesh(wl.N, torch.as_tensor(X)), oracle_gas(wl), dt,
                     wl.nsteps).numpy()
    e, e2 = _rel_l2_momentum(got, ref), _rel_l2_momentum(got - U, ref - U)
    say("curved TGV N=3, 10 steps: rel L2", e, "increment", e2)
    assert np.all(e < TOL) and np.all(e2 < 1e-9)


# ------------------------------------------------- wavy-walled channels

@pytest.mark.parametrize("N,n,viscous,suth,flux", [
    (3, (2, 3, 2), True, False, "kg_llf"),
    (5, (2, 2, 2), True, False, "kg_llf"),
    (3, (3, 2, 2), False, False, "kg_llf"),
    (5, (2, 3, 2), True, True, "kg_llf"),
    (5, (2, 3, 2), True, False, "ec_roe"),
])
def test_wavy_channel_rhs_against_oracle(N, n, viscous, suth, flux):
    need_gpu()
    say("wavy channel rhs", N, n, viscous, suth, flux)
    X = workloads.wavy_channel_nodes(dgsem.lgl(N)[0], n, amp=0.06)
    bc = ("periodic", "wall", "periodic")
    mesh = cv.CurvMesh(N, torch.as_tensor(X), bc=bc, T_wall=1.3)
    g = Gas(gamma=1.4, R=1.0, mu=0.02, Pr=0.72, sutherland=True, T_ref=1.0, S=0.4) if suth else GAS
    U = random_state(mesh, g.gamma, g.R, np.random.default_rng(60 + N)).numpy()
    S = _solver(N, X, g, bc=bc, T_wall=1.3, viscous=viscous, flux=flux)
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = cv.rhs(torch.as_tensor(U), mesh, g, viscous=viscous, flux=flux).numpy()
    e = rel_l2(got, ref)
    say("  rel L2", e)
    assert np.all(e < TOL)


def test_wavy_channel_rk_steps_and_rest_state():
    """Five RK steps of a Poiseuille-like flow between wavy walls against the
    oracle; fluid at rest at the wall temperature stays at rest."""
    need_gpu()
    N, n = 3, (3, 3, 2)
    X = workloads.wavy_channel_nodes(dgsem.lgl(N)[0], n, amp=0.06)
    bc = ("periodic", "wall", "periodic")
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=1e-2, Pr=0.72)
    mesh = cv.CurvMesh(N, torch.as_tensor(X), bc=bc, T_wall=1.0)
    Y = X[1]
    u = 1.2 * np.clip(1.0 - Y * Y, 0.0, None)
    rho = np.ones_like(u)
    p = g.R * rho
    E = p / 0.4 + 0.5 * rho * u * u
    z = np.zeros_like(u)
    U = np.stack([rho, rho * u, z, z, E])
    S = _solver(N, X, g, bc=bc, T_wall=1.0)
    dt, nsteps = 2e-4, 5
    S.set_state(to_dev(U))
    S.rk_step(dt, nsteps)
    S.sync()
    got = S.get_state().cpu().numpy().reshape(U.shape)
    ref = cv.rk_step(torch.as_tensor(U), mesh, g, dt, nsteps).numpy()
    e, e2 = _rel_l2_momentum(got, ref), _rel_l2_momentum(got - U, ref - U)
    say("wavy channel 5 steps rel L2", e, "increment", e2)
    assert np.all(e < TOL) and np.all(e2 < 1e-9)
    rest = np.stack([rho, z, z, z, E - 0.5 * rho * u * u])
    out = S.eval_rhs(to_dev(rest)).cpu().numpy()
    S.sync()
    assert np.abs(out).max() < 1e-12 * g.R * 2 * N * N


# ------------------------------------------- full N=7, 32^3 curved workload

@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = workloads.WORKLOADS["tgv_n7_32x32x32_curved"]
    say("building", wl.name)
    U, dt = state(wl)
    X = wl.nodes(dgsem.lgl(wl.N)[0])
    S = dgsem.solver_for(wl)
    return wl, U, dt, X, S


SAMPLES = [(0, 0, 0), (31, 17, 5), (13, 31, 30)]


def _order_sensitivity(P, Xp, N, g, ref):
    """Largest relative change of the oracle's result at the patch centre when
    its collocation derivatives are summed sequentially, forwards or
    backwards, instead of by its matrix product: the rounding spread of the
    definition itself, computed from the oracle only."""
    import oracle.curvilinear as cvm
    orig = cvm._apply_D

    def seq(q, D, na, rev):
        qm = q.movedim(na, -1)
        out = torch.zeros_like(qm)
        for m in (range(D.shape[0] - 1, -1, -1) if rev else range(D.shape[0])):
            out = out + qm[..., m:m + 1] * D[:, m].to(q.dtype)
        return out.movedim(-1, na)

    out = []
    try:
        for rev in (False, True):
            cvm._apply_D = lambda q, D, na, rev=rev: seq(q, D, na, rev)
            out.append(rel_l2(cv.rhs(P, cv.CurvMesh(N, Xp), g).numpy()[:, 1, 1, 1], ref))
    finally:
        cvm._apply_D = orig
    return np.max(out, axis=0)


def test_full_size_curved_rhs_sampled(big):
    """The Ma = 0.1 Taylor-Green state of the bench.  Its momentum right-hand
    side cancels terms of the size of the mean pressure p0 = 71 times the
    metric terms, and the metric terms (derivatives of products of
    derivatives of the node coordinates) carry rounding that depends on the
    summation order: summing the oracle's own derivatives in another order
    moves its momentum result by ~1e-11 relative here.  The bound per variable
    is 20x that spread (computed in the test from the oracle alone), floored
    at 1e-12; the strict 1e-12 check of the same mesh and launch is the
    well-conditioned state below."""
    wl, U, dt, X, S = big
    Ut = S.eval_rhs(to_dev(U)).cpu().numpy().reshape(U.shape)
    S.sync()
    g = oracle_gas(wl)
    for c in SAMPLES:
        say("sample", c)
        P = torch.as_tensor(np.ascontiguousarray(periodic_patch(U, c, 1)))
        Xp = torch.as_tensor(np.ascontiguousarray(periodic_patch(X, c, 1)))
        ref = cv.rhs(P, cv.CurvMesh(wl.N, Xp), g).numpy()[:, 1, 1, 1]
        spread = _order_sensitivity(P, Xp, wl.N, g, ref)
        tol = np.maximum(TOL, 20.0 * spread)
        got = Ut[:, c[2], c[1], c[0]]
        e = rel_l2(got, ref)
        say("  rel L2", e, "oracle summation-order spread", spread)
        assert np.all(e < tol)


def test_full_size_curved_rhs_sampled_well_conditioned(big):
    """Same mesh and launch with a random state of pressure ~1 (no low-Mach
    cancellation): 1e-12 per variable at sampled elements."""
    wl, U, dt, X, S = big
    rng = np.random.default_rng(2024)
    shape = U.shape[1:]
    rho = 1.0 + 0.2 * rng.uniform(-1, 1, size=shape)
    vel = 0.5 * rng.uniform(-1, 1, size=(3,) + shape)
    p = 1.0 + 0.2 * rng.uniform(-1, 1, size=shape)
    E = p / 0.4 + 0.5 * rho * (vel ** 2).sum(0)
    V = np.stack([rho, rho * vel[0], rho * vel[1], rho * vel[2], E])
    del rho, vel, p, E
    Vt = S.eval_rhs(to_dev(V)).cpu().numpy().reshape(V.shape)
    S.sync()
    g = oracle_gas(wl)
    for c in SAMPLES:
        say("sample", c)
        P = torch.as_tensor(np.ascontiguousarray(periodic_patch(V, c, 1)))
        Xp = np.ascontiguousarray(periodic_patch(X, c, 1))
        ref = cv.rhs(P, cv.CurvMesh(wl.N, torch.as_tensor(Xp)), g).numpy()[:, 1, 1, 1]
        e = rel_l2(Vt[:, c[2], c[1], c[0]], ref)
        say("  rel L2", e)
        assert np.all(e < TOL)


def test_full_size_curved_conservation(big):
    """Twenty steps: the discrete integrals sum w J U of all five conserved
    variables stay constant (J from the oracle's metric terms)."""
    wl, U, dt, X, S = big
    S.set_state(to_dev(U))
    S.rk_step(dt, 20)
    S.sync()
    Un = S.get_state().cpu().numpy().reshape(U.shape)
    wq = cv.CurvMesh(wl.N, torch.as_tensor(X)).quadrature_weights().numpy()
    for v in range(5):
        i0, i1 = (wq * U[v]).sum(), (wq * Un[v]).sum()
        mag = (wq * np.abs(U[v])).sum()
        say("  integral", v, i0, i1 - i0)
        assert abs(i1 - i0) < 1e-12 * mag


def test_curved_rejected_combinations():
    need_gpu()
    N = 3
    X = _warped(N, (2, 2, 2), 0.05)
    spec = dgsem.MeshSpec(N, None, ("periodic", "wallmodel", "periodic"), nodes=X)
    with pytest.raises(dgsem.DgsemError) as ei:
        dgsem.Solver(spec, 1.4, 1.0, 0.02, 0.72)
    assert ei.value.status == dgsem.DG_EUNSUPPORTED
    S = _solver(N, X, GAS, with_adjoint=True)
    U = to_dev(random_state(cv.CurvMesh(N, torch.as_tensor(X)), 1.4, 1.0, np.random.default_rng(3)).numpy())
    for call in (lambda: S.eval_rhs_vjp(U, U), lambda: S.eval_lift(U), lambda: S.kinetic_energy(U)):
        with pytest.raises(dgsem.DgsemError) as ei:
            call()
        assert ei.value.status == dgsem.DG_EUNSUPPORTED
    # a mirrored mesh has J < 0 at every node: binding the workspace fails
    Xm = X.copy()
    Xm[0] = -Xm[0]
    with pytest.raises(dgsem.DgsemError) as ei:
        _solver(N, Xm, GAS)
    assert ei.value.status == dgsem.DG_EINVAL
