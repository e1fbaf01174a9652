"""CPU pins of the oracle's curvilinear split-form DGSEM.

* metric terms: the discrete metric identities sum_i D_i (J a^i_n) = 0 hold to
  rounding for the curl form on a warped mesh (and fail for the cross-product
  form: negative control); on an affine box J a^i = J s_i e_i and J = the
  element volume / 8 exactly;
* reduction: an axis-aligned box given by its node coordinates reproduces the
  (pinned) Cartesian operator, viscous and inviscid;
* rotation equivariance: the box rotated by an orthogonal Q with the velocity
  rotated by Q gives Q times the momentum right-hand side and the same mass
  and energy right-hand side (a transposed metric or a wrong index fails);
* free-stream preservation on a warped periodic mesh (curl form, to rounding;
  the cross form does not preserve it);
* conservation of mass, momentum and energy on the warped mesh:
  sum w J Ut = 0 to rounding;
* order N of the truncation error against a manufactured Navier-Stokes
  solution on warped meshes (4^3 -> 8^3 elements);
* isothermal walls: an axis-aligned channel given by its nodes reproduces the
  Cartesian operator with walls (itself pinned by the exact discrete
  Poiseuille state); fluid at rest at the wall temperature between wavy
  walls has Ut = 0 to rounding (and is disturbed by another wall
  temperature); mass is conserved between wavy walls;
* the entropy-conserving / Roe pair on curved elements: the Roe flux along a
  normal vector equals the pinned axis-aligned Roe flux for axis normals and
  is rotation invariant; an affine box reproduces the Cartesian operator;
  the Euler central form conserves the total entropy on warped meshes
  (Kennedy-Gruber does not; Roe dissipation makes the rate negative); free
  streams are preserved.
"""

import math

import numpy as np
import pytest
import torch

from oracle import curvilinear as cv
from oracle.basis import diff_matrix, lgl
from oracle.dgsem import _apply_D, rhs as rhs_cart
from oracle.mesh import NODE_AXIS, Mesh, uniform_faces
from oracle.physics import Gas
from paper_2606_18927_amd.workloads import warped_nodes

from _cases import random_faces, random_state

TWO_PI = 2 * math.pi
GAS = Gas(gamma=1.4, R=1.0, mu=0.02, Pr=0.72)


def _warped(N, n, amp=0.05):
    xi, _ = lgl(N)
    return cv.CurvMesh(N, torch.as_tensor(warped_nodes(xi.numpy(), n, amp=amp)))


def _box_nodes(mesh: Mesh):
    return torch.stack(mesh.coords())


@pytest.mark.parametrize("N", [3, 5])
def test_metric_identities(N):
    mesh = _warped(N, (2, 3, 2))
    D = diff_matrix(N)
    for form, ok in (("curl", True), ("cross", False)):
        m = cv.CurvMesh(N, mesh.X, metric_form=form)
        Ja, J = cv.metrics(m)
        assert J.min() > 0
        scale = max(Ja[i][n].abs().max().item() for i in range(3) for n in range(3))
        res = max(sum(_apply_D(Ja[i][n], D, NODE_AXIS[i]) for i in range(3)).abs().max().item() for n in range(3))
        if ok:
            assert res < 1e-13 * scale * N * N
        else:
            assert res > 1e-4 * scale


def test_affine_metrics_exact():
    rng = np.random.default_rng(2)
    box = Mesh(3, tuple(random_faces(n, 0.0, 2.0, rng) for n in (2, 3, 2)))
    Ja, J = cv.metrics(cv.CurvMesh(3, _box_nodes(box)))
    Jc = box.jacobian().expand(box.shape)
    assert torch.allclose(J, Jc, rtol=1e-14, atol=0)
    for i in range(3):
        for n in range(3):
            ref = (Jc * box.scale(i)) if i == n else torch.zeros(box.shape, dtype=torch.float64)
            assert torch.allclose(Ja[i][n], ref.expand(box.shape), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("viscous", [True, False])
def test_reduces_to_cartesian_operator(viscous):
    rng = np.random.default_rng(4)
    box = Mesh(3, tuple(random_faces(n, 0.0, TWO_PI, rng) for n in (2, 3, 2)))
    U = random_state(box, GAS.gamma, GAS.R, rng)
    ref = rhs_cart(U, box, GAS, viscous=viscous)
    got = cv.rhs(U, cv.CurvMesh(3, _box_nodes(box)), GAS, viscous=viscous)
    for v in range(5):
        assert torch.linalg.norm(got[v] - ref[v]) <= 1e-13 * torch.linalg.norm(ref[v])


def test_rotation_equivariance():
    rng = np.random.default_rng(6)
    N = 3
    box = Mesh(N, tuple(random_faces(n, 0.0, TWO_PI, rng) for n in (2, 2, 3)))
    U = random_state(box, GAS.gamma, GAS.R, rng)
    ref = rhs_cart(U, box, GAS)
    # rotation about the axis (1, 2, 2)/3 by 0.7 rad
    a = np.array([1.0, 2.0, 2.0]) / 3.0
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    Q = torch.as_tensor(np.eye(3) + math.sin(0.7) * K + (1 - math.cos(0.7)) * K @ K)
    X = torch.einsum("ab,b...->a...", Q, _box_nodes(box))
    Ur = U.clone()
    Ur[1:4] = torch.einsum("ab,b...->a...", Q, U[1:4])
    got = cv.rhs(Ur, cv.CurvMesh(N, X), GAS)
    refr = ref.clone()
    refr[1:4] = torch.einsum("ab,b...->a...", Q, ref[1:4])
    for v in range(5):
        assert torch.linalg.norm(got[v] - refr[v]) <= 1e-12 * torch.linalg.norm(refr[v])
    # a transposed rotation of the velocity breaks it
    Ut = U.clone()
    Ut[1:4] = torch.einsum("ba,b...->a...", Q, U[1:4])
    bad = cv.rhs(Ut, cv.CurvMesh(N, X), GAS)
    assert torch.linalg.norm(bad[1] - refr[1]) > 1e-3 * torch.linalg.norm(refr[1])


@pytest.mark.parametrize("N", [3, 5])
def test_free_stream_preservation_warped(N):
    mesh = _warped(N, (2, 2, 3), amp=0.08)
    shape = mesh.shape
    rho, u, v, w, p = 1.3, 0.4, -0.25, 0.15, 2.0
    E = p / (GAS.gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)
    U = torch.stack([torch.full(shape, x, dtype=torch.float64) for x in (rho, rho * u, rho * v, rho * w, E)])
    scale = (abs(rho * u) + p + E) * 2 * N * N  # flux magnitude x derivative scale
    out = cv.rhs(U, mesh, GAS)
    assert out.abs().max().item() < 1e-12 * scale
    bad = cv.rhs(U, cv.CurvMesh(N, mesh.X, metric_form="cross"), GAS)
    assert bad.abs().max().item() > 1e-5 * scale


def test_conservation_warped():
    rng = np.random.default_rng(8)
    N = 3
    mesh = _warped(N, (2, 3, 2), amp=0.08)
    U = random_state(mesh, GAS.gamma, GAS.R, rng)
    out = cv.rhs(U, mesh, GAS)
    wq = mesh.quadrature_weights()
    for v in range(5):
        tot = (wq * out[v]).sum().item()
        mag = (wq * out[v].abs()).sum().item()
        assert abs(tot) < 1e-13 * mag, (v, tot, mag)


def _mms():
    import test_oracle_operator as op
    return op._mms_source(GAS), op._eval


@pytest.mark.parametrize("N", [3, 4])
def test_manufactured_truncation_order_warped(N):
    (S, Uf), ev = _mms()
    errs = []
    for n in (4, 8):
        m = _warped(N, (n, n, n), amp=0.04)
        X, Y, Z = m.X[0], m.X[1], m.X[2]
        U0 = torch.stack([ev(f, X, Y, Z, 0.0) for f in Uf])
        h = 1e-6
        dUdt = (torch.stack([ev(f, X, Y, Z, h) for f in Uf]) - torch.stack([ev(f, X, Y, Z, -h) for f in Uf])) / (2 * h)
        src = torch.stack([ev(f, X, Y, Z, 0.0) for f in S])
        r = cv.rhs(U0, m, GAS, source=src) - dUdt
        wq = m.quadrature_weights()
        errs.append([math.sqrt((wq * r[v] ** 2).sum().item()) for v in range(5)])
    for v in range(5):
        eoc = math.log2(errs[0][v] / errs[1][v])
        assert eoc > N - 0.35, (v, errs, eoc)


# --------------------------------------------------------------- walls

def _wavy(N, n, amp=0.06):
    from paper_2606_18927_amd.workloads import wavy_channel_nodes
    xi, _ = lgl(N)
    X = torch.as_tensor(wavy_channel_nodes(xi.numpy(), n, amp=amp))
    return cv.CurvMesh(N, X, bc=("periodic", "wall", "periodic"), T_wall=1.3)


@pytest.mark.parametrize("viscous", [True, False])
def test_walls_reduce_to_cartesian_operator(viscous):
    from _cases import channel_mesh
    rng = np.random.default_rng(14)
    box = channel_mesh(3, 2, 3, 2, T_wall=1.3)
    U = random_state(box, GAS.gamma, GAS.R, rng)
    ref = rhs_cart(U, box, GAS, viscous=viscous)
    m = cv.CurvMesh(3, _box_nodes(box), bc=box.bc, T_wall=box.T_wall)
    got = cv.rhs(U, m, GAS, viscous=viscous)
    for v in range(5):
        assert torch.linalg.norm(got[v] - ref[v]) <= 1e-13 * torch.linalg.norm(ref[v])


@pytest.mark.parametrize("N", [3, 5])
def test_fluid_at_rest_between_wavy_walls(N):
    """Uniform pressure, zero velocity and T = T_wall: every flux balance is
    exactly zero (metric identities, the wall pressure flux, zero gradients)."""
    m = _wavy(N, (2, 3, 2))
    p = 1.3 * GAS.R * 2.0  # rho = 2, T = T_wall
    shape = m.shape
    U = torch.stack([torch.full(shape, 2.0, dtype=torch.float64)] + [torch.zeros(shape, dtype=torch.float64)] * 3
                    + [torch.full(shape, p / (GAS.gamma - 1.0), dtype=torch.float64)])
    out = cv.rhs(U, m, GAS)
    assert out.abs().max().item() < 1e-12 * p * 2 * N * N
    # moving fluid or a different wall temperature is not at rest
    m2 = cv.CurvMesh(N, m.X, bc=m.bc, T_wall=1.5)
    assert cv.rhs(U, m2, GAS).abs().max().item() > 1e-6


def test_mass_conservation_between_wavy_walls():
    rng = np.random.default_rng(15)
    m = _wavy(3, (2, 3, 2))
    U = random_state(m, GAS.gamma, GAS.R, rng)
    out = cv.rhs(U, m, GAS)
    wq = m.quadrature_weights()
    tot = (wq * out[0]).sum().item()
    mag = (wq * out[0].abs()).sum().item()
    assert abs(tot) < 1e-13 * mag
    # energy is not conserved (the walls conduct heat), momentum feels the wall pressure
    assert abs((wq * out[4]).sum().item()) > 1e-8 * (wq * out[4].abs()).sum().item()


# ------------------------------------- entropy-conserving / Roe pair

def _random_prims(rng, shape=(7,)):
    from oracle.physics import primitives
    rho = 1.0 + 0.3 * rng.uniform(-1, 1, shape)
    vel = 0.6 * rng.uniform(-1, 1, (3,) + shape)
    p = 1.0 + 0.3 * rng.uniform(-1, 1, shape)
    E = p / 0.4 + 0.5 * rho * (vel ** 2).sum(0)
    U = torch.as_tensor(np.stack([rho, rho * vel[0], rho * vel[1], rho * vel[2], E]))
    return primitives(U, GAS), U


def test_roe_flux_metric_axis_normals_match_axis_flux():
    from oracle.physics import roe_flux
    rng = np.random.default_rng(21)
    L, _ = _random_prims(rng)
    R, _ = _random_prims(rng)
    for d in range(3):
        for sig in (0.37, 2.5):
            s = [torch.full((7,), sig if c == d else 0.0, dtype=torch.float64) for c in range(3)]
            got = cv.roe_flux_metric(L, R, s, GAS)
            ref = roe_flux(L, R, d, GAS)
            for v in range(5):
                assert torch.allclose(got[v], sig * ref[v], rtol=1e-14, atol=1e-14)


def test_roe_flux_metric_rotation_invariance():
    from oracle.physics import Prim
    rng = np.random.default_rng(22)
    L, _ = _random_prims(rng)
    R, _ = _random_prims(rng)
    s = [torch.as_tensor(rng.uniform(-1, 1, 7)) for _ in range(3)]
    a = np.array([2.0, -1.0, 2.0]) / 3.0
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    Q = np.eye(3) + math.sin(1.1) * K + (1 - math.cos(1.1)) * K @ K
    rot = lambda v: [sum(Q[i, j] * v[j] for j in range(3)) for i in range(3)]  # noqa: E731
    Lr = Prim(L.rho, tuple(rot(L.vel)), L.p, L.T, L.e, L.E)
    Rr = Prim(R.rho, tuple(rot(R.vel)), R.p, R.T, R.e, R.E)
    f = cv.roe_flux_metric(L, R, s, GAS)
    fr = cv.roe_flux_metric(Lr, Rr, rot(s), GAS)
    for v, ref in ((0, f[0]), (4, f[4])):
        assert torch.allclose(fr[v], ref, rtol=1e-13, atol=1e-13)
    mom = rot(f[1:4])
    for c in range(3):
        assert torch.allclose(fr[1 + c], mom[c], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("viscous", [True, False])
def test_ec_reduces_to_cartesian_operator(viscous):
    rng = np.random.default_rng(23)
    box = Mesh(3, tuple(random_faces(n, 0.0, TWO_PI, rng) for n in (2, 3, 2)))
    U = random_state(box, GAS.gamma, GAS.R, rng)
    ref = rhs_cart(U, box, GAS, viscous=viscous, flux="ec_roe")
    got = cv.rhs(U, cv.CurvMesh(3, _box_nodes(box)), GAS, viscous=viscous, flux="ec_roe")
    for v in range(5):
        assert torch.linalg.norm(got[v] - ref[v]) <= 1e-13 * torch.linalg.norm(ref[v])


def _entropy_rate(U, mesh, out):
    from oracle.physics import entropy_variables, primitives
    v = entropy_variables(primitives(U, GAS), GAS)
    wq = mesh.quadrature_weights()
    terms = sum(wq * v[k] * out[k] for k in range(5))
    return terms.sum().item(), terms.abs().sum().item()


@pytest.mark.parametrize("N", [3, 5])
def test_ec_entropy_conservation_on_warped_mesh(N):
    """Euler, central surface flux: the curvilinear entropy-conserving split
    form conserves the total entropy semi-discretely (metric identities plus
    Tadmor's condition); the Kennedy-Gruber form does not; the Roe
    dissipation makes the entropy rate negative."""
    rng = np.random.default_rng(24 + N)
    mesh = _warped(N, (2, 2, 3), amp=0.08)
    U = random_state(mesh, GAS.gamma, GAS.R, rng)
    tot, mag = _entropy_rate(U, mesh, cv.rhs(U, mesh, GAS, viscous=False, central_only=True, flux="ec_roe"))
    assert abs(tot) < 1e-12 * mag
    tot_kg, mag_kg = _entropy_rate(U, mesh, cv.rhs(U, mesh, GAS, viscous=False, central_only=True))
    assert abs(tot_kg) > 1e-6 * mag_kg
    tot_roe, mag_roe = _entropy_rate(U, mesh, cv.rhs(U, mesh, GAS, viscous=False, flux="ec_roe"))
    assert tot_roe < -1e-6 * mag_roe


def test_ec_free_stream_preservation_warped():
    N = 5
    mesh = _warped(N, (2, 2, 3), amp=0.08)
    shape = mesh.shape
    rho, u, v, w, p = 1.3, 0.4, -0.25, 0.15, 2.0
    E = p / (GAS.gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)
    U = torch.stack([torch.full(shape, x, dtype=torch.float64) for x in (rho, rho * u, rho * v, rho * w, E)])
    out = cv.rhs(U, mesh, GAS, flux="ec_roe")
    assert out.abs().max().item() < 1e-12 * (abs(rho * u) + p + E) * 2 * N * N
