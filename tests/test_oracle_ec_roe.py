"""CPU pins of the oracle's entropy-conserving volume flux and Roe surface flux.

What fixes each function, independently of its own formulas:

* ln_mean: the definition (a - b) / (ln a - ln b) evaluated with 50-digit
  decimal arithmetic;
* ec_flux: consistency with the Euler flux, symmetry, and Tadmor's entropy
  conservation condition [[v]] . f# = [[rho u_d]] with the entropy variables
  of -rho s / (gamma - 1) (the Kennedy-Gruber flux, a negative control, fails it);
* roe_waves: Roe's property U, sum alpha_k r_k = [[U]] and
  sum lambda_k alpha_k r_k = [[f_d]] exactly for the Roe average;
* the Roe dissipation: |A(U~)| [[U]] with A the complex-step Jacobian of the
  Euler flux at the Roe-average state and |A| from numpy's eigendecomposition;
* harten_hyman_abs: >= |lambda|, equal where |lambda| >= delta, continuous at
  delta, delta / 2 at lambda = 0;
* the operator: free-stream preservation (uniform and stretched meshes, walls)
  and semi-discrete entropy conservation, sum_e J_e sum_n w_n v_n . Ut_n = 0, of
  the Euler split form with the entropy-conserving surface flux on a periodic
  mesh (again failed by the Kennedy-Gruber form).
"""

from decimal import Decimal, getcontext

import numpy as np
import pytest
import torch

from oracle.dgsem import rhs
from oracle.mesh import Mesh
from oracle.physics import (Gas, conservative, ec_flux, entropy_variables, euler_flux,
                            harten_hyman_abs, kg_flux, ln_mean, primitives, roe_flux, roe_waves)

from _cases import channel_mesh, random_faces, random_state

GAS = Gas(gamma=1.4, R=1.0, mu=0.0, Pr=0.72)


def _prims(rng, n, vel_amp=1.0, spread=0.5):
    rho = torch.tensor(1.0 + spread * rng.uniform(-1, 1, n))
    u = [torch.tensor(vel_amp * rng.uniform(-1, 1, n)) for _ in range(3)]
    p = torch.tensor(1.0 + spread * rng.uniform(-1, 1, n))
    E = p / (GAS.gamma - 1.0) + 0.5 * rho * sum(x * x for x in u)
    return primitives(torch.stack([rho, rho * u[0], rho * u[1], rho * u[2], E]), GAS)


def _rel(a, b):
    a, b = torch.stack(list(a)), torch.stack(list(b))
    return float((a - b).abs().max() / b.abs().max())


def test_ln_mean_against_decimal_definition():
    getcontext().prec = 50
    rng = np.random.default_rng(1)
    a = 10.0 ** rng.uniform(-2, 2, 400)
    rel = 10.0 ** rng.uniform(-13, 0.0, 400)
    b = a * (1.0 + rel * rng.choice([-0.9, 1.0], 400))
    got = ln_mean(torch.tensor(a), torch.tensor(b)).numpy()
    worst = 0.0
    for x, y, g in zip(a, b, got):
        X, Y = Decimal(float(x)), Decimal(float(y))
        ref = (X - Y) / (X.ln() - Y.ln()) if X != Y else X
        worst = max(worst, abs(float((Decimal(float(g)) - ref) / ref)))
    assert worst < 6e-16, worst
    # equal arguments and symmetry
    t = torch.tensor([0.3, 2.0, 7.5], dtype=torch.float64)
    assert torch.equal(ln_mean(t, t), t)
    assert torch.equal(ln_mean(torch.tensor(a), torch.tensor(b)), ln_mean(torch.tensor(b), torch.tensor(a)))


@pytest.mark.parametrize("d", [0, 1, 2])
def test_ec_flux_consistent_and_symmetric(d):
    rng = np.random.default_rng(2 + d)
    A, B = _prims(rng, 50), _prims(rng, 50)
    assert _rel(ec_flux(A, A, d, GAS), euler_flux(A, d)) < 4e-15
    assert _rel(ec_flux(A, B, d, GAS), ec_flux(B, A, d, GAS)) < 4e-16


@pytest.mark.parametrize("d", [0, 1, 2])
def test_ec_flux_tadmor_entropy_conservation(d):
    rng = np.random.default_rng(10 + d)
    A, B = _prims(rng, 200), _prims(rng, 200)
    vA, vB = entropy_variables(A, GAS), entropy_variables(B, GAS)

    def defect(f):
        terms = [(vB[k] - vA[k]) * f[k] for k in range(5)]
        psi = B.rho * B.vel[d] - A.rho * A.vel[d]
        scale = sum(t.abs() for t in terms) + psi.abs()
        return ((sum(terms) - psi).abs() / scale).max().item()

    assert defect(ec_flux(A, B, d, GAS)) < 2e-13
    assert defect(kg_flux(A, B, d)) > 1e-4  # negative control: not entropy conservative


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_property_u(d):
    rng = np.random.default_rng(20 + d)
    L, R = _prims(rng, 100), _prims(rng, 100)
    lam, alpha, r = roe_waves(L, R, d, GAS)
    UL, UR = conservative(L), conservative(R)
    dU = [sum(alpha[k] * r[k][v] for k in range(4)) for v in range(5)]
    dF = [sum(lam[k] * alpha[k] * r[k][v] for k in range(4)) for v in range(5)]
    fL, fR = euler_flux(L, d), euler_flux(R, d)
    assert _rel(dU, [UR[v] - UL[v] for v in range(5)]) < 1e-13
    assert _rel(dF, [fR[v] - fL[v] for v in range(5)]) < 1e-13


def _euler_flux_cons(Uc, d):
    return torch.stack(euler_flux(primitives(Uc, GAS), d))


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_dissipation_against_eigendecomposition(d):
    rng = np.random.default_rng(30 + d)
    for _ in range(20):
        L, R = _prims(rng, 1), _prims(rng, 1)
        # Roe-average state from its definition
        sl, sr = torch.sqrt(L.rho), torch.sqrt(R.rho)
        u = [(sl * L.vel[c] + sr * R.vel[c]) / (sl + sr) for c in range(3)]
        H = (sl * (L.E + L.p) / L.rho + sr * (R.E + R.p) / R.rho) / (sl + sr)
        rho = sl * sr
        q2 = sum(x * x for x in u)
        p = rho * (GAS.gamma - 1.0) / GAS.gamma * (H - 0.5 * q2)
        E = p / (GAS.gamma - 1.0) + 0.5 * rho * q2
        Ut = torch.stack([rho, rho * u[0], rho * u[1], rho * u[2], E]).reshape(5).to(torch.complex128)
        A = np.zeros((5, 5))
        h = 1e-30
        for j in range(5):
            e = torch.zeros(5, dtype=torch.complex128)
            e[j] = 1j * h
            A[:, j] = (_euler_flux_cons((Ut + e).reshape(5, 1), d).reshape(5).imag / h).numpy()
        ev, V = np.linalg.eig(A)
        absA = np.real(V @ np.diag(np.abs(ev)) @ np.linalg.inv(V))
        dU = (torch.stack(conservative(R)) - torch.stack(conservative(L))).reshape(5).numpy()
        ref = 0.5 * absA @ dU
        central = torch.stack(ec_flux(L, R, d, GAS)).reshape(5).numpy()
        got = central - torch.stack(roe_flux(L, R, d, GAS, entropy_fix=False)).reshape(5).numpy()
        assert np.abs(got - ref).max() < 1e-11 * (np.abs(ref).max() + np.abs(dU).max())


def test_harten_hyman_abs_properties():
    lam = torch.linspace(-2.0, 2.0, 4001, dtype=torch.float64)
    lam_L, lam_R = lam - 0.3, lam + 0.2  # delta = max(0.3, 0.2) = 0.3 everywhere
    a = harten_hyman_abs(lam, lam_L, lam_R)
    assert torch.all(a >= lam.abs() - 1e-16)
    far = lam.abs() >= 0.3
    assert torch.equal(a[far], lam.abs()[far])
    t = lambda x: torch.tensor(x, dtype=torch.float64)  # noqa: E731
    assert abs(harten_hyman_abs(t(0.0), t(-0.3), t(0.2)).item() - 0.15) < 1e-16
    near = harten_hyman_abs(t(0.3 - 1e-12), t(-1e-12), t(0.5 - 1e-12))
    assert abs(near.item() - 0.3) < 1e-11  # continuous at |lambda| = delta
    # no correction when the characteristic speeds do not cross (delta = 0)
    b = harten_hyman_abs(lam, lam + 0.1, lam - 0.1)
    assert torch.equal(b, lam.abs())


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_flux_consistency(d):
    rng = np.random.default_rng(40 + d)
    A = _prims(rng, 30)
    assert _rel(roe_flux(A, A, d, GAS), euler_flux(A, d)) < 4e-15


@pytest.mark.parametrize("viscous", [False, True])
def test_ec_roe_free_stream(viscous):
    g = Gas(gamma=1.4, R=1.0, mu=0.02 if viscous else 0.0, Pr=0.72)
    rng = np.random.default_rng(50)
    mesh = Mesh(3, tuple(random_faces(n, 0.0, 2.0, rng) for n in (3, 2, 3)))
    shape = mesh.shape
    c = [torch.full(shape, x, dtype=torch.float64) for x in (1.2, 0.3, -0.2, 0.1, 3.0)]
    U = torch.stack([c[0], c[0] * c[1], c[0] * c[2], c[0] * c[3],
                     c[4] / 0.4 + 0.5 * c[0] * (c[1] ** 2 + c[2] ** 2 + c[3] ** 2)])
    Ut = rhs(U, mesh, g, viscous=viscous, flux="ec_roe")
    assert Ut.abs().max().item() < 1e-12 * U.abs().max().item()
    # at rest in the stretched channel with isothermal walls at the gas temperature
    mesh = channel_mesh(3, 2, 3, 2, T_wall=2.5)
    shape = mesh.shape
    rho = torch.full(shape, 1.2, dtype=torch.float64)
    z = torch.zeros(shape, dtype=torch.float64)
    U = torch.stack([rho, z, z, z, rho * 2.5 / 0.4])  # p = rho R T, T = 2.5
    Ut = rhs(U, mesh, g, viscous=viscous, flux="ec_roe")
    assert Ut.abs().max().item() < 1e-12 * U.abs().max().item()


@pytest.mark.parametrize("N", [2, 3, 4])
def test_semi_discrete_entropy_conservation(N):
    rng = np.random.default_rng(60 + N)
    mesh = Mesh(N, tuple(random_faces(n, 0.0, 2.0, rng) for n in (2, 3, 2)))
    U = random_state(mesh, GAS.gamma, GAS.R, rng, vel_amp=0.5, p_mean=1.0, p_amp=0.2)
    wq = mesh.quadrature_weights().to(torch.float64)  # w_i w_j w_k J_e per node

    def rate(flux):
        Ut = rhs(U, mesh, GAS, viscous=False, central_only=True, flux=flux)
        v = entropy_variables(primitives(U, GAS), GAS)
        terms = sum(v[k] * Ut[k] for k in range(5)) * wq
        return terms.sum().item() / terms.abs().sum().item()

    assert abs(rate("ec_roe")) < 1e-13
    assert abs(rate("kg_llf")) > 1e-6  # the Kennedy-Gruber split form does not conserve entropy
