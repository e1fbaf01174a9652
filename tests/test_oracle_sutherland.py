"""CPU pins of Sutherland's viscosity law in the oracle's gas model.

* tabulated viscosity of air at atmospheric pressure (200-600 K; e.g. the
  property tables of Incropera & DeWitt, Fundamentals of Heat and Mass
  Transfer, Table A.4) against the law with the usual air constants
  mu_ref = 1.716e-5 Pa s at T_ref = 273.15 K and S = 110.4 K: within 1.5 %
  (a dropped power or a misplaced S misses by 10 % or more);
* mu(T_ref) = mu_ref; the logarithmic slope d ln mu / d ln T = 3/2 - T / (T + S)
  (complex step), which gives the limits mu ~ T^(3/2) for T << S and
  mu ~ T^(1/2) for T >> S;
* kappa(T) / mu(T) = c_p / Pr at every T;
* the operator on a state of uniform temperature T0 (periodic and with
  isothermal walls at T0) equals the constant-viscosity operator with
  mu = mu(T0), to rounding.
The order of the operator with temperature-dependent viscosity is pinned by a
manufactured solution in the operator pins.
"""

import numpy as np
import pytest
import torch

from oracle.dgsem import rhs
from oracle.mesh import Mesh
from oracle.physics import Gas

from _cases import channel_mesh, random_faces, state_from_prims

AIR = Gas(gamma=1.4, R=287.0, mu=1.716e-5, Pr=0.71, sutherland=True, T_ref=273.15, S=110.4)
# T [K] -> mu [1e-7 Pa s], air at 1 atm
TABLE = {200: 132.5, 250: 159.6, 300: 184.6, 350: 208.2, 400: 230.1, 450: 250.7, 500: 270.1, 600: 305.8}


def test_air_viscosity_table():
    for T, mu in TABLE.items():
        got = AIR.mu_of(float(T))
        assert abs(got / (mu * 1e-7) - 1.0) < 0.015, (T, got)


def test_reference_value_and_log_slope():
    assert AIR.mu_of(273.15) == pytest.approx(1.716e-5, rel=1e-15)
    g = Gas(mu=0.3, sutherland=True, T_ref=2.0, S=0.7)
    h = 1e-30
    for T in (1e-3, 0.1, 1.0, 5.0, 1e3):
        # d ln mu / d ln T by the complex step of ln mu(T e^s) at s = 0
        z = torch.tensor(np.log(T) + 1j * h, dtype=torch.complex128)
        slope = (torch.log(g.mu_of(torch.exp(z)))).imag.item() / h
        assert slope == pytest.approx(1.5 - T / (T + 0.7), rel=1e-13, abs=1e-15)
    assert g.mu_of(2.0) == pytest.approx(0.3, rel=1e-15)
    # the constant law ignores T
    assert Gas(mu=0.3).mu_of(123.0) == 0.3


def test_conductivity_ratio():
    for T in (50.0, 273.15, 900.0):
        cp = AIR.gamma * AIR.R / (AIR.gamma - 1.0)
        assert AIR.kappa_of(T) / AIR.mu_of(T) == pytest.approx(cp / AIR.Pr, rel=1e-15)


def _uniform_T_state(mesh, T0, rng):
    X, Y, Z = mesh.coords()
    rho = 1.0 + 0.2 * torch.sin(X + 0.3) * torch.cos(Y) + 0.1 * torch.sin(Z)
    u = 0.3 * torch.sin(Y) * torch.cos(Z)
    v = 0.2 * torch.cos(X + Z)
    w = 0.1 * torch.sin(X - Y)
    if mesh.bc[1] != "periodic":  # no-slip walls at y = -1, 1
        u, v, w = [q * (1 - Y * Y) for q in (u, v, w)]
    p = rho * 1.0 * T0  # R = 1
    return state_from_prims(rho, u, v, w, p, 1.4)


@pytest.mark.parametrize("walls", [False, True])
def test_uniform_temperature_reduces_to_constant_viscosity(walls):
    rng = np.random.default_rng(3)
    T0 = 1.7
    gs = Gas(gamma=1.4, R=1.0, mu=0.01, Pr=0.72, sutherland=True, T_ref=1.0, S=0.4)
    gc = Gas(gamma=1.4, R=1.0, mu=gs.mu_of(T0), Pr=0.72)
    if walls:
        mesh = channel_mesh(3, 2, 3, 2, T_wall=T0)
    else:
        mesh = Mesh(3, tuple(random_faces(n, 0.0, 2 * np.pi, rng) for n in (2, 3, 2)))
    U = _uniform_T_state(mesh, T0, rng)
    a, b = rhs(U, mesh, gs), rhs(U, mesh, gc)
    for v in range(5):
        assert torch.linalg.norm(a[v] - b[v]) <= 1e-13 * torch.linalg.norm(b[v]) + 1e-13
    # and the viscosity matters for this state
    g2 = Gas(gamma=1.4, R=1.0, mu=0.01, Pr=0.72)
    assert torch.linalg.norm(rhs(U, mesh, g2)[1] - b[1]) > 1e-6 * torch.linalg.norm(b[1])


def test_reverse_mode_through_sutherland_matches_complex_step():
    """<(dL/dU)^T lam, v> = <lam, (dL/dU) v>: the oracle's reverse mode through
    mu(T) and kappa(T) against its complex-step derivative (which evaluates the
    law at complex temperatures)."""
    from oracle.adjoint import rhs_jvp_cs, rhs_vjp
    rng = np.random.default_rng(44)
    mesh = Mesh(3, tuple(random_faces(n, 0.0, 2.0, rng) for n in (3, 2, 2)))
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=0.02, Pr=0.72, sutherland=True, T_ref=1.0, S=110.4 / 288.15)
    from _cases import random_state
    U = random_state(mesh, g.gamma, g.R, rng, vel_amp=1.0, p_mean=1.0 / (1.4 * 0.01), p_amp=0.05)
    lam = torch.tensor(rng.standard_normal(U.shape))
    v = torch.tensor(rng.standard_normal(U.shape))
    a = (rhs_vjp(U, lam, mesh, g) * v).sum().item()
    b = (lam * rhs_jvp_cs(U, v, mesh, g)).sum().item()
    assert abs(a - b) <= 1e-13 * abs(b)
