"""CPU pins of the oracle's algebraic wall-stress model.

* the returned u_tau satisfies Spalding's law (residual at rounding level) and
  is bracketed by the viscous-sublayer bound u_tau^2 >= nu u / h;
* limits of the law: u+ -> y+ in the viscous sublayer; the log law
  u+ = ln(y+ / 0.1108) / 0.4 deep in the log layer;
* the Van Driest closed form against a numerical quadrature of
  int_0^u sqrt(T_w / T(u')) du' with the Crocco-Busemann temperature, and its
  incompressible limit u_VD -> u;
* the wall stress grows with the velocity, points along the wall-parallel
  velocity and ignores the wall-normal component;
* wall_stress_field: one face per wall element and side, the interface node at
  the stated distance (a state linear in the wall distance makes every node's
  stress equal to the single-point model evaluated at that distance).
"""

import math

import numpy as np
import pytest
import torch
from scipy.integrate import quad

from oracle.mesh import Mesh, tanh_faces, uniform_faces
from oracle.physics import Gas
from oracle.wallmodel import (KAPPA, SPALDING_C, recovery_factor, solve_u_tau, spalding_y_plus,
                              van_driest, wall_stress, wall_stress_field)

GAS = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=1e-4, Pr=0.72)


@pytest.mark.parametrize("u,h,nu", [(1.0, 0.05, 1e-4), (0.3, 1e-3, 1e-4), (2.0, 0.2, 1e-6), (1e-3, 1e-2, 1e-3)])
def test_u_tau_solves_spalding(u, h, nu):
    ut = solve_u_tau(u, h, nu)
    yp, up = h * ut / nu, u / ut
    assert abs(yp - spalding_y_plus(up)) < 1e-12 * yp
    assert ut * ut >= nu * u / h * (1 - 1e-15)


def test_exp_tail_against_decimal():
    from decimal import Decimal, getcontext
    from oracle.wallmodel import exp_tail
    getcontext().prec = 60
    for k in (1e-6, 1e-3, 0.3, 0.99, 1.5, 3.0, 4.99, 5.01, 12.0, 40.0):
        for m in (4, 5):
            K = Decimal(k)
            ref = K.exp() - sum(K ** n / math.factorial(n) for n in range(m))
            assert abs(Decimal(exp_tail(k, m)) - ref) <= Decimal(4e-16) * abs(ref), (k, m)


def test_viscous_sublayer_and_log_law_limits():
    # sublayer: y+ << 1 gives u+ = y+, i.e. u_tau^2 = nu u / h
    u, h, nu = 1e-4, 1e-4, 1e-3
    ut = solve_u_tau(u, h, nu)
    assert abs(ut * ut / (nu * u / h) - 1.0) < 1e-6
    # log layer: y+ = 1e6 gives u+ = ln(y+ / C) / kappa up to the polynomial terms
    nu, h = 1e-6, 1.0
    for up_target in (38.0, 42.0):
        yp = spalding_y_plus(up_target)
        ut = yp * nu / h
        u = up_target * ut
        got = solve_u_tau(u, h, nu)
        assert abs(got / ut - 1.0) < 1e-13
        assert abs(up_target - math.log(yp / SPALDING_C) / KAPPA) < 2e-3


def test_van_driest_closed_form_against_quadrature():
    cp = GAS.gamma * GAS.R / (GAS.gamma - 1.0)
    r = recovery_factor(GAS)
    for u, T_h in ((1.0, 1.0), (3.0, 0.5), (8.0, 1.2)):
        u_vd, T_w = van_driest(u, T_h, GAS)
        assert abs(T_w - (T_h + r * u * u / (2 * cp))) < 1e-15 * T_w
        ref, _ = quad(lambda s: math.sqrt(T_w / (T_w - r * s * s / (2 * cp))), 0.0, u, epsabs=0, epsrel=2e-13)
        assert abs(u_vd - ref) < 1e-12 * ref
        assert u_vd >= u
    # incompressible limit: u / a -> 0
    u_vd, _ = van_driest(1e-6, 1.0, GAS)
    assert abs(u_vd / 1e-6 - 1.0) < 1e-12


def test_wall_stress_direction_and_monotonicity():
    mu = lambda T: 1e-4  # noqa: E731
    n = [0.0, 1.0, 0.0]
    a = wall_stress(1.0, [1.0, 0.0, 0.0], 71.4, n, 0.05, GAS, mu)
    b = wall_stress(1.0, [1.5, 0.0, 0.0], 71.4, n, 0.05, GAS, mu)
    assert a[0] > 0 and b[0] > a[0] and a[1] == 0 and a[2] == 0
    # the wall-normal velocity does not enter; the direction follows u_par
    c = wall_stress(1.0, [0.6, 0.3, 0.8], 71.4, n, 0.05, GAS, mu)
    d = wall_stress(1.0, [0.6, -0.7, 0.8], 71.4, n, 0.05, GAS, mu)
    assert np.allclose(c, d, rtol=0, atol=0)
    assert abs(c[0] / c[2] - 0.6 / 0.8) < 1e-15 and c[1] == 0
    assert np.all(wall_stress(1.0, [0.0, 0.4, 0.0], 71.4, n, 0.05, GAS, mu) == 0)


def test_wall_stress_field_layout_and_distance():
    N = 3
    mesh = Mesh(N, (uniform_faces(2, 0, 1), tanh_faces(3, 2.0), uniform_faces(2, 0, 1)),
                bc=("periodic", "wall", "periodic"), T_wall=1.0)
    nz, ny, nx, NP = mesh.shape[0], mesh.shape[1], mesh.shape[2], mesh.NP
    X, Y, Z = mesh.coords()
    # streamwise velocity linear in the distance from the nearer wall: every
    # node at the interface index has the same state and wall distance up to
    # the element widths of the two wall elements (equal by symmetry)
    dist = 1.0 - torch.abs(Y)
    rho = torch.ones(mesh.shape, dtype=torch.float64)
    u = 3.0 * dist
    p = torch.full(mesh.shape, 71.4, dtype=torch.float64)
    E = p / 0.4 + 0.5 * rho * u * u
    z = torch.zeros_like(u)
    U = torch.stack([rho, rho * u, z, z, E])
    mu = lambda T: 1e-4  # noqa: E731
    for n_wm in (1, 2):
        tau = wall_stress_field(U, mesh, GAS, n_wm, mu)
        assert tau.shape == (2 * nx * nz, 3, NP * NP)
        from oracle.basis import lgl
        xi, _ = lgl(N)
        h = (xi[n_wm].item() + 1.0) * (mesh.faces[1][1] - mesh.faces[1][0]) / 2.0
        ref = wall_stress(1.0, [3.0 * h, 0.0, 0.0], 71.4, [0, 1, 0], h, GAS, mu)
        assert np.allclose(tau[:, 0, :], ref[0], rtol=1e-12, atol=0)
        assert np.all(tau[:, 1:, :] == 0)
