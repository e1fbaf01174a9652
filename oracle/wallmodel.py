"""Algebraic equilibrium wall-stress model of the oracle (test infrastructure only).

Paper Sec. 3 (wall models for compressible flows, and their GPU port): at an
interface point a distance h_wm from the wall the model takes the
instantaneous wall-parallel velocity, maps it to an equivalent incompressible
velocity with the Van Driest transform, and solves Spalding's law of the wall
for the wall shear stress, which is then imposed on the viscous flux at a slip
wall.  Spalding's law as the paper prints it (kappa = 0.4, with the quartic
term):

    y+ = u+ + 0.1108 [exp(0.4 u+) - 1 - 0.4 u+ - (0.4 u+)^2/2! - (0.4 u+)^3/3! - (0.4 u+)^4/4!],

u+ = u / u_tau, y+ = h u_tau / nu_w, tau_w = rho_w u_tau^2.

Readings (the paper gives no formulas beyond Spalding's law and refers the
compressible extension to other work):

* interface point: the LGL node n_wm (1 <= n_wm <= N, counted from the wall)
  on the wall-normal line through each wall-face node; h_wm is its distance
  from the wall;
* wall-parallel velocity u_par = |u - (u . n) n| at that node, direction
  t = (u - (u . n) n) / u_par (zero stress if u_par = 0);
* Van Driest transform for an adiabatic wall with the Crocco-Busemann
  temperature T = T_w - r u^2 / (2 c_p): u_VD = int_0^u sqrt(rho / rho_w) du'
  = a arcsin(u_par / a), a^2 = 2 c_p T_w / r, with the adiabatic wall
  temperature T_w = T_h + r u_par^2 / (2 c_p) and recovery factor r = Pr^(1/3);
* wall properties: rho_w = p_h / (R T_w) (pressure constant across the
  layer), mu_w = mu(T_w) of the gas model, nu_w = mu_w / rho_w;
* the root u_tau > 0 of y+(u_tau) - f(u+(u_tau)), which is unique because the
  residual increases strictly with u_tau; here found by Brent's method
  (scipy.optimize.brentq), a different method from the GPU's safeguarded Newton
  iteration, so the two agree only if both find the root;
* output: the wall-stress vector tau_w t per wall-face node.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq

from .physics import Gas

__all__ = ["KAPPA", "SPALDING_C", "exp_tail", "spalding_y_plus", "van_driest", "solve_u_tau", "wall_stress",
           "recovery_factor"]

KAPPA = 0.4
SPALDING_C = 0.1108


def exp_tail(k: float, m: int) -> float:
    """exp(k) - sum_{n < m} k^n / n! for k >= 0: directly for k > 5 (where the
    tail is most of exp(k)), else as the series sum_{n >= m} k^n / n! (no
    cancellation near k = 0; terms to n = m + 44, the last below 1e-29 of the sum)."""
    if k > 5.0:
        return math.exp(k) - sum(k ** n / math.factorial(n) for n in range(m))
    return sum(k ** n / math.factorial(n) for n in range(m, m + 45))


def spalding_y_plus(u_plus: float) -> float:
    """Spalding's law y+(u+) as printed in the paper (quartic variant)."""
    return u_plus + SPALDING_C * exp_tail(KAPPA * u_plus, 5)


def recovery_factor(gas: Gas) -> float:
    return gas.Pr ** (1.0 / 3.0)


def van_driest(u_par: float, T_h: float, gas: Gas):
    """(u_VD, T_w): equivalent incompressible velocity and adiabatic wall temperature."""
    cp = gas.gamma * gas.R / (gas.gamma - 1.0)
    r = recovery_factor(gas)
    T_w = T_h + r * u_par * u_par / (2.0 * cp)
    a = math.sqrt(2.0 * cp * T_w / r)
    return a * math.asin(u_par / a), T_w


def solve_u_tau(u: float, h: float, nu: float) -> float:
    """u_tau > 0 with h u_tau / nu = spalding_y_plus(u / u_tau) (Brent's method)."""
    if u <= 0.0:
        return 0.0

    def F(x):
        if KAPPA * u / x > 700.0:  # exp overflows: far below the root
            return -math.inf
        return h * x / nu - spalding_y_plus(u / x)

    lo = math.sqrt(nu * u / h)  # u+ <= y+ makes this a lower bound of the root
    if F(lo) >= 0.0:  # the root is the bound itself to rounding (deep viscous sublayer)
        return lo
    hi = 2.0 * lo
    while F(hi) <= 0.0:
        lo, hi = hi, 2.0 * hi
    while not math.isfinite(F(lo)):  # stays below the root: F is -inf only for u+ > 1750
        lo = math.sqrt(lo * hi)
    return brentq(F, lo, hi, xtol=1e-300, rtol=4.0 * np.finfo(float).eps, maxiter=500)


def wall_stress(rho: float, vel, p: float, normal, h: float, gas: Gas, mu_of_T):
    """Wall-stress vector (3,) for the state (rho, vel, p) at the interface point
    a distance h from a wall with unit normal `normal` (pointing into the fluid)."""
    vel = np.asarray(vel, dtype=np.float64)
    n = np.asarray(normal, dtype=np.float64)
    ut = vel - np.dot(vel, n) * n
    u_par = float(np.linalg.norm(ut))
    if u_par == 0.0:
        return np.zeros(3)
    T_h = p / (rho * gas.R)
    u_vd, T_w = van_driest(u_par, T_h, gas)
    rho_w = p / (gas.R * T_w)
    nu_w = mu_of_T(T_w) / rho_w
    u_tau = solve_u_tau(u_vd, h, nu_w)
    return rho_w * u_tau * u_tau * ut / u_par


def wall_stress_field(U, mesh, gas: Gas, n_wm: int, mu_of_T) -> np.ndarray:
    """Wall-stress vectors of every wall-face node of the mesh, shaped
    (n_wall_faces, 3, (N+1)^2).  Wall faces in order: wall directions d = x, y, z;
    lower wall then upper wall; the elements of the wall with the first of the
    other two element indices fastest; face nodes (a, b) = (j, k), (i, k), (i, j)
    for d = x, y, z, a fastest."""
    from .basis import lgl
    from .mesh import PERIODIC
    from .physics import primitives
    N, NP = mesh.N, mesh.N + 1
    xi, _ = lgl(N)
    xi = xi.numpy()
    P = primitives(U, gas)
    rho, p = P.rho.numpy(), P.p.numpy()
    vel = [v.numpy() for v in P.vel]
    nel = mesh.nelem  # (nx, ny, nz)
    out = []
    for d in range(3):
        if mesh.bc[d] == PERIODIC:
            continue
        others = [c for c in range(3) if c != d]
        width = np.diff(np.asarray(mesh.faces[d], dtype=np.float64))
        for side in (0, 1):
            ed = 0 if side == 0 else nel[d] - 1
            nd = n_wm if side == 0 else N - n_wm
            h = (xi[n_wm] + 1.0) * width[ed] / 2.0
            normal = np.zeros(3)
            normal[d] = 1.0 if side == 0 else -1.0
            for eb in range(nel[others[1]]):
                for ea in range(nel[others[0]]):
                    e = [0, 0, 0]
                    e[d], e[others[0]], e[others[1]] = ed, ea, eb
                    face = np.zeros((3, NP * NP))
                    for bn in range(NP):
                        for an in range(NP):
                            node = [0, 0, 0]
                            node[d], node[others[0]], node[others[1]] = nd, an, bn
                            idx = (e[2], e[1], e[0], node[2], node[1], node[0])
                            v = [vel[c][idx] for c in range(3)]
                            face[:, an + NP * bn] = wall_stress(rho[idx], v, p[idx], normal, h, gas, mu_of_T)
                    out.append(face)
    return np.array(out).reshape(-1, 3, NP * NP)
