"""Gas model and fluxes of the oracle (test infrastructure only).

Paper Sec. 4: the working fluid is an ideal gas and the scheme is a split-form
DG discretisation with viscous fluxes.  The paper's own production choices
(Chandrashekar entropy-conserving volume flux, Roe/Harten surface flux,
Sutherland viscosity) are not the configuration built here; the workloads use
the readings below, each written from its published definition:

* ideal gas:   p = (gamma - 1) (E - rho |u|^2 / 2),   T = p / (rho R),
               c = sqrt(gamma p / rho),   e = E / rho;
* Euler flux along direction d:
               f_d = (rho u_d, rho u u_d + p delta_1d, rho v u_d + p delta_2d,
                      rho w u_d + p delta_3d, (E + p) u_d);
* Kennedy-Gruber two-point volume flux, {{x}} = (x_a + x_b) / 2:
               f#_d = ({{rho}}{{u_d}}, {{rho}}{{u_d}}{{u}} + {{p}} delta_1d, ...,
                       {{rho}}{{u_d}}{{e}} + {{p}}{{u_d}});
* Newtonian/Fourier viscous flux with constant viscosity mu,
  tau = mu (grad u + grad u^T - 2/3 (div u) I), kappa = mu gamma R / ((gamma-1) Pr):
               f_v,d = (0, tau_1d, tau_2d, tau_3d, u_a tau_ad + kappa dT/dx_d);
* local Lax-Friedrichs (Rusanov) surface flux whose central part is the
  Kennedy-Gruber flux: F* = f#_d(U_L, U_R) - lambda/2 (U_R - U_L),
  lambda = max(|u_d,L| + c_L, |u_d,R| + c_R);
* isothermal no-slip wall: convective flux (0, p_int n, 0) with the interior
  pressure; lifting wall value (u, v, w, T) = (0, 0, 0, T_wall); viscous flux
  f_v with zero wall velocity and the interior gradients.

All functions are complex-step safe: |z| and max(a, b) take the branch chosen
by the real part (ties go to the first argument).
"""

from __future__ import annotations

from dataclasses import dataclass

import torch

__all__ = ["Gas", "primitives", "euler_flux", "kg_flux", "viscous_flux",
           "llf_flux", "wall_convective_flux", "rabs", "rmax"]


@dataclass(frozen=True)
class Gas:
    gamma: float = 1.4
    R: float = 1.0
    mu: float = 0.0
    Pr: float = 0.72

    @property
    def kappa(self) -> float:
        return self.mu * self.gamma * self.R / ((self.gamma - 1.0) * self.Pr)

    @property
    def cv(self) -> float:
        return self.R / (self.gamma - 1.0)


def _re(z: torch.Tensor) -> torch.Tensor:
    return torch.real(z) if z.is_complex() else z


def rabs(z: torch.Tensor) -> torch.Tensor:
    """|z| for real z, and its analytic continuation sign(Re z) z for complex z."""
    return z * torch.sign(_re(z))


def rmax(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """max(a, b) choosing by real part; ties go to a."""
    return torch.where(_re(a) >= _re(b), a, b)


class Prim:
    """Primitive variables at a set of nodes (all tensors of one shape)."""

    __slots__ = ("rho", "vel", "p", "T", "e", "E")

    def __init__(self, rho, vel, p, T, e, E):
        self.rho, self.vel, self.p, self.T, self.e, self.E = rho, vel, p, T, e, E

    def c(self, gas: Gas):
        return torch.sqrt(gas.gamma * self.p / self.rho)


def primitives(U, gas: Gas) -> Prim:
    """Ideal-gas recovery of (rho, u, v, w, p, T, e) from U = (rho, rho u, rho v, rho w, E)."""
    rho, mx, my, mz, E = U[0], U[1], U[2], U[3], U[4]
    u, v, w = mx / rho, my / rho, mz / rho
    p = (gas.gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w))
    T = p / (rho * gas.R)
    e = E / rho
    return Prim(rho, (u, v, w), p, T, e, E)


def conservative(P: Prim):
    rho = P.rho
    return [rho, rho * P.vel[0], rho * P.vel[1], rho * P.vel[2], P.E]


def euler_flux(P: Prim, d: int):
    ud = P.vel[d]
    f = [P.rho * ud]
    for a in range(3):
        fa = P.rho * P.vel[a] * ud
        if a == d:
            fa = fa + P.p
        f.append(fa)
    f.append((P.E + P.p) * ud)
    return f


def kg_flux(A: Prim, B: Prim, d: int):
    """Kennedy-Gruber two-point flux f#_d(A, B) (symmetric in A, B)."""
    avg = lambda x, y: 0.5 * (x + y)  # noqa: E731
    rho = avg(A.rho, B.rho)
    ud = avg(A.vel[d], B.vel[d])
    p = avg(A.p, B.p)
    e = avg(A.e, B.e)
    mass = rho * ud
    f = [mass]
    for a in range(3):
        fa = mass * avg(A.vel[a], B.vel[a])
        if a == d:
            fa = fa + p
        f.append(fa)
    f.append(mass * e + p * ud)
    return f


def viscous_flux(vel, grad, d: int, gas: Gas):
    """f_v,d for velocity vel = (u, v, w) and grad[q][b] = d q / d x_b, q in (u, v, w, T)."""
    mu = gas.mu
    div = grad[0][0] + grad[1][1] + grad[2][2]
    tau = []
    for a in range(3):
        t = mu * (grad[a][d] + grad[d][a])
        if a == d:
            t = t - (2.0 / 3.0) * mu * div
        tau.append(t)
    energy = vel[0] * tau[0] + vel[1] * tau[1] + vel[2] * tau[2] + gas.kappa * grad[3][d]
    zero = torch.zeros_like(tau[0])
    return [zero, tau[0], tau[1], tau[2], energy]


def llf_flux(L: Prim, R: Prim, UL, UR, d: int, gas: Gas, central_only: bool = False):
    """Local Lax-Friedrichs flux with the Kennedy-Gruber flux as its central part."""
    f = kg_flux(L, R, d)
    if central_only:
        return f
    lam = rmax(rabs(L.vel[d]) + L.c(gas), rabs(R.vel[d]) + R.c(gas))
    return [f[v] - 0.5 * lam * (UR[v] - UL[v]) for v in range(5)]


def wall_convective_flux(P: Prim, d: int):
    """Convective flux through an impermeable wall: only the interior pressure acts."""
    zero = torch.zeros_like(P.p)
    f = [zero]
    for a in range(3):
        f.append(P.p if a == d else zero)
    f.append(zero)
    return f
