"""Derivatives of the oracle operator (test infrastructure only).

* ``rhs_vjp``: (dL/dU)^T lam by reverse-mode differentiation (torch.autograd)
  of the oracle's own ``rhs``; exact up to rounding for the function the oracle
  computes.  Non-smooth points (|.| and max in the Lax-Friedrichs speed) take
  the derivative of the branch chosen by the real part, ties to the first
  argument (reading; such points have measure zero for random states).
* ``rhs_jvp_cs``: (dL/dU) v by the complex step Im L(U + i h v) / h, which has
  no subtractive cancellation; pins ``rhs_vjp`` through <lam, J v> = <J^T lam, v>.
* ``rollout_grad``: gradient of J(U_T) = kinetic_energy after nsteps RK steps
  with respect to the initial nodal state U_0 (Euclidean, not mass-weighted).
* ``ke_grad``: closed form dJ/dU = (w J / |Omega|) (-|u|^2/2, u, v, w, 0).
"""

from __future__ import annotations

import torch

from .dgsem import kinetic_energy, rhs, rk_step
from .mesh import Mesh
from .physics import Gas

__all__ = ["rhs_vjp", "rhs_jvp_cs", "rollout", "rollout_grad", "rollout_dir_cs",
           "ke_grad"]


def rhs_vjp(U: torch.Tensor, lam: torch.Tensor, mesh: Mesh, gas: Gas, **opts) -> torch.Tensor:
    Ur = U.detach().clone().requires_grad_(True)
    out = rhs(Ur, mesh, gas, **opts)
    (g,) = torch.autograd.grad(out, Ur, grad_outputs=lam)
    return g.detach()


def rhs_jvp_cs(U: torch.Tensor, v: torch.Tensor, mesh: Mesh, gas: Gas, h: float = 1e-30,
               **opts) -> torch.Tensor:
    Uc = U.to(torch.complex128) + 1j * h * v.to(torch.complex128)
    return torch.imag(rhs(Uc, mesh, gas, **opts)) / h


def rollout(U0: torch.Tensor, mesh: Mesh, gas: Gas, dt: float, nsteps: int, **opts):
    return kinetic_energy(rk_step(U0, mesh, gas, dt, nsteps, **opts), mesh)


def rollout_grad(U0: torch.Tensor, mesh: Mesh, gas: Gas, dt: float, nsteps: int, **opts):
    Ur = U0.detach().clone().requires_grad_(True)
    J = rollout(Ur, mesh, gas, dt, nsteps, **opts)
    (g,) = torch.autograd.grad(J, Ur)
    return J.detach(), g.detach()


def rollout_dir_cs(U0: torch.Tensor, d: torch.Tensor, mesh: Mesh, gas: Gas, dt: float,
                   nsteps: int, h: float = 1e-30, **opts) -> float:
    """Directional derivative <dJ/dU0, d> by the complex step through the whole rollout."""
    Uc = U0.to(torch.complex128) + 1j * h * d.to(torch.complex128)
    return float(torch.imag(rollout(Uc, mesh, gas, dt, nsteps, **opts))) / h


def ke_grad(U: torch.Tensor, mesh: Mesh) -> torch.Tensor:
    wq = mesh.quadrature_weights()
    scale = wq / wq.sum()
    rho = U[0]
    u, v, w = U[1] / rho, U[2] / rho, U[3] / rho
    return torch.stack([scale * (-0.5 * (u * u + v * v + w * w)), scale * u, scale * v,
                        scale * w, torch.zeros_like(rho)])
