"""CPU pins of the oracle's slip, adiabatic wall with the modelled wall stress.

* lifting: exact for polynomial fields of degree <= N that are continuous
  across elements and whose normal velocity vanishes at the walls (the slip
  wall value keeps the tangential velocity and the temperature);
* global balances, which the DG surface terms must reproduce exactly with LGL
  quadrature: mass and total energy are conserved (no mass flux, pressure-only
  convective flux, adiabatic stationary wall), and the rate of x-momentum is
  minus the face quadrature of the modelled x wall stress over both walls;
* the wall stress enters with the sign of a drag: a flow in +x loses x-momentum.
"""

import numpy as np
import torch

from oracle.basis import lgl
from oracle.dgsem import lift, rhs
from oracle.mesh import Mesh, tanh_faces, uniform_faces
from oracle.physics import Gas
from oracle.wallmodel import wall_stress_field

from _cases import state_from_prims


def _mesh(N, wm_node=2):
    return Mesh(N, (uniform_faces(2, 0, 2.0), tanh_faces(4, 2.0), uniform_faces(2, 0, 1.0)),
                bc=("periodic", "wallmodel", "periodic"), wm_node=wm_node)


def test_lifting_exact_at_slip_walls():
    g = Gas(gamma=1.4, R=1.0, mu=0.01, Pr=0.72)
    m = _mesh(3)
    X, Y, Z = m.coords()
    u = 1.2 + 0.3 * Y + 0.2 * Y ** 2          # slip: any tangential velocity at the wall
    v = 0.1 * (1 - Y ** 2)                    # zero normal velocity at y = +-1
    w = 0.05 * Y ** 3
    T = 1.0 + 0.1 * Y ** 2                    # any temperature (adiabatic: no jump imposed)
    U = state_from_prims(torch.ones_like(X), u, v, w, g.R * T, g.gamma)
    grad = lift(U, m, g)
    assert torch.allclose(grad[0][1], 0.3 + 0.4 * Y, atol=1e-12, rtol=0)
    assert torch.allclose(grad[1][1], -0.2 * Y, atol=1e-12, rtol=0)
    assert torch.allclose(grad[2][1], 0.15 * Y ** 2, atol=1e-12, rtol=0)
    assert torch.allclose(grad[3][1], 0.2 * Y, atol=1e-12, rtol=0)


def test_global_balances_with_wall_model():
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=1e-3, Pr=0.72)
    N = 4
    m = _mesh(N, wm_node=2)
    X, Y, Z = m.coords()
    rng = np.random.default_rng(3)
    u = 1.0 * (1 - Y ** 8) + 0.2 + 0.05 * torch.sin(np.pi * X) * torch.cos(2 * np.pi * Z)
    v = 0.05 * torch.sin(np.pi * X) * (1 - Y ** 2) + 0.01 * torch.as_tensor(rng.standard_normal(X.shape))
    w = 0.05 * torch.cos(2 * np.pi * Z) * (1 - Y ** 2)
    rho = 1.0 + 0.01 * torch.sin(np.pi * X)
    T = torch.ones_like(X)
    U = state_from_prims(rho, u, v, w, rho * g.R * T, g.gamma)
    Ut = rhs(U, m, g)
    wq = m.quadrature_weights().to(torch.float64)
    rate = [(wq * Ut[k]).sum().item() for k in range(5)]
    scale = [(wq * Ut[k].abs()).sum().item() for k in range(5)]
    assert abs(rate[0]) < 1e-12 * scale[0]
    assert abs(rate[4]) < 1e-12 * scale[4]
    # x-momentum: minus the LGL face quadrature of the x wall stress of both walls
    tau = wall_stress_field(U, m, g, m.wm_node, lambda T_: g.mu)  # (2 nx nz, 3, NP^2)
    _, wl = lgl(N)
    wab = (wl[:, None] * wl[None, :]).reshape(-1).numpy()  # node ab = a + NP b -> w_a w_b
    nx, nz = m.nelem[0], m.nelem[2]
    hx = np.diff(m.faces[0]) / 2.0
    hz = np.diff(m.faces[2]) / 2.0
    force = 0.0
    for side in (0, 1):
        for ez in range(nz):
            for ex in range(nx):
                f = side * nx * nz + ex + nx * ez
                force += hx[ex] * hz[ez] * float((wab * tau[f, 0]).sum())
    assert force > 0
    assert abs(rate[1] + force) < 1e-11 * (scale[1] + abs(force))
