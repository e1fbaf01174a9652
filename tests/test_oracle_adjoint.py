"""Pins of the oracle's derivatives (CPU only).

The reverse-mode VJP of the oracle is checked against the complex-step JVP
(no cancellation, exact to rounding) through the dot-product identity
<lam, J v> = <J^T lam, v>, against a brute-force complex-step Jacobian on a tiny
mesh, and the rollout gradient against complex-step directional derivatives
of the whole RK rollout.  The kinetic-energy gradient has a closed form.
"""

import numpy as np
import pytest
import torch

from oracle.adjoint import ke_grad, rhs_jvp_cs, rhs_vjp, rollout, rollout_dir_cs, rollout_grad
from oracle.dgsem import kinetic_energy
from oracle.mesh import Mesh, uniform_faces

from _cases import channel_mesh, gas, random_faces, random_state


def _periodic(N, n, seed):
    rng = np.random.default_rng(seed)
    return Mesh(N, tuple(random_faces(k, 0.0, 2.0 + d, rng) for d, k in enumerate(n)))


@pytest.mark.parametrize("kind", ["periodic", "channel"])
def test_vjp_dot_product_against_complex_step(kind):
    rng = np.random.default_rng(5)
    g = gas(mu=0.05)
    m = _periodic(3, (2, 3, 2), 5) if kind == "periodic" else channel_mesh(2, 2, 3, 2)
    U = random_state(m, g.gamma, g.R, rng)
    for _ in range(3):
        lam = torch.tensor(rng.standard_normal(U.shape))
        v = torch.tensor(rng.standard_normal(U.shape))
        lhs = (lam * rhs_jvp_cs(U, v, m, g)).sum().item()
        rhs_ = (rhs_vjp(U, lam, m, g) * v).sum().item()
        assert abs(lhs - rhs_) < 1e-12 * (abs(lhs) + 1.0), (lhs, rhs_)


def test_vjp_equals_brute_force_jacobian_transpose():
    rng = np.random.default_rng(6)
    g = gas(mu=0.1)
    m = Mesh(1, (uniform_faces(2, 0, 1), uniform_faces(2, 0, 1.5), uniform_faces(2, 0, 2)))
    U = random_state(m, g.gamma, g.R, rng)
    n = U.numel()
    J = torch.zeros(n, n, dtype=torch.float64)
    for k in range(n):
        e = torch.zeros(n, dtype=torch.float64)
        e[k] = 1.0
        J[:, k] = rhs_jvp_cs(U, e.reshape(U.shape), m, g).reshape(-1)
    lam = torch.tensor(rng.standard_normal(U.shape))
    want = (J.T @ lam.reshape(-1)).reshape(U.shape)
    got = rhs_vjp(U, lam, m, g)
    assert torch.allclose(got, want, rtol=1e-12, atol=1e-12 * want.abs().max().item())


def test_kinetic_energy_gradient_closed_form():
    rng = np.random.default_rng(8)
    g = gas()
    m = channel_mesh(3, 2, 2, 2)
    U = random_state(m, g.gamma, g.R, rng).requires_grad_(True)
    (auto,) = torch.autograd.grad(kinetic_energy(U, m), U)
    assert torch.allclose(auto, ke_grad(U.detach(), m), rtol=1e-13, atol=1e-18)


def test_rollout_gradient_against_complex_step_directions():
    rng = np.random.default_rng(9)
    g = gas(mu=0.05)
    m = channel_mesh(2, 2, 2, 2)
    U0 = random_state(m, g.gamma, g.R, rng, vel_amp=0.3)
    dt, nsteps = 2e-3, 3
    J, grad = rollout_grad(U0, m, g, dt, nsteps)
    assert abs(J.item() - rollout(U0, m, g, dt, nsteps).item()) < 1e-15
    for r in range(3):
        d = torch.tensor(rng.standard_normal(U0.shape)) * U0.abs().mean(dim=tuple(range(1, 7)), keepdim=True)
        cs = rollout_dir_cs(U0, d, m, g, dt, nsteps)
        ad = (grad * d).sum().item()
        assert abs(cs - ad) < 1e-12 * (abs(cs) + 1e-12), (cs, ad)


@pytest.mark.parametrize("kind,amp", [("periodic", 0.2), ("channel", 0.2), ("periodic", 0.004)])
def test_ec_roe_vjp_dot_product_against_complex_step(kind, amp):
    """The entropy-conserving volume flux with Roe's surface flux: density and
    pressure spreads of 20 % put most logarithmic means on the atanh form,
    0.4 % keeps them all on the series (f^2 < 1e-4)."""
    rng = np.random.default_rng(9)
    g = gas(mu=0.05)
    m = _periodic(3, (2, 3, 2), 7) if kind == "periodic" else channel_mesh(2, 2, 3, 2)
    U = random_state(m, g.gamma, g.R, rng, p_amp=amp, rho_amp=amp)
    for _ in range(3):
        lam = torch.tensor(rng.standard_normal(U.shape))
        v = torch.tensor(rng.standard_normal(U.shape))
        lhs = (lam * rhs_jvp_cs(U, v, m, g, flux="ec_roe")).sum().item()
        rhs_ = (rhs_vjp(U, lam, m, g, flux="ec_roe") * v).sum().item()
        assert abs(lhs - rhs_) < 1e-12 * (abs(lhs) + 1.0), (lhs, rhs_)


def test_ln_mean_derivative_closed_form():
    """d/da of the logarithmic mean (a - b) / ln(a / b) is
    (ln(a / b) - (a - b) / a) / ln(a / b)^2; on both sides of the series switch."""
    from oracle.physics import ln_mean
    a0 = torch.tensor([1.3, 0.7, 1.0, 2.0, 1.01, 0.995], dtype=torch.float64)
    b = torch.tensor([1.0, 1.0, 1.2, 1.9, 1.0, 1.0], dtype=torch.float64)
    a = a0.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(ln_mean(a, b).sum(), a)
    L = torch.log(a0 / b)
    want = (L - (a0 - b) / a0) / (L * L)
    assert torch.allclose(g, want, rtol=1e-9, atol=0)
