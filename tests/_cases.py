"""Small mesh/state builders for the CPU pins of the oracle (no operator arithmetic)."""

import numpy as np
import torch

from oracle.mesh import Mesh, tanh_faces, uniform_faces
from oracle.physics import Gas


def random_faces(n, lo, hi, rng, jitter=0.35):
    f = uniform_faces(n, lo, hi)
    h = (hi - lo) / n
    inner = f[1:-1] + rng.uniform(-jitter, jitter, size=n - 1) * h
    return np.concatenate(([lo], inner, [hi]))


def random_state(mesh, gamma, R, rng, vel_amp=0.5, p_mean=1.0, p_amp=0.2, rho_amp=0.2, const_p=False):
    """Conservative state with rho > 0, p > 0 (independent per node)."""
    shape = mesh.shape
    rho = 1.0 + rho_amp * rng.uniform(-1, 1, size=shape)
    u = vel_amp * rng.uniform(-1, 1, size=(3,) + shape)
    p = np.full(shape, p_mean) if const_p else p_mean * (1.0 + p_amp * rng.uniform(-1, 1, size=shape))
    E = p / (gamma - 1.0) + 0.5 * rho * (u ** 2).sum(0)
    return torch.tensor(np.stack([rho, rho * u[0], rho * u[1], rho * u[2], E]))


def state_from_prims(rho, u, v, w, p, gamma):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return torch.stack([torch.as_tensor(x, dtype=torch.float64) for x in (rho, rho * u, rho * v, rho * w, E)])


def channel_mesh(N, nx, ny, nz, alpha=2.0, T_wall=1.0):
    return Mesh(N, (uniform_faces(nx, 0, 2 * np.pi), tanh_faces(ny, alpha), uniform_faces(nz, 0, np.pi)),
                bc=("periodic", "wall", "periodic"), T_wall=T_wall)


def gas(mu=0.01, gamma=1.4, R=1.0, Pr=0.72):
    return Gas(gamma=gamma, R=R, mu=mu, Pr=Pr)
