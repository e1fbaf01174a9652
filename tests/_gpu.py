"""Helpers shared by the GPU parity tests: building matching oracle/HIP cases
from one seeded input, error metrics, and oracle patches for sampled checks."""

import sys

import numpy as np
import pytest
import torch

from oracle.dgsem import from_flat
from oracle.mesh import Mesh
from oracle.physics import Gas
from paper_2606_18927_amd import dgsem, workloads

requires_gpu = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_mesh(wl):
    return Mesh(wl.N, wl.faces(), bc=wl.bc, T_wall=wl.T_wall, wm_node=wl.wm_node)


def oracle_gas(wl):
    if wl.sutherland is None:
        return Gas(gamma=wl.gamma, R=wl.R, mu=wl.mu, Pr=wl.Pr)
    return Gas(gamma=wl.gamma, R=wl.R, mu=wl.mu, Pr=wl.Pr, sutherland=True, T_ref=wl.sutherland[0],
               S=wl.sutherland[1])


def state(wl):
    """Seeded conservative state (5, nz, ny, nx, NP, NP, NP) and dt.

    Node positions use the library's own LGL nodes; the state is an input to
    both sides, so where its node positions came from does not matter."""
    xi, _ = dgsem.lgl(wl.N)
    return workloads.make_state(wl, xi)


def to_dev(U):
    return torch.as_tensor(np.ascontiguousarray(U).reshape(-1), dtype=torch.float64).cuda()


def rel_l2(got, ref):
    """Per-variable relative L2 error of (5, ...) arrays."""
    g = np.asarray(got).reshape(5, -1)
    r = np.asarray(ref).reshape(5, -1)
    return np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)


def grad_rel_err(got, ref):
    """Per-component relative L2 error of (12, ...) gradient arrays.  A component
    that vanishes mathematically (e.g. grad T of an isothermal state) holds only
    rounding noise of size eps |q| s sum|D|, so its norm is floored at 0.1 of the
    largest component (all lifted quantities are O(1) in these workloads)."""
    g = np.asarray(got).reshape(12, -1)
    r = np.asarray(ref).reshape(12, -1)
    nr = np.linalg.norm(r, axis=1)
    return np.linalg.norm(g - r, axis=1) / np.maximum(nr, 0.1 * nr.max())


def custom(kind, N, nelem, **kw):
    return workloads.Workload(f"{kind}_n{N}_{nelem}", kind, N, tuple(nelem), nsteps=1, **kw)


def periodic_patch(U, center, radius):
    """Elements within `radius` of `center` (ex, ey, ez), periodic wrap, of a
    state shaped (5, nz, ny, nx, ...): returns the (5, p, p, p, ...) sub-block."""
    nz, ny, nx = U.shape[1:4]
    ex, ey, ez = center
    ix = [(ex + o) % nx for o in range(-radius, radius + 1)]
    iy = [(ey + o) % ny for o in range(-radius, radius + 1)]
    iz = [(ez + o) % nz for o in range(-radius, radius + 1)]
    return U[:, iz][:, :, iy][:, :, :, ix]


def uniform_patch_mesh(N, h, radius, gas_wl):
    p = 2 * radius + 1
    faces = tuple(h[d] * np.arange(p + 1, dtype=np.float64) for d in range(3))
    return Mesh(N, faces, bc=("periodic",) * 3, T_wall=gas_wl.T_wall)


__all__ = ["requires_gpu", "need_gpu", "say", "oracle_mesh", "oracle_gas", "state", "to_dev",
           "rel_l2", "grad_rel_err", "custom", "periodic_patch", "uniform_patch_mesh", "from_flat"]
