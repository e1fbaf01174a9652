"""Axis-aligned tensor-product hexahedral mesh of the oracle (test infrastructure only).

Elements are boxes [X_a, X_{a+1}] x [Y_b, Y_{b+1}] x [Z_c, Z_{c+1}] given by
strictly increasing face coordinates per direction; every element maps to the
reference cube [-1, 1]^3 by an affine map, so its Jacobian is
J_e = dx dy dz / 8 and the metric scale along direction d is s_d = 2 / d_d
(paper Sec. 2: the operator is applied per hexahedral element; Sec. 3/4 use
periodic and wall boundaries).

Each direction is periodic or closed at both ends by an isothermal no-slip
wall or by a slip, adiabatic wall whose shear stress comes from the wall-stress
model (the wall readings are stated in ``physics`` and ``dgsem``).

Tensor layout used throughout the oracle: a nodal field is a tensor of shape
(nz, ny, nx, N+1, N+1, N+1) indexed [ez, ey, ex, k, j, i]; this is the row-major
view of the canonical flat layout  e = ex + nx (ey + ny ez),
node = i + (N+1) (j + (N+1) k), flat = node + (N+1)^3 e.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .basis import lgl

__all__ = ["Mesh", "ELEM_AXIS", "NODE_AXIS", "uniform_faces", "tanh_faces", "PERIODIC", "WALL",
           "WALL_MODEL"]

# axis of a nodal field (nz, ny, nx, k, j, i) that runs along direction d
ELEM_AXIS = (2, 1, 0)
NODE_AXIS = (5, 4, 3)

PERIODIC = "periodic"
WALL = "wall"
WALL_MODEL = "wallmodel"  # slip, adiabatic wall with the wall-stress model (``wallmodel``)


def uniform_faces(n: int, lo: float, hi: float) -> np.ndarray:
    return lo + (hi - lo) * np.arange(n + 1, dtype=np.float64) / n


def tanh_faces(n: int, alpha: float) -> np.ndarray:
    """Wall-clustered faces on [-1, 1]: y_j = tanh(alpha (2j/n - 1)) / tanh(alpha)."""
    j = np.arange(n + 1, dtype=np.float64)
    return np.tanh(alpha * (2.0 * j / n - 1.0)) / np.tanh(alpha)


@dataclass
class Mesh:
    N: int
    faces: tuple  # three 1-D float64 arrays (x, y, z face coordinates)
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    T_wall: float = 1.0
    wm_node: int = 1  # interface LGL node (from the wall) of WALL_MODEL ends

    def __post_init__(self):
        self.faces = tuple(np.asarray(f, dtype=np.float64) for f in self.faces)
        for f in self.faces:
            if f.ndim != 1 or f.size < 2 or np.any(np.diff(f) <= 0):
                raise ValueError("face coordinates must be strictly increasing")
        for b in self.bc:
            if b not in (PERIODIC, WALL, WALL_MODEL):
                raise ValueError(f"unknown boundary kind {b!r}")

    @property
    def NP(self) -> int:
        return self.N + 1

    @property
    def nelem(self):
        return tuple(f.size - 1 for f in self.faces)  # (nx, ny, nz)

    @property
    def shape(self):
        nx, ny, nz = self.nelem
        NP = self.NP
        return (nz, ny, nx, NP, NP, NP)

    @property
    def n_elements(self) -> int:
        nx, ny, nz = self.nelem
        return nx * ny * nz

    @property
    def n_dof(self) -> int:
        return self.n_elements * self.NP ** 3

    def widths(self, d: int) -> torch.Tensor:
        return torch.tensor(np.diff(self.faces[d]), dtype=torch.float64)

    def scale(self, d: int) -> torch.Tensor:
        """s_d = 2 / width_d, shaped to broadcast against a nodal field."""
        s = 2.0 / self.widths(d)
        shape = [1] * 6
        shape[ELEM_AXIS[d]] = -1
        return s.reshape(shape)

    def jacobian(self) -> torch.Tensor:
        """J_e = dx dy dz / 8, shaped (nz, ny, nx, 1, 1, 1)."""
        jx = self.widths(0).reshape(1, 1, -1, 1, 1, 1) / 2.0
        jy = self.widths(1).reshape(1, -1, 1, 1, 1, 1) / 2.0
        jz = self.widths(2).reshape(-1, 1, 1, 1, 1, 1) / 2.0
        return jx * jy * jz

    def coords(self):
        """Physical node coordinates (x, y, z), each a nodal field."""
        xi, _ = lgl(self.N)
        out = []
        for d in range(3):
            f = torch.tensor(self.faces[d], dtype=torch.float64)
            lo, hi = f[:-1], f[1:]
            # [element, node] table: x = x_lo + (xi + 1) (x_hi - x_lo) / 2
            tab = lo[:, None] + (xi[None, :] + 1.0) * (hi - lo)[:, None] / 2.0
            shape = [1] * 6
            shape[ELEM_AXIS[d]] = tab.shape[0]
            shape[NODE_AXIS[d]] = tab.shape[1]
            out.append(tab.reshape(shape).expand(self.shape).clone())
        return tuple(out)

    def quadrature_weights(self) -> torch.Tensor:
        """w_i w_j w_k J_e per node (the LGL collocation quadrature)."""
        _, w = lgl(self.N)
        wk = w.reshape(1, 1, 1, -1, 1, 1)
        wj = w.reshape(1, 1, 1, 1, -1, 1)
        wi = w.reshape(1, 1, 1, 1, 1, -1)
        return self.jacobian() * wk * wj * wi
