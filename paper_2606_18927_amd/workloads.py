"""Seeded synthetic inputs: Taylor-Green vortex and stretched-channel states.

This module is the only code shared by the HIP path's callers and the CPU
oracle's tests, and it holds none of the operator's arithmetic: it turns an
analytic initial condition into a conservative nodal state, picks a time step
from the initial primitive fields, and draws the seeded perturbations and
finite-difference directions.  Node positions come from the caller (the LGL
nodes ``xi`` of whichever implementation is used), so no basis code lives here.

Initial conditions (the paper prescribes no workload for the operator itself;
Sec. 2.2 notes that its throughput does not depend on the solution, and Sec. 3
uses a channel with a wall-refined y spacing and perturbed velocities):

* Taylor-Green vortex on [0, 2 pi]^3 at Ma = 0.1, Re = 1600, Pr = 0.72,
  gamma = 1.4 with rho0 = U0 = L = 1 and T0 = 1 (so R = p0 = 1/(gamma Ma^2)):
    u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = p0 + (cos 2x + cos 2y)(cos 2z + 2)/16,  rho = p / (R T0);
  optionally plus a velocity perturbation amp * U(-1, 1) drawn per node and
  component (numpy PCG64, canonical node order, components u, v, w).
* Channel [0, 2 pi] x [-1, 1] x [0, pi], y faces tanh(alpha (2j/n - 1))/tanh(alpha)
  with alpha = 2, isothermal walls at y = +-1 (T_wall = 1), bulk Ma = 0.1,
  Re_b = U_b (2 delta) / nu = 5600: rho = 1, T = 1, R = 1/(gamma Ma^2),
    u = 1.5 (1 - y^2) + a (1 - y^2) xi_u,  v = a (1 - y^2) xi_v,
    w = a (1 - y^2) xi_w,  a = 0.05,  xi ~ U(-1, 1).
The conservative energy of a state is E = p/(gamma - 1) + rho |u|^2 / 2.

Time step (held fixed over a run):
  dt = CFL * min over nodes of 1 / sum_d [ (2N+1)(|u_d| + c)/h_d
                                           + (2N+1)^2 max(4/3, gamma/Pr) (mu/rho)/h_d^2 ]
with h_d the element width; it only selects an input, parity does not depend on it.

Layout of every returned state: float64 array of shape (5, nz, ny, nx, N+1, N+1, N+1),
which is the canonical flat layout [v][e][k][j][i] with e = ex + nx (ey + ny ez).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "WORKLOADS", "tgv_faces", "channel_faces", "node_coords", "warped_nodes", "wavy_channel_nodes",
           "make_state", "cfl_dt", "fd_direction"]

TGV_SEED = 20260001
CHANNEL_SEED = 20260003


@dataclass
class Workload:
    name: str
    kind: str                 # "tgv" | "channel" | "freestream"
    N: int
    nelem: tuple              # (nx, ny, nz)
    nsteps: int
    precision: str = "fp64"   # "fp64" | "mixed"
    noise: float = 0.0
    seed: int = TGV_SEED
    cfl: float = 0.5
    checkpoint_every: int = 0
    flux: str = "kg_llf"      # "kg_llf" | "ec_roe"
    wall: str = "wall"        # channel ends: "wall" (isothermal) | "wallmodel" (slip, modelled stress)
    wm_node: int = 1          # interface LGL node of "wallmodel" ends
    sutherland: tuple | None = None  # (T_ref, S) of Sutherland's law; None: constant viscosity
    warp: float = 0.0         # > 0: curved elements, the periodic warped box of warped_nodes(amp=warp)
    extra: dict = field(default_factory=dict)

    # gas / physics parameters -------------------------------------------
    @property
    def gamma(self) -> float:
        return 1.4

    @property
    def Ma(self) -> float:
        return 0.1

    @property
    def R(self) -> float:
        return 1.0 / (self.gamma * self.Ma ** 2)

    @property
    def mu(self) -> float:
        return 1.0 / 1600.0 if self.kind in ("tgv", "freestream") else 2.0 / 5600.0

    @property
    def Pr(self) -> float:
        return 0.72

    @property
    def T_wall(self) -> float:
        return 1.0

    @property
    def bc(self):
        return ("periodic", self.wall, "periodic") if self.kind == "channel" else ("periodic",) * 3

    def faces(self):
        nx, ny, nz = self.nelem
        if self.kind == "channel":
            return channel_faces(nx, ny, nz)
        return tgv_faces(nx), tgv_faces(ny), tgv_faces(nz)

    def nodes(self, xi):
        """Node coordinates (3, nz, ny, nx, NP, NP, NP) of a curved workload, else None."""
        if not self.warp:
            return None
        lengths = tuple(float(f[-1] - f[0]) for f in self.faces())
        return warped_nodes(xi, self.nelem, lengths, self.warp)

    @property
    def n_dof(self) -> int:
        nx, ny, nz = self.nelem
        return nx * ny * nz * (self.N + 1) ** 3


WORKLOADS = {
    # small Taylor-Green case: full oracle comparison in seconds
    "tgv_n3_4x4x4": Workload("tgv_n3_4x4x4", "tgv", 3, (4, 4, 4), nsteps=10),
    # N=7 Taylor-Green with 1 % seeded velocity noise, 16.8 M nodes
    "tgv_n7_32x32x32": Workload("tgv_n7_32x32x32", "tgv", 7, (32, 32, 32), nsteps=100,
                                noise=0.01, seed=TGV_SEED),
    "tgv_n7_32x32x32_mixed": Workload("tgv_n7_32x32x32_mixed", "tgv", 7, (32, 32, 32),
                                      nsteps=100, noise=0.01, seed=TGV_SEED, precision="mixed"),
    # the same with the entropy-conserving volume flux and the Roe surface flux
    "tgv_n7_32x32x32_ec": Workload("tgv_n7_32x32x32_ec", "tgv", 7, (32, 32, 32), nsteps=100,
                                   noise=0.01, seed=TGV_SEED, flux="ec_roe"),
    # the same with Sutherland's law (air's S / T_ref = 110.4 K / 288.15 K, T_ref = T0)
    "tgv_n7_32x32x32_sutherland": Workload("tgv_n7_32x32x32_sutherland", "tgv", 7, (32, 32, 32),
                                           nsteps=100, noise=0.01, seed=TGV_SEED,
                                           sutherland=(1.0, 110.4 / 288.15)),
    # the same on curved elements: the periodic box warped by 5 % of its size
    "tgv_n7_32x32x32_curved": Workload("tgv_n7_32x32x32_curved", "tgv", 7, (32, 32, 32), nsteps=100,
                                       noise=0.01, seed=TGV_SEED, warp=0.05),
    # the paper's throughput workload: a uniform free stream in the periodic
    # box at N = 7 (its throughput does not depend on the solution)
    "freestream_n7_32x32x32": Workload("freestream_n7_32x32x32", "freestream", 7, (32, 32, 32), nsteps=100),
    # small curved Taylor-Green case for full oracle comparisons
    "tgv_n3_4x4x4_curved": Workload("tgv_n3_4x4x4_curved", "tgv", 3, (4, 4, 4), nsteps=10, warp=0.05),
    # stretched channel for the adjoint: N=5, 16^3 elements, 50 steps
    "channel_n5_16x16x16": Workload("channel_n5_16x16x16", "channel", 5, (16, 16, 16),
                                    nsteps=50, seed=CHANNEL_SEED),
    # large stretched channel: N=5, 48x32x48 elements, 500 steps, checkpoint every 25
    "channel_n5_48x32x48": Workload("channel_n5_48x32x48", "channel", 5, (48, 32, 48),
                                    nsteps=500, seed=CHANNEL_SEED, precision="mixed",
                                    checkpoint_every=25),
    # the large channel with wall-modelled slip walls (interface node 2) and
    # Sutherland's law, FP64
    "channel_n5_48x32x48_wm": Workload("channel_n5_48x32x48_wm", "channel", 5, (48, 32, 48),
                                       nsteps=100, seed=CHANNEL_SEED, wall="wallmodel", wm_node=2,
                                       sutherland=(1.0, 110.4 / 288.15)),
}


def tgv_faces(n: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(n + 1, dtype=np.float64) / n


def channel_faces(nx: int, ny: int, nz: int, alpha: float = 2.0):
    fx = 2.0 * np.pi * np.arange(nx + 1, dtype=np.float64) / nx
    j = np.arange(ny + 1, dtype=np.float64)
    fy = np.tanh(alpha * (2.0 * j / ny - 1.0)) / np.tanh(alpha)
    fz = np.pi * np.arange(nz + 1, dtype=np.float64) / nz
    return fx, fy, fz


def node_coords(xi, faces):
    """Node coordinates (X, Y, Z), each shaped (nz, ny, nx, NP, NP, NP)."""
    xi = np.asarray(xi, dtype=np.float64)
    NP = xi.size
    tabs = []
    for f in faces:
        f = np.asarray(f, dtype=np.float64)
        tabs.append(f[:-1, None] + (xi[None, :] + 1.0) * np.diff(f)[:, None] / 2.0)
    nx, ny, nz = (t.shape[0] for t in tabs)
    X = tabs[0].reshape(1, 1, nx, 1, 1, NP)
    Y = tabs[1].reshape(1, ny, 1, 1, NP, 1)
    Z = tabs[2].reshape(nz, 1, 1, NP, 1, 1)
    shape = (nz, ny, nx, NP, NP, NP)
    return (np.broadcast_to(X, shape).copy(), np.broadcast_to(Y, shape).copy(),
            np.broadcast_to(Z, shape).copy())


def warped_nodes(xi, nelem, lengths=(2.0 * np.pi,) * 3, amp=0.05):
    """Node coordinates (3, nz, ny, nx, NP, NP, NP) of a periodic warped box: the
    uniform tensor mesh of [0, L_x] x [0, L_y] x [0, L_z] with nelem elements,
    node positions x_lo (1 - xi)/2 + x_hi (1 + xi)/2 (exact at the element
    ends, so neighbours share their face nodes), each displaced by
      dx = amp L_x sin(2 pi y / L_y) sin(2 pi z / L_z),
      dy = amp L_y sin(2 pi x / L_x) sin(2 pi z / L_z),
      dz = amp L_z sin(2 pi x / L_x) sin(2 pi y / L_y)
    evaluated at the undisplaced position; the displacement is periodic, so
    the mesh stays periodic with the box's periods."""
    xi = np.asarray(xi, dtype=np.float64)
    NP = xi.size
    tabs = []
    for n, L in zip(nelem, lengths):
        f = L * np.arange(n + 1, dtype=np.float64) / n
        tabs.append(f[:-1, None] * (1.0 - xi[None, :]) / 2.0 + f[1:, None] * (1.0 + xi[None, :]) / 2.0)
    nx, ny, nz = nelem
    shape = (nz, ny, nx, NP, NP, NP)
    X = np.broadcast_to(tabs[0].reshape(1, 1, nx, 1, 1, NP), shape)
    Y = np.broadcast_to(tabs[1].reshape(1, ny, 1, 1, NP, 1), shape)
    Z = np.broadcast_to(tabs[2].reshape(nz, 1, 1, NP, 1, 1), shape)
    Lx, Ly, Lz = lengths
    sx, sy, sz = np.sin(2 * np.pi * X / Lx), np.sin(2 * np.pi * Y / Ly), np.sin(2 * np.pi * Z / Lz)
    return np.stack([X + amp * Lx * sy * sz, Y + amp * Ly * sx * sz, Z + amp * Lz * sx * sy])


def wavy_channel_nodes(xi, nelem, lengths=(2.0 * np.pi, 2.0, np.pi), amp=0.05):
    """Node coordinates (3, nz, ny, nx, NP, NP, NP) of a channel with wavy walls:
    the uniform tensor mesh of [0, L_x] x [-L_y/2, L_y/2] x [0, L_z] (nodes
    exact at the element ends), each node displaced by
      dx = amp L_x sin(2 pi z / L_z) cos(pi y / L_y),
      dy = amp L_y sin(2 pi x / L_x) sin(2 pi z / L_z) / 2,
      dz = amp L_z sin(2 pi x / L_x) cos(pi y / L_y),
    at its undisplaced position: periodic in x and z, walls y = +-L_y/2 + dy."""
    xi = np.asarray(xi, dtype=np.float64)
    NP = xi.size
    lo = (0.0, -lengths[1] / 2.0, 0.0)
    tabs = []
    for n, L, a in zip(nelem, lengths, lo):
        f = a + L * np.arange(n + 1, dtype=np.float64) / n
        tabs.append(f[:-1, None] * (1.0 - xi[None, :]) / 2.0 + f[1:, None] * (1.0 + xi[None, :]) / 2.0)
    nx, ny, nz = nelem
    shape = (nz, ny, nx, NP, NP, NP)
    X = np.broadcast_to(tabs[0].reshape(1, 1, nx, 1, 1, NP), shape)
    Y = np.broadcast_to(tabs[1].reshape(1, ny, 1, 1, NP, 1), shape)
    Z = np.broadcast_to(tabs[2].reshape(nz, 1, 1, NP, 1, 1), shape)
    Lx, Ly, Lz = lengths
    sx, sz, cy = np.sin(2 * np.pi * X / Lx), np.sin(2 * np.pi * Z / Lz), np.cos(np.pi * Y / Ly)
    return np.stack([X + amp * Lx * sz * cy, Y + amp * Ly * sx * sz / 2.0, Z + amp * Lz * sx * cy])


def _widths(faces):
    """Element width of each direction broadcast to nodal shape."""
    hx = np.diff(faces[0]).reshape(1, 1, -1, 1, 1, 1)
    hy = np.diff(faces[1]).reshape(1, -1, 1, 1, 1, 1)
    hz = np.diff(faces[2]).reshape(-1, 1, 1, 1, 1, 1)
    return hx, hy, hz


def _prim_state(wl: Workload, xi):
    X, Y, Z = node_coords(xi, wl.faces()) if not wl.warp else tuple(wl.nodes(xi))
    gamma = wl.gamma
    if wl.kind == "tgv":
        p0 = 1.0 / (gamma * wl.Ma ** 2)
        u = np.sin(X) * np.cos(Y) * np.cos(Z)
        v = -np.cos(X) * np.sin(Y) * np.cos(Z)
        w = np.zeros_like(X)
        p = p0 + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
        rho = p / (wl.R * 1.0)
        if wl.noise:
            rng = np.random.default_rng(wl.seed)
            xi3 = rng.uniform(-1.0, 1.0, size=(3,) + X.shape)
            u = u + wl.noise * xi3[0]
            v = v + wl.noise * xi3[1]
            w = w + wl.noise * xi3[2]
    elif wl.kind == "freestream":
        u = np.full_like(X, 0.3)
        v = np.full_like(X, -0.2)
        w = np.full_like(X, 0.1)
        rho = np.ones_like(X)
        p = np.full_like(X, 1.0 / (gamma * wl.Ma ** 2))
    elif wl.kind == "channel":
        a = 0.05
        rng = np.random.default_rng(wl.seed)
        xi3 = rng.uniform(-1.0, 1.0, size=(3,) + X.shape)
        env = 1.0 - Y * Y
        u = 1.5 * env + a * env * xi3[0]
        v = a * env * xi3[1]
        w = a * env * xi3[2]
        rho = np.ones_like(X)
        p = rho * wl.R * 1.0
    else:
        raise ValueError(f"unknown workload kind {wl.kind!r}")
    return rho, u, v, w, p


def make_state(wl: Workload, xi):
    """Conservative initial state (5, nz, ny, nx, NP, NP, NP) and its time step."""
    rho, u, v, w, p = _prim_state(wl, xi)
    E = p / (wl.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    U = np.stack([rho, rho * u, rho * v, rho * w, E])
    dt = cfl_dt(wl, rho, (u, v, w), p)
    return U, dt


def cfl_dt(wl: Workload, rho, vel, p) -> float:
    hs = _widths(wl.faces())
    c = np.sqrt(wl.gamma * p / rho)
    k = 2 * wl.N + 1
    visc = max(4.0 / 3.0, wl.gamma / wl.Pr) * wl.mu / rho
    denom = 0.0
    for d in range(3):
        denom = denom + k * (np.abs(vel[d]) + c) / hs[d] + k * k * visc / hs[d] ** 2
    return float(wl.cfl * np.min(1.0 / denom))


def fd_direction(U0: np.ndarray, r: int) -> np.ndarray:
    """Seeded direction d = xi * rms_v(U0) per conserved variable, xi ~ N(0, 1), seed 1000 + r."""
    rng = np.random.default_rng(1000 + r)
    xi = rng.standard_normal(U0.shape)
    rms = np.sqrt(np.mean(U0.reshape(U0.shape[0], -1) ** 2, axis=1))
    return xi * rms.reshape((-1,) + (1,) * (U0.ndim - 1))
