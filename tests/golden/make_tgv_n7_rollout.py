"""Write the oracle's 100-step rollout of the N = 7, 32^3-element Taylor-Green
workload (tests/golden/tgv_n7_32x32x32_100steps.npz).

Calls only ``oracle/`` and the seeded inputs of
``paper_2606_18927_amd.workloads`` (no HIP code).  The paper validates its GPU
port by the deviation between CPU and GPU results of the same run, which stays
at floating-point rounding (Sec. 3.3); this file lets the GPU tests do the same
for the whole operator over the full 100-step run.

The run: the seeded state of the workload (1 % velocity noise, PCG64 seed
20260001, node positions from the oracle's LGL nodes), its CFL-0.5 time step,
100 steps of the five-stage low-storage RK scheme with the oracle's right-hand
side.  Each right-hand side is evaluated in z-slabs of SLAB elements with one
halo element on each side (periodic wrap) and only the slab's own elements
kept.  That is exact: an element's right-hand side depends on its face
neighbours' states and on their lifted gradients at the shared face, and a
neighbour's gradient at the face nodes it shares with the slab takes lifting
corrections only from that face and from faces normal to x and y, whose
elements lie in the same z-layer; the halo's own wrong z-neighbour (the slab
wraps periodically) touches only the halo's far face nodes.

Stored: the state of 64 fixed elements after step 1 and after step 100
(float64, (64, 5, 8, 8, 8), element e = ex + 32 (ey + 32 ez)); the kinetic
energy (LGL quadrature, the oracle's objective) and the quadrature integrals of
the five conserved variables after step 100; the per-variable L2 norm over all
nodes of U_100 - U_0.

Takes a few CPU hours.  A resume file of the state every 10 steps is kept in
--scratch (default: the system temporary directory), so an interrupted run
continues where it stopped.
"""

from __future__ import annotations

import argparse
import os
import sys
import tempfile
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.basis import lgl  # noqa: E402
from oracle.dgsem import RK_A, RK_B, kinetic_energy, rhs  # noqa: E402
from oracle.mesh import Mesh  # noqa: E402
from oracle.physics import Gas  # noqa: E402
from paper_2606_18927_amd import workloads  # noqa: E402

WORKLOAD = "tgv_n7_32x32x32"
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv_n7_32x32x32_100steps.npz")
SAMPLE_SEED = 20260101
N_SAMPLES = 64
SLAB = 16


def sample_elements(nE: int) -> np.ndarray:
    """64 fixed element indices: the four of the single-step patch tests, the
    eight corners of the box and 52 drawn without replacement (seed 20260101)."""
    fixed = [0 + 32 * (0 + 32 * 0), 31 + 32 * (17 + 32 * 5), 13 + 32 * (31 + 32 * 30),
             7 + 32 * (8 + 32 * 16)]
    fixed += [x + 32 * (y + 32 * z) for z in (0, 31) for y in (0, 31) for x in (0, 31)]
    fixed = list(dict.fromkeys(fixed))
    rng = np.random.default_rng(SAMPLE_SEED)
    rest = [int(e) for e in rng.permutation(nE) if int(e) not in fixed]
    return np.array(fixed + rest[:N_SAMPLES - len(fixed)], dtype=np.int64)


class _SlabMesh(Mesh):
    """A z-slab of a periodic mesh: its elements keep the widths (hence the
    scales s_d = 2 / width_d) of the elements they stand for; np.diff of
    shifted face coordinates could differ from them in the last bit."""

    def __init__(self, mesh: Mesh, idx):
        wz = np.diff(mesh.faces[2])[idx]
        super().__init__(mesh.N, (mesh.faces[0], mesh.faces[1],
                                  np.concatenate(([0.0], np.cumsum(wz)))), bc=mesh.bc,
                         T_wall=mesh.T_wall)
        self._wz = torch.tensor(wz, dtype=torch.float64)

    def widths(self, d: int) -> torch.Tensor:
        return self._wz.clone() if d == 2 else super().widths(d)


def slab_rhs(U: torch.Tensor, mesh: Mesh, gas: Gas, slab: int = SLAB) -> torch.Tensor:
    """L(U) of a mesh periodic in z, evaluated slab by slab (module docstring)."""
    nz = U.shape[1]
    out = torch.empty_like(U)
    for z0 in range(0, nz, slab):
        b = min(slab, nz - z0)
        idx = [(z0 + o) % nz for o in range(-1, b + 1)]
        r = rhs(U[:, idx].contiguous(), _SlabMesh(mesh, idx), gas)
        out[:, z0:z0 + b] = r[:, 1:b + 1]
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--scratch", default=tempfile.gettempdir())
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--steps", type=int, default=100)
    a = ap.parse_args()
    if a.threads:
        torch.set_num_threads(a.threads)
    wl = workloads.WORKLOADS[WORKLOAD]
    N = wl.N
    xi, _ = lgl(N)
    U0, dt = workloads.make_state(wl, xi.numpy())
    mesh = Mesh(N, wl.faces())
    gas = Gas(wl.gamma, wl.R, wl.mu, wl.Pr)
    nz, ny, nx = wl.nelem[2], wl.nelem[1], wl.nelem[0]
    samples = sample_elements(nx * ny * nz)
    sz, sy, sx = samples // (nx * ny), (samples // nx) % ny, samples % nx

    resume = os.path.join(a.scratch, f"{WORKLOAD}_oracle_resume.npz")
    U = torch.as_tensor(U0.copy())
    step0 = 0
    after1 = None
    if os.path.exists(resume):
        z = np.load(resume)
        U = torch.as_tensor(z["U"])
        step0 = int(z["step"])
        after1 = z["after1"]
        print(f"resumed at step {step0}", flush=True)
    t_start = time.time()
    for n in range(step0, a.steps):
        G = torch.zeros_like(U)
        for s in range(5):
            G = RK_A[s] * G + dt * slab_rhs(U, mesh, gas)
            U = U + RK_B[s] * G
        if n == 0:
            after1 = U.numpy()[:, sz, sy, sx].transpose(1, 0, 2, 3, 4).copy()
        el = time.time() - t_start
        print(f"step {n + 1}/{a.steps} done, {el:.0f} s since start", flush=True)
        if (n + 1) % 10 == 0 and n + 1 < a.steps:
            np.savez(resume + ".tmp.npz", U=U.numpy(), step=n + 1, after1=after1)
            os.replace(resume + ".tmp.npz", resume)

    Un = U.numpy()
    wq = mesh.quadrature_weights().numpy()
    integrals = np.array([(wq * Un[v]).sum() for v in range(5)])
    inc_norm = np.linalg.norm((Un - U0).reshape(5, -1), axis=1)
    np.savez(OUT, samples=samples, after1=after1,
             after100=Un[:, sz, sy, sx].transpose(1, 0, 2, 3, 4).copy(),
             ke=np.array(float(kinetic_energy(U, mesh))), integrals=integrals,
             increment_l2=inc_norm, dt=np.array(dt), steps=np.array(a.steps))
    print("wrote", OUT, flush=True)
    if os.path.exists(resume):
        os.remove(resume)


if __name__ == "__main__":
    main()
