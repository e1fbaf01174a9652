"""Mixed precision with the paper's LES physics (GPU) against FP64: Sutherland's
law and the algebraic wall model with slip adiabatic walls.

The FP32 parts are those of the mixed path (lifting, volume fluxes, line
sums); mu(T) is evaluated from the node's FP64 temperature in the face-flux
kernel and from T_ref + (T - T_ref) in the right-hand side; the wall stress
(Newton solve of Spalding's law) and the surface fluxes stay FP64.  Bound as
for the other mixed paths: relative L2 error per conserved variable <= 1e-4
for Ut against the FP64 oracle and for the change of the state over RK steps
against the FP64 path.
"""

import numpy as np
import pytest
import torch

from oracle.dgsem import rhs
from oracle.mesh import Mesh, tanh_faces, uniform_faces
from oracle.physics import Gas
from paper_2606_18927_amd import dgsem, workloads

from _gpu import need_gpu, oracle_gas, oracle_mesh, rel_l2, say, state, to_dev

pytestmark = pytest.mark.gpu
BOUND = 1e-4
T_REF, S_AIR = 1.0, 110.4 / 288.15


def _table(name, got, ref):
    g = np.asarray(got).reshape(5, -1)
    r = np.asarray(ref).reshape(5, -1)
    rel = rel_l2(g, r)
    say(f"{name}: rel L2 {np.array2string(rel, precision=2)}  max abs "
        f"{np.array2string(np.abs(g - r).max(1), precision=2)}")
    return rel


def _channel_state(mesh, g, rng):
    X, Y, Z = [c.numpy() for c in mesh.coords()]
    rho = 1.0 + 0.05 * np.sin(X) * np.cos(2 * Z)
    u = 1.2 * (1 - 0.5 * Y * Y) * (1 + 0.05 * rng.uniform(-1, 1, X.shape))
    v = 0.05 * (1 - Y * Y) * rng.uniform(-1, 1, X.shape)
    w = 0.05 * (1 - Y * Y) * rng.uniform(-1, 1, X.shape)
    p = g.R * (1.0 + 0.05 * np.cos(X + Y))
    E = p / (g.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


@pytest.mark.parametrize("bc,flux", [
    (("periodic", "wallmodel", "periodic"), "kg_llf"),
    (("periodic", "wall", "periodic"), "kg_llf"),
    (("periodic", "wallmodel", "periodic"), "ec_roe"),
    (("periodic",) * 3, "kg_llf"),
])
def test_mixed_sutherland_wall_model_rhs_against_fp64_oracle(bc, flux):
    need_gpu()
    rng = np.random.default_rng(17)
    mesh = Mesh(5, (uniform_faces(3, 0, 2 * np.pi), tanh_faces(4, 2.0), uniform_faces(2, 0, np.pi)),
                bc=bc, T_wall=1.0, wm_node=2)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=2e-3, Pr=0.72, sutherland=True, T_ref=T_REF, S=S_AIR)
    U = _channel_state(mesh, g, rng)
    ref = rhs(torch.as_tensor(U), mesh, g, flux=flux).numpy()
    spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall, mesh.wm_node)
    S = dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, sutherland=(T_REF, S_AIR), precision="mixed", flux=flux)
    Ut = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    assert np.all(_table(f"mixed {bc} {flux} Sutherland Ut", Ut, ref) < BOUND)


def test_mixed_wall_model_channel_full_size_against_fp64():
    """The wall-modelled channel (N = 5, 48 x 32 x 48, slip walls, Sutherland):
    Ut and 5 RK steps of the mixed path against the FP64 GPU path (itself
    matched to the oracle)."""
    need_gpu()
    wl = workloads.WORKLOADS["channel_n5_48x32x48_wm"]
    U, _ = state(wl)
    dt = 2e-5
    Ud = to_dev(U)
    Ut, Un = {}, {}
    for prec in ("fp64", "mixed"):
        S = dgsem.solver_for(wl, precision=prec)
        Ut[prec] = S.eval_rhs(Ud).cpu().numpy().reshape(5, -1)
        S.set_state(Ud)
        S.rk_step(dt, 5)
        S.sync()
        Un[prec] = S.get_state().cpu().numpy().reshape(5, -1)
        del S
        torch.cuda.empty_cache()
    U0 = U.reshape(5, -1)
    assert np.all(_table("channel wm 48x32x48 Ut mixed vs fp64", Ut["mixed"], Ut["fp64"]) < BOUND)
    rel = _table("channel wm 48x32x48 5 steps mixed vs fp64, increment", Un["mixed"] - U0, Un["fp64"] - U0)
    assert np.all(rel < BOUND)
