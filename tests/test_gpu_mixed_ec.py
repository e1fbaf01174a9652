"""Mixed precision with the entropy-conserving / Roe pair (GPU) against FP64.

The volume flux differencing runs in FP32 relative to each element's
reference state: the log means of rho and beta in FP32 (series below
f^2 = 1e-2), p^ - p_ref and 1/beta_ln - 1/beta_ref formed without FP32
differences of O(p_ref) terms, and the reference parts added back in FP64;
primitive recovery, the Roe surface flux, the accumulation of Ut and the RK
update stay FP64.  Bound as for the Kennedy-Gruber mixed path: relative L2
error per conserved variable <= 1e-4 for Ut against the FP64 oracle, and for
the change of the state over an RK run against the FP64 path.
"""

import numpy as np
import pytest
import torch

from oracle.dgsem import rhs, rk_step
from oracle.mesh import Mesh
from oracle.physics import Gas
from paper_2606_18927_amd import dgsem, workloads

from _cases import random_faces, random_state
from _gpu import custom, need_gpu, oracle_gas, oracle_mesh, rel_l2, say, state, to_dev

pytestmark = pytest.mark.gpu
BOUND = 1e-4
EC = dict(flux="ec_roe")

CASES = [
    ("tgv_n3_4x4x4", lambda: custom("tgv", 3, (4, 4, 4), flux="ec_roe")),
    ("tgv_n7_4x4x4_noise", lambda: custom("tgv", 7, (4, 4, 4), noise=0.01, seed=11, flux="ec_roe")),
    ("channel_n5_3x4x2", lambda: custom("channel", 5, (3, 4, 2), seed=workloads.CHANNEL_SEED, flux="ec_roe")),
]


def _table(name, got, ref):
    g = np.asarray(got).reshape(5, -1)
    r = np.asarray(ref).reshape(5, -1)
    rel = rel_l2(g, r)
    say(f"{name}: rel L2 {np.array2string(rel, precision=2)}  max abs "
        f"{np.array2string(np.abs(g - r).max(1), precision=2)}")
    return rel


@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_mixed_ec_rhs_against_fp64_oracle(case):
    need_gpu()
    wl = dict(CASES)[case]()
    U, _ = state(wl)
    ref = rhs(torch.as_tensor(U), oracle_mesh(wl), oracle_gas(wl), **EC).numpy()
    S = dgsem.solver_for(wl, precision="mixed")
    Ut = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    assert np.all(_table(f"{case} mixed ec_roe Ut", Ut, ref) < BOUND)


@pytest.mark.parametrize("N,n,bc", [
    (5, (2, 3, 2), ("periodic",) * 3),
    (3, (3, 2, 2), ("periodic", "wall", "periodic")),
])
def test_mixed_ec_large_jumps(N, n, bc):
    """Random nodal states with 20 % density and pressure spreads: most log
    means of the pairs take the atanh form in FP32."""
    need_gpu()
    rng = np.random.default_rng(90 + N)
    lo = [-1.0 if b != "periodic" else 0.0 for b in bc]
    mesh = Mesh(N, tuple(random_faces(n[d], lo[d], lo[d] + 2.0, rng) for d in range(3)), bc=bc, T_wall=1.1)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=0.01, Pr=0.72)
    U = random_state(mesh, g.gamma, g.R, rng, vel_amp=1.0, p_mean=g.R, p_amp=0.2, rho_amp=0.2).numpy()
    ref = rhs(torch.as_tensor(U), mesh, g, **EC).numpy()
    spec = dgsem.MeshSpec(mesh.N, mesh.faces, mesh.bc, mesh.T_wall)
    S = dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, precision="mixed", **EC)
    Ut = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    assert np.all(_table(f"random N={N} {bc} mixed ec_roe Ut", Ut, ref) < BOUND)


def test_mixed_ec_rk_steps_against_fp64_oracle():
    need_gpu()
    wl = CASES[0][1]()
    U, dt = state(wl)
    nsteps = 10
    Uref = rk_step(torch.as_tensor(U), oracle_mesh(wl), oracle_gas(wl), dt, nsteps, **EC).numpy()
    S = dgsem.solver_for(wl, precision="mixed")
    S.set_state(to_dev(U))
    S.rk_step(dt, nsteps)
    S.sync()
    Un = S.get_state().cpu().numpy()
    U0 = U.reshape(5, -1)
    rel = _table("tgv_n3 mixed ec_roe 10 steps, increment", Un.reshape(5, -1) - U0, Uref.reshape(5, -1) - U0)
    assert np.all(rel < BOUND)


def test_mixed_ec_full_size_against_fp64():
    """N = 7, 32^3 Taylor-Green + 1 % noise: the right-hand side and 20 RK
    steps of the mixed path against the FP64 GPU path (itself matched to the
    oracle on sampled elements)."""
    need_gpu()
    wl = workloads.WORKLOADS["tgv_n7_32x32x32_ec"]
    U, dt = state(wl)
    Ud = to_dev(U)
    Ut, Un = {}, {}
    for prec in ("fp64", "mixed"):
        S = dgsem.solver_for(wl, precision=prec)
        Ut[prec] = S.eval_rhs(Ud).cpu().numpy().reshape(5, -1)
        S.set_state(Ud)
        S.rk_step(dt, 20)
        S.sync()
        Un[prec] = S.get_state().cpu().numpy().reshape(5, -1)
        del S
        torch.cuda.empty_cache()
    U0 = U.reshape(5, -1)
    assert np.all(_table("tgv_n7_32^3 ec_roe Ut mixed vs fp64", Ut["mixed"], Ut["fp64"]) < BOUND)
    rel = _table("tgv_n7_32^3 ec_roe 20 steps mixed vs fp64, increment", Un["mixed"] - U0, Un["fp64"] - U0)
    assert np.all(rel < BOUND)
