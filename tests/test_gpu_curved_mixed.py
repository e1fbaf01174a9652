"""Curved hexahedra in mixed precision (GPU) against FP64.

The Kennedy-Gruber pair on curved elements with the LDS fields, gradients,
sweep metrics and line sums in FP32 (p, e and T relative to each element's
first node) and the primitive recovery, lifting corrections, surface fluxes,
1/J scaling and RK update in FP64 (Navier-Stokes, Euler and the central
flux; periodic boxes and wavy walls).  The entropy-conserving / Roe pair the
same way, its FP32 sweep relative to the element's (p, beta) (Navier-Stokes,
Euler, central, Sutherland; warped boxes, wavy walls, the Ma = 0.1
Taylor-Green state).  Bound as for the other mixed paths:
relative L2 error per conserved variable <= 1e-4 for Ut against the FP64
oracle and for the change of the state over RK steps against the FP64 path.
"""

import numpy as np
import pytest
import torch

from oracle import curvilinear as cv
from oracle.physics import Gas
from paper_2606_18927_amd import dgsem, workloads

from _cases import random_state
from _gpu import need_gpu, oracle_gas, say, state, to_dev

pytestmark = pytest.mark.gpu
BOUND = 1e-4
GAS = Gas(gamma=1.4, R=1.0, mu=0.02, Pr=0.72)


def _solver(N, X, g, bc=("periodic",) * 3, T_wall=1.0, **kw):
    spec = dgsem.MeshSpec(N, None, bc, T_wall, nodes=X)
    suth = (g.T_ref, g.S) if g.sutherland else None
    return dgsem.Solver(spec, g.gamma, g.R, g.mu, g.Pr, sutherland=suth, precision="mixed", **kw)


def _table(name, got, ref, momentum_norm=False):
    g = np.asarray(got).reshape(5, -1)
    r = np.asarray(ref).reshape(5, -1)
    num = np.linalg.norm(g - r, axis=1)
    den = np.linalg.norm(r, axis=1)
    if momentum_norm:  # rho w of the Taylor-Green state is small: the whole momentum's norm
        den[1:4] = np.linalg.norm(r[1:4])
    rel = num / den
    say(f"{name}: rel L2 {np.array2string(rel, precision=2)}")
    return rel


@pytest.mark.parametrize("N,n,amp,suth,viscous,central", [
    (3, (2, 3, 2), 0.08, False, True, False),
    (5, (2, 2, 3), 0.05, False, True, False),
    (7, (2, 2, 2), 0.05, False, True, False),
    (5, (2, 2, 2), 0.08, True, True, False),
    (3, (3, 2, 2), 0.08, False, False, False),
    (5, (2, 2, 2), 0.08, False, True, True),
])
def test_curved_mixed_rhs_against_fp64_oracle(N, n, amp, suth, viscous, central):
    need_gpu()
    say("curved mixed rhs", N, n, amp, suth, viscous, central)
    X = workloads.warped_nodes(dgsem.lgl(N)[0], n, amp=amp)
    mesh = cv.CurvMesh(N, torch.as_tensor(X))
    g = Gas(gamma=1.4, R=1.0, mu=0.02, Pr=0.72, sutherland=True, T_ref=1.0, S=0.4) if suth else GAS
    U = random_state(mesh, g.gamma, g.R, np.random.default_rng(40 + N)).numpy()
    S = _solver(N, X, g, viscous=viscous, central_only=central)
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = cv.rhs(torch.as_tensor(U), mesh, g, viscous=viscous, central_only=central).numpy()
    assert np.all(_table(f"curved mixed N={N}", got, ref) < BOUND)


def test_curved_mixed_wavy_channel_against_fp64_oracle():
    need_gpu()
    N, n = 5, (2, 3, 2)
    X = workloads.wavy_channel_nodes(dgsem.lgl(N)[0], n, amp=0.06)
    bc = ("periodic", "wall", "periodic")
    mesh = cv.CurvMesh(N, torch.as_tensor(X), bc=bc, T_wall=1.3)
    U = random_state(mesh, GAS.gamma, GAS.R, np.random.default_rng(61)).numpy()
    S = _solver(N, X, GAS, bc=bc, T_wall=1.3)
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = cv.rhs(torch.as_tensor(U), mesh, GAS).numpy()
    assert np.all(_table("curved mixed wavy channel", got, ref) < BOUND)


def test_curved_mixed_low_mach_tgv_rhs_and_steps():
    """The Ma = 0.1 Taylor-Green state on the warped N = 3 box, where the
    reference subtraction carries the accuracy: Ut against the FP64 oracle
    and ten RK steps (increment) against it."""
    need_gpu()
    wl = workloads.WORKLOADS["tgv_n3_4x4x4_curved"]
    U, dt = state(wl)
    X = wl.nodes(dgsem.lgl(wl.N)[0])
    mesh = cv.CurvMesh(wl.N, torch.as_tensor(X))
    g = oracle_gas(wl)
    S = dgsem.solver_for(wl, precision="mixed")
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = cv.rhs(torch.as_tensor(U), mesh, g).numpy()
    assert np.all(_table("curved mixed TGV N=3 Ut", got, ref, momentum_norm=True) < BOUND)
    S.set_state(to_dev(U))
    S.rk_step(dt, 10)
    S.sync()
    Un = S.get_state().cpu().numpy().reshape(U.shape)
    Uref = cv.rk_step(torch.as_tensor(U), mesh, g, dt, 10).numpy()
    rel = _table("curved mixed TGV N=3 10 steps, increment", Un - U, Uref - U, momentum_norm=True)
    assert np.all(rel < BOUND)


def test_curved_mixed_full_size_against_fp64():
    """N = 7, 32^3 warped Taylor-Green: Ut and 20 RK steps of the mixed path
    against the FP64 GPU path (itself matched to the oracle)."""
    need_gpu()
    wl = workloads.WORKLOADS["tgv_n7_32x32x32_curved"]
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
    assert np.all(_table("curved 32^3 Ut mixed vs fp64", Ut["mixed"], Ut["fp64"], True) < BOUND)
    rel = _table("curved 32^3 20 steps mixed vs fp64, increment", Un["mixed"] - U0, Un["fp64"] - U0, True)
    assert np.all(rel < BOUND)


@pytest.mark.parametrize("N,n,amp,suth,viscous,central", [
    (3, (2, 3, 2), 0.08, False, True, False),
    (5, (2, 2, 3), 0.05, False, True, False),
    (7, (2, 2, 2), 0.05, True, True, False),
    (3, (3, 2, 2), 0.08, False, False, False),
    (5, (2, 2, 2), 0.08, False, False, True),
])
def test_curved_mixed_entropy_conserving_against_fp64_oracle(N, n, amp, suth, viscous, central):
    """Random nodal states with 20 % density and pressure spreads, so most
    FP32 log means take their atanh form."""
    need_gpu()
    say("curved mixed ec_roe rhs", N, n, amp, suth, viscous, central)
    X = workloads.warped_nodes(dgsem.lgl(N)[0], n, amp=amp)
    mesh = cv.CurvMesh(N, torch.as_tensor(X))
    g = Gas(gamma=1.4, R=1.0, mu=0.02, Pr=0.72, sutherland=True, T_ref=1.0, S=0.4) if suth else GAS
    U = random_state(mesh, g.gamma, g.R, np.random.default_rng(140 + N)).numpy()
    S = _solver(N, X, g, viscous=viscous, central_only=central, flux="ec_roe")
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = cv.rhs(torch.as_tensor(U), mesh, g, viscous=viscous, central_only=central, flux="ec_roe").numpy()
    assert np.all(_table(f"curved mixed ec_roe N={N}", got, ref) < BOUND)


def test_curved_mixed_entropy_conserving_wavy_channel_and_tgv():
    """Between wavy isothermal walls (N = 5) against the FP64 oracle, and the
    Ma = 0.1 Taylor-Green state on the warped N = 3 box: Ut and ten RK steps
    (increment) against the oracle."""
    need_gpu()
    N, n = 5, (2, 3, 2)
    X = workloads.wavy_channel_nodes(dgsem.lgl(N)[0], n, amp=0.06)
    bc = ("periodic", "wall", "periodic")
    mesh = cv.CurvMesh(N, torch.as_tensor(X), bc=bc, T_wall=1.3)
    U = random_state(mesh, GAS.gamma, GAS.R, np.random.default_rng(161)).numpy()
    S = _solver(N, X, GAS, bc=bc, T_wall=1.3, flux="ec_roe")
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = cv.rhs(torch.as_tensor(U), mesh, GAS, flux="ec_roe").numpy()
    assert np.all(_table("curved mixed ec_roe wavy channel", got, ref) < BOUND)
    wl = workloads.WORKLOADS["tgv_n3_4x4x4_curved"]
    U, dt = state(wl)
    X = wl.nodes(dgsem.lgl(wl.N)[0])
    mesh = cv.CurvMesh(wl.N, torch.as_tensor(X))
    g = oracle_gas(wl)
    S = dgsem.solver_for(wl, precision="mixed", flux="ec_roe")
    got = S.eval_rhs(to_dev(U)).cpu().numpy()
    S.sync()
    ref = cv.rhs(torch.as_tensor(U), mesh, g, flux="ec_roe").numpy()
    assert np.all(_table("curved mixed ec_roe TGV N=3 Ut", got, ref, momentum_norm=True) < BOUND)
    S.set_state(to_dev(U))
    S.rk_step(dt, 10)
    S.sync()
    Un = S.get_state().cpu().numpy().reshape(U.shape)
    Uref = cv.rk_step(torch.as_tensor(U), mesh, g, dt, 10, flux="ec_roe").numpy()
    rel = _table("curved mixed ec_roe TGV N=3 10 steps, increment", Un - U, Uref - U, momentum_norm=True)
    assert np.all(rel < BOUND)


def test_curved_mixed_entropy_conserving_full_size_against_fp64():
    """N = 7, 32^3 warped Taylor-Green with the entropy-conserving / Roe pair:
    Ut and 5 RK steps of the mixed path against the FP64 GPU path."""
    need_gpu()
    wl = workloads.WORKLOADS["tgv_n7_32x32x32_curved"]
    U, dt = state(wl)
    Ud = to_dev(U)
    Ut, Un = {}, {}
    for prec in ("fp64", "mixed"):
        S = dgsem.solver_for(wl, precision=prec, flux="ec_roe")
        Ut[prec] = S.eval_rhs(Ud).cpu().numpy().reshape(5, -1)
        S.set_state(Ud)
        S.rk_step(dt, 5)
        S.sync()
        Un[prec] = S.get_state().cpu().numpy().reshape(5, -1)
        del S
        torch.cuda.empty_cache()
    U0 = U.reshape(5, -1)
    assert np.all(_table("curved ec_roe 32^3 Ut mixed vs fp64", Ut["mixed"], Ut["fp64"], True) < BOUND)
    rel = _table("curved ec_roe 32^3 5 steps mixed vs fp64, increment", Un["mixed"] - U0, Un["fp64"] - U0, True)
    assert np.all(rel < BOUND)
