"""Mixed-precision forward (GPU): per-variable errors against FP64.

Stated bound (FP32 rounding, 6e-8, times the conditioning of the low-Mach
operator, about 1e3 once the reference subtraction has removed p ~ 71 and
e ~ 179 from the FP32 sums): relative L2 error per conserved variable <= 1e-4 for
Ut against the FP64 oracle, and <= 1e-4 for the change of the state over an RK
run against the FP64 reference, with the reference-state subtraction on.
Without the subtraction the errors must be larger (the subtraction is what
keeps p ~ 1/(gamma Ma^2) from swamping FP32).

The errors measured here are printed per variable (max abs and rel L2) and,
for the full N = 7, 32^3 Taylor-Green run of 100 steps, written as
mixed_errors.json to the folder named by DGSEM_RESULTS_DIR when that is set.
"""

import json
import os

import numpy as np
import pytest
import torch

from oracle.dgsem import rhs, rk_step
from paper_2606_18927_amd import dgsem, workloads

from _gpu import custom, need_gpu, oracle_gas, oracle_mesh, rel_l2, say, state, to_dev

pytestmark = pytest.mark.gpu
BOUND = 1e-4

CASES = [
    ("tgv_n3_4x4x4", lambda: workloads.WORKLOADS["tgv_n3_4x4x4"]),
    ("tgv_n7_4x4x4_noise", lambda: custom("tgv", 7, (4, 4, 4), noise=0.01, seed=11)),
    ("channel_n5_3x4x2", lambda: custom("channel", 5, (3, 4, 2), seed=workloads.CHANNEL_SEED)),
]


def _table(name, got, ref):
    g = np.asarray(got).reshape(5, -1)
    r = np.asarray(ref).reshape(5, -1)
    rel = rel_l2(g, r)
    mx = np.abs(g - r).max(1)
    say(f"{name}: rel L2 {np.array2string(rel, precision=2)}  max abs {np.array2string(mx, precision=2)}")
    return rel, mx


@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_mixed_rhs_against_fp64_oracle(case):
    need_gpu()
    wl = dict(CASES)[case]()
    U, _ = state(wl)
    ref = rhs(torch.as_tensor(U), oracle_mesh(wl), oracle_gas(wl)).numpy()
    errs = {}
    for prec in ("mixed", "mixed_noref"):
        S = dgsem.solver_for(wl, precision=prec)
        Ut = S.eval_rhs(to_dev(U)).cpu().numpy()
        S.sync()
        errs[prec], _ = _table(f"{case} {prec} Ut", Ut, ref)
    assert np.all(errs["mixed"] < BOUND)
    # the reference-state subtraction is what keeps FP32 usable at Ma = 0.1
    assert errs["mixed_noref"].max() > 3 * errs["mixed"].max()


def test_mixed_rk_steps_against_fp64_oracle():
    need_gpu()
    wl = workloads.WORKLOADS["tgv_n3_4x4x4"]
    U, dt = state(wl)
    Uref = rk_step(torch.as_tensor(U), oracle_mesh(wl), oracle_gas(wl), dt, wl.nsteps).numpy()
    S = dgsem.solver_for(wl, precision="mixed")
    S.set_state(to_dev(U))
    S.rk_step(dt, wl.nsteps)
    S.sync()
    Un = S.get_state().cpu().numpy()
    U0 = U.reshape(5, -1)
    rel, _ = _table("tgv_n3 mixed 10 steps increment", Un.reshape(5, -1) - U0, Uref.reshape(5, -1) - U0)
    assert np.all(rel < BOUND)


def test_mixed_full_size_run_against_fp64():
    """N=7, 32^3 Taylor-Green + 1 % noise, 100 steps: mixed vs the FP64 GPU
    operator (itself matched to the oracle to 1e-12 on sampled elements)."""
    need_gpu()
    wl = workloads.WORKLOADS["tgv_n7_32x32x32_mixed"]
    U, dt = state(wl)
    Ud = to_dev(U)
    out = {}
    for prec in ("fp64", "mixed"):
        S = dgsem.solver_for(wl, precision=prec)
        S.set_state(Ud)
        S.rk_step(dt, wl.nsteps)
        S.sync()
        out[prec] = S.get_state().cpu().numpy().reshape(5, -1)
        del S
        torch.cuda.empty_cache()
    U0 = U.reshape(5, -1)
    rel_inc, mx = _table("tgv_n7_32^3 mixed vs fp64, 100 steps, increment", out["mixed"] - U0, out["fp64"] - U0)
    rel_state, _ = _table("tgv_n7_32^3 mixed vs fp64, 100 steps, state", out["mixed"], out["fp64"])
    names = ["rho", "rho_u", "rho_v", "rho_w", "E"]
    out_dir = os.environ.get("DGSEM_RESULTS_DIR")
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "mixed_errors.json"), "w") as f:
            json.dump({"workload": wl.name, "steps": wl.nsteps,
                       "increment_rel_l2": dict(zip(names, rel_inc.tolist())),
                       "max_abs": dict(zip(names, mx.tolist())),
                       "state_rel_l2": dict(zip(names, rel_state.tolist()))}, f, indent=1)
    assert np.all(rel_inc < BOUND)
