"""The full N = 7, 32^3-element Taylor-Green run (100 RK steps) on the GPU
against the stored FP64 oracle rollout of the same run (GPU).

The paper validates its GPU port by the deviation between CPU and GPU results
of the same simulation, which stays at floating-point rounding (Sec. 3.3).
``tests/golden/tgv_n7_32x32x32_100steps.npz`` holds the oracle's state of 64
fixed elements after step 1 and after step 100, the kinetic energy and the
per-variable L2 norm of U_100 - U_0 over all nodes; it was written by
``tests/golden/make_tgv_n7_rollout.py``, which calls only ``oracle/``.  The
initial state is the seeded workload at the oracle's LGL node positions, as in
that script.

Bounds (per conserved variable, over the 64 sampled elements):
* FP64, the state: relative L2 <= 1e-12.
* FP64, the increment U_n - U_0: relative L2 <= 1e-10.  A single
  right-hand side agrees with the oracle to 1e-12 relative, at the limit the
  low-Mach conditioning leaves (momentum right-hand sides are small
  differences of O(p0) terms); the increment is dt times a sum of 5 n such
  right-hand sides, so its error can reach 5 n x 1e-12 relative if the
  rounding differences do not cancel, 1e-10 for n = 20; the run is smooth and
  short (t = 0.021, no amplification), and the errors of different stages
  are unrelated, so they grow like a random walk, well inside 1e-10.
* FP64: the kinetic energy to 1e-13 relative; the global increment norms to
  1e-10 relative.
* Mixed precision (FP32 lifting, volume fluxes and line sums with the
  reference-state subtraction), the increment: relative L2 <= 1e-4, the
  bound stated for the mixed method; the per-variable errors are printed and,
  when DGSEM_RESULTS_DIR names a folder, written there
  (rollout_golden_errors.json).
"""

import json
import os

import numpy as np
import pytest
import torch

from oracle.basis import lgl
from paper_2606_18927_amd import dgsem, workloads

from _gpu import need_gpu, say, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tgv_n7_32x32x32_100steps.npz")
NAMES = ["rho", "rho_u", "rho_v", "rho_w", "E"]


def _rel(got, ref):
    g = np.asarray(got).reshape(5, -1)
    r = np.asarray(ref).reshape(5, -1)
    return np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1), np.abs(g - r).max(axis=1)


@pytest.fixture(scope="module")
def golden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(GOLDEN):
        pytest.skip("stored oracle rollout not generated")
    z = np.load(GOLDEN)
    wl = workloads.WORKLOADS["tgv_n7_32x32x32"]
    xi, _ = lgl(wl.N)
    U, dt = workloads.make_state(wl, xi.numpy())
    assert dt == float(z["dt"])
    s = z["samples"]
    nx, ny = wl.nelem[0], wl.nelem[1]
    idx = (s // (nx * ny), (s // nx) % ny, s % nx)
    return wl, U, dt, z, idx


def _run(wl, U, dt, precision, idx):
    """States of the sampled elements (64, 5, 8, 8, 8) after 1 and 100 steps,
    the kinetic energy and the global increment norms after 100 steps."""
    S = dgsem.solver_for(wl, precision=precision)
    Ud = to_dev(U)
    S.set_state(Ud)
    S.rk_step(dt, 1)
    S.sync()
    a1 = S.get_state().cpu().numpy().reshape(U.shape)[:, idx[0], idx[1], idx[2]].transpose(1, 0, 2, 3, 4)
    S.rk_step(dt, wl.nsteps - 1)
    S.sync()
    Un = S.get_state()
    ke = S.kinetic_energy(Un).item()
    inc = (Un.view(5, -1) - Ud.view(5, -1)).norm(dim=1).cpu().numpy()
    a100 = Un.cpu().numpy().reshape(U.shape)[:, idx[0], idx[1], idx[2]].transpose(1, 0, 2, 3, 4)
    del S
    torch.cuda.empty_cache()
    return a1, a100, ke, inc


def _compare(tag, got, ref, U0s):
    """(state rel L2, increment rel L2, increment max abs) per variable."""
    g = got.transpose(1, 0, 2, 3, 4)
    r = ref.transpose(1, 0, 2, 3, 4)
    u0 = U0s.transpose(1, 0, 2, 3, 4)
    st, _ = _rel(g, r)
    inc, mx = _rel(g - u0, r - u0)
    say(tag, "state rel L2", st, "increment rel L2", inc, "increment max abs", mx)
    return st, inc, mx


def test_full_run_fp64_against_oracle(golden):
    wl, U, dt, z, idx = golden
    say("N=7 32^3 Taylor-Green, 100 steps, FP64 vs the stored oracle rollout")
    a1, a100, ke, inc = _run(wl, U, dt, "fp64", idx)
    U0s = U[:, idx[0], idx[1], idx[2]].transpose(1, 0, 2, 3, 4)
    st1, inc1, _ = _compare("step 1:", a1, z["after1"], U0s)
    st, incr, _ = _compare("step 100:", a100, z["after100"], U0s)
    ke_err = abs(ke - float(z["ke"])) / abs(float(z["ke"]))
    gl = np.abs(inc - z["increment_l2"]) / z["increment_l2"]
    say("kinetic energy rel", ke_err, "global increment norms rel", gl)
    assert np.all(st1 < 1e-12) and np.all(inc1 < 1e-10)
    assert np.all(st < 1e-12) and np.all(incr < 1e-10)
    assert ke_err < 1e-13
    assert np.all(gl < 1e-10)


def test_full_run_mixed_against_oracle(golden):
    wl, U, dt, z, idx = golden
    say("N=7 32^3 Taylor-Green, 100 steps, mixed precision vs the stored FP64 oracle rollout")
    a1, a100, ke, inc = _run(wl, U, dt, "mixed", idx)
    U0s = U[:, idx[0], idx[1], idx[2]].transpose(1, 0, 2, 3, 4)
    st, incr, mx = _compare("step 100:", a100, z["after100"], U0s)
    ke_err = abs(ke - float(z["ke"])) / abs(float(z["ke"]))
    say("kinetic energy rel", ke_err)
    out_dir = os.environ.get("DGSEM_RESULTS_DIR")
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "rollout_golden_errors.json"), "w") as f:
            json.dump({"workload": wl.name, "steps": wl.nsteps, "precision": "mixed",
                       "reference": "stored FP64 oracle rollout, 64 sampled elements",
                       "state_rel_l2": dict(zip(NAMES, st.tolist())),
                       "increment_rel_l2": dict(zip(NAMES, incr.tolist())),
                       "increment_max_abs": dict(zip(NAMES, mx.tolist())),
                       "kinetic_energy_rel": ke_err}, f, indent=1)
    assert np.all(incr < 1e-4)
