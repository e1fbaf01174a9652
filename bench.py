"""Throughput of the split-form DGSEM RK step on one MI355X.

Workload: Taylor-Green vortex at N = 7 on 32^3 periodic elements (16.8 M DOF,
DOF = one LGL node), 1 % seeded velocity noise, FP64, the five-stage
low-storage RK at CFL 0.5.  One "step" is one RK step: five stages, each a
face viscous-flux kernel and a fused lifting + right-hand-side + RK-update kernel.

Prints one JSON line.  `value` is ns per DOF per RK stage (FP64), i.e. the
paper's PID (Eq. 1) with one GPU; lower is better.  Also reported:
  roofline      the fused RHS/RK kernel's algorithmic HBM bytes per launch (256
                B per DOF: read U, the 12 lifted gradient components and G,
                write G and U) over its mean launch time (HIP events on the
                launch stream) vs 8 TB/s; the step at 392 B per DOF; this
                design's own smaller traffic beside it;
  fp64_compute  algorithmic FP64 flops per DOF and stage over the step time vs
                78.6 TFLOP/s (and the rocprofv3-counted flops while valid);
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload;
  mixed         the same step in mixed precision (when requested / available);
  ec_roe        the same step with the entropy-conserving volume flux and the
                Roe surface flux (FP64);
  sutherland    the same step with Sutherland's viscosity law (FP64);
  curved        the same step on curved elements (the periodic box warped by
                5 %): per-node metric terms, contravariant fluxes; FP64 and
                mixed precision, each flux pair;
  wall_model    the N = 5, 48x32x48 channel with wall-modelled slip walls and
                Sutherland's law (FP64) beside the same channel with
                isothermal walls and constant viscosity, and the wall-stress
                kernel alone (algorithmic bytes over its event-timed launch);
  freestream_context  the paper's throughput workload (uniform free stream,
                N = 7, same mesh), FP64;
  adjoint       the N = 5, 48x32x48 channel, 500 steps, checkpoint every 25:
                mixed forward, FP64 adjoint; adjoint/forward time ratio,
                memory, gradient error against the all-FP64 gradient.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
METRIC = "ns per DOF per RK stage (FP64 vs mixed) at N=7; adjoint/forward time ratio"

# Algorithmic HBM bytes per DOF and launch (N = 7: 3 face-flux values per DOF,
# 6 faces x 4 components x 64 face nodes / 512 nodes; 8 B FP64, 4 B FP32):
#   face flux kernel: read U (5) + write the face viscous fluxes (3)
#   fused RHS + RK:   read U (5) + the neighbours' face fluxes (3) + G (5, not on
#                     the first stage, A_1 = 0) + write G (5) + U' (5)
def alg_bytes(precision: str, N: int = 7):
    r = 8 if precision == "fp64" else 4
    ff = 24.0 / (N + 1) * r
    return {"face": 40 + ff, "rk": 40 + ff + 40 + 40 + 40, "rk_first": 40 + ff + 40 + 40}


# The method's algorithmic HBM bytes per DOF and RK stage, counted for a
# lifting kernel that writes the 12 lifted gradient components and a
# right-hand-side stage kernel that reads them (8 B per FP64 value):
#   right-hand side + RK stage: read U (40) + gradients (96) + G (40),
#                               write G (40) + U (40)          = 256 B
#   whole stage: + lifting (read U 40, write gradients 96)     = 392 B
# The roofline entry prices the dominant kernel (the fused right-hand side +
# RK stage) at the 256 B it stands for, the step at 392 B; this design's own
# smaller traffic (gradients recomputed, never stored) is reported beside it.
RHS_STAGE_BYTES_PER_DOF = 256.0
STORED_GRADIENT_BYTES_PER_DOF = 392.0

# Algorithmic FP64 flops per DOF and RK stage at N = 7 (Cartesian elements,
# pairs evaluated once per symmetric pair, a division counted as one):
# Kennedy-Gruber pairs 417, lifting sweeps 192, viscous-flux sweeps 192,
# viscous flux 44, surface fluxes (0.375 face nodes per DOF) 40, primitives
# 20, RK update 20, scaling 15.
ALG_FLOPS_PER_DOF_STAGE = 940.0
# FP64 flops per DOF and stage counted with rocprofv3 (SQ_INSTS_VALU_{ADD,MUL,
# FMA,TRANS}_F64 x 64 lanes, FMA twice) on k_rhs + k_face_flux of this
# workload; valid only for the kernel sources they were counted on.
COUNTED_FLOPS = {"sources_sha256_prefix": "d24ddbf48a2f0125", "per_dof_stage": 1302.25 + 219.375}

# HBM bytes per launch of k_rhs<7,double> on this workload, from rocprofv3
# counter passes (profiles/k_rhs_k_face_flux_tgv_n7_32x32x32.md): reads
# 128 x 13,968,395.1 TCC_EA0_RDREQ_128B + 64 x 2,077.0 RDREQ_64B, writes
# WRITE_SIZE 1,310,764.8 KiB.  Valid only for the kernel sources it was
# counted on; reported as null once they change.
COUNTED_TRAFFIC = {"sources_sha256_prefix": "d24ddbf48a2f0125", "bytes_per_launch": 3130310656.0}
TRAFFIC_SOURCES = ("fwd_kernels.hip", "dg_device.hpp", "dg_internal.hpp")
# The same for k_rhs_curv<7,double,true,true,false> on the curved workload
# (profiles/k_rhs_curv_k_face_flux_curv_tgv_n7_32x32x32_curved.md): reads
# 128 x 35,124,061.3 RDREQ_128B + 64 x 1,876.9 RDREQ_64B, writes 1,310,738.8 KiB;
# and for its mixed-precision instance k_rhs_curv<7,float,true,true,false>:
# reads 128 x 27,055,205.1 RDREQ_128B + 64 x 4,193.1 RDREQ_64B, writes
# 1,310,720.3 KiB.
COUNTED_TRAFFIC_CURVED = {"sources_sha256_prefix": "f059d7093f7e0d5b", "bytes_per_launch": 5838196499.0}
COUNTED_TRAFFIC_CURVED_MIXED = {"sources_sha256_prefix": "f059d7093f7e0d5b", "bytes_per_launch": 4805512198.0}
TRAFFIC_SOURCES_CURVED = ("curv_kernels.hip", "dg_device.hpp", "dg_internal.hpp")


def counted_traffic(counted=COUNTED_TRAFFIC, sources=TRAFFIC_SOURCES):
    """A counted figure (bytes or flops) if the kernel sources still hash to
    the value it was counted on, else None."""
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2606_18927_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != counted["sources_sha256_prefix"]:
        return None
    return counted["bytes_per_launch"] if "bytes_per_launch" in counted else counted["per_dof_stage"]


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tgv_n7_32x32x32")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-ec", action="store_true", help="skip the entropy-conserving / Roe flux leg")
    ap.add_argument("--no-curved", action="store_true", help="skip the curved-element leg")
    ap.add_argument("--no-physics", action="store_true",
                    help="skip the Sutherland and wall-model legs")
    ap.add_argument("--adjoint-steps", type=int, default=500,
                    help="steps of the adjoint leg (the channel case as configured: 500, K = 25)")
    return ap.parse_args()


def time_steps(S, dt, steps, warmup):
    import torch
    S.rk_step(dt, warmup)
    S.sync()
    torch.cuda.synchronize()
    S.timing_begin(steps * 10 + 4)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(S.stream)
    S.rk_step(dt, steps)
    end.record(S.stream)
    torch.cuda.synchronize()
    S.sync()
    ms = start.elapsed_time(end)
    lift_ms, rk_ms, n_lift, n_rk = S.timing_end()
    return ms, lift_ms, rk_ms, n_lift, n_rk


def repeat_steps(S, dt, steps, reps=5):
    """The same `steps` RK steps timed `reps` more times back to back (HIP
    events on the context's stream): ms per run, for min / median."""
    import torch
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(S.stream)
        S.rk_step(dt, steps)
        b.record(S.stream)
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    S.sync()
    return out


def _leg(wl_name, r):
    return {"workload": wl_name, "ns_per_dof_stage": r["ns_per_dof_stage"], "ms_per_step": r["ms_per_step"],
            "rk_kernel_ms": r["rk_kernel_ms"], "face_kernel_ms": r["face_kernel_ms"],
            "step_alg_gbs": r["step_alg_gbs"], "step_frac": r["step_alg_gbs"] / HBM_PEAK_GBS}


def curved_alg_bytes(N: int = 7, mixed: bool = False):
    """Algorithmic bytes per DOF and stage of the curved-element kernels:
    k_rhs_curv reads U 40, the neighbours' face fluxes 24 (6 (N+1)^2 faces x 4
    values per element; FP32 in mixed precision), G 40 (not on stage 1) and the
    metric terms 80 (J a^i_n and 1/J), and writes G and U (80);
    k_face_flux_curv reads U 40 and the metric terms of the face nodes only,
    and writes the face fluxes."""
    NP = N + 1
    ff = 24.0 / NP * (4 if mixed else 8)
    face_nodes = 2 * NP * NP + (N - 1) * 4 * N
    return {"face": 40 + 80.0 * face_nodes / NP ** 3 + ff, "rk": 40 + ff + 40 + 80 + 80,
            "rk_first": 40 + ff + 80 + 80}


def run_curved(steps, warmup, flux=None, precision="fp64"):
    """The Taylor-Green step on the warped (curved) N = 7, 32^3 mesh (the
    workload's Kennedy-Gruber / Lax-Friedrichs pair unless `flux`)."""
    import torch

    from paper_2606_18927_amd import dgsem, workloads
    wl = workloads.WORKLOADS["tgv_n7_32x32x32_curved"]
    xi, _ = dgsem.lgl(wl.N)
    U, dt = workloads.make_state(wl, xi)
    S = dgsem.solver_for(wl, flux=flux, precision=precision)
    S.set_state(torch.as_tensor(U.reshape(-1)).cuda())
    del U
    ms, lift_ms, rk_ms, n_lift, n_rk = time_steps(S, dt, steps, warmup)
    dof, stages = S.n_dof, steps * 5
    b = curved_alg_bytes(wl.N, precision == "mixed")
    rk_bytes = dof * (b["rk"] * (stages - steps) + b["rk_first"] * steps) / stages
    rk_s = rk_ms / 1e3 / n_rk
    face_s = lift_ms / 1e3 / max(n_lift, 1)
    step_bytes = dof * (b["face"] * stages + b["rk"] * (stages - steps) + b["rk_first"] * steps)
    out = {"workload": wl.name, "warp": wl.warp, "flux": flux or wl.flux, "precision": precision,
           "ns_per_dof_stage": ms * 1e6 / (dof * stages),
           "ms_per_step": ms / steps, "rk_kernel": "k_rhs_curv", "rk_kernel_ms": rk_ms / n_rk,
           "face_kernel_ms": lift_ms / max(n_lift, 1), "rk_bytes_per_launch": rk_bytes,
           "rk_kernel_gbs": rk_bytes / rk_s / 1e9, "rk_frac": rk_bytes / rk_s / 1e9 / HBM_PEAK_GBS,
           "face_kernel_gbs": dof * b["face"] / face_s / 1e9,
           "step_alg_bytes_per_dof": step_bytes / (dof * stages), "step_alg_gbs": step_bytes / (ms / 1e3) / 1e9,
           "step_frac": step_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    counted = COUNTED_TRAFFIC_CURVED if precision == "fp64" else COUNTED_TRAFFIC_CURVED_MIXED
    traffic = counted_traffic(counted, TRAFFIC_SOURCES_CURVED) if flux is None else None
    out["rk_traffic"] = traffic
    out["rk_traffic_over_algorithmic"] = None if traffic is None else traffic / rk_bytes
    del S
    torch.cuda.empty_cache()
    return out


def run_wall_model(steps, warmup):
    """The wall-modelled channel (FP64, Sutherland) beside the isothermal one,
    and the wall-stress kernel alone: per wall-face node it reads the
    interface node's state (40 B) and writes the stress vector (24 B)."""
    import torch

    from paper_2606_18927_amd import dgsem, workloads
    wl = workloads.WORKLOADS["channel_n5_48x32x48_wm"]
    wl_iso = workloads.WORKLOADS["channel_n5_48x32x48"]
    xi, _ = dgsem.lgl(wl.N)
    U, dt = workloads.make_state(wl, xi)
    out = {}
    r, Ud = run_precision(wl, U, dt, "fp64", steps, warmup)
    out["wall_model"] = _leg(wl.name, r)
    r, _ = run_precision(wl, U, dt, "mixed", steps, warmup)
    out["wall_model_mixed"] = _leg(wl.name + " (mixed)", r)
    # the paper's production combination: entropy-conserving / Roe pair,
    # Sutherland's law and the wall model
    import dataclasses
    wl_prod = dataclasses.replace(wl, flux="ec_roe")
    r, _ = run_precision(wl_prod, U, dt, "fp64", steps, warmup)
    out["production_ec_roe"] = _leg(wl.name + " (ec_roe)", r)
    r, _ = run_precision(wl_prod, U, dt, "mixed", steps, warmup)
    out["production_ec_roe_mixed"] = _leg(wl.name + " (ec_roe, mixed)", r)
    r, _ = run_precision(wl_iso, U, dt, "fp64", steps, warmup)
    out["isothermal_constant_mu"] = _leg(wl_iso.name + " (fp64)", r)
    S = dgsem.solver_for(wl, precision="fp64")
    NP = wl.N + 1
    nodes = S.wall_faces() * NP * NP
    tau = torch.empty(nodes * 3, dtype=torch.float64, device="cuda")
    for _ in range(3):
        S.wall_stress(Ud, wl.wm_node, tau)
    S.sync()
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(S.stream)
    for _ in range(reps):
        S.wall_stress(Ud, wl.wm_node, tau)
    e1.record(S.stream)
    torch.cuda.synchronize()
    S.sync()
    ms = e0.elapsed_time(e1) / reps
    alg = nodes * (40 + 24)
    out["k_wall_stress"] = {"ms_per_launch": ms, "wall_face_nodes": nodes, "alg_bytes": alg,
                            "gbs": alg / (ms / 1e3) / 1e9, "frac": alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                            "note": "launch- and latency-bound (one Newton solve per lane)"}
    out["dt"] = dt
    del S
    torch.cuda.empty_cache()
    return out


def cpu_baseline(wl):
    """The oracle (unchanged) on a periodic 16x16x16-element sample of the same
    N = 7 Taylor-Green state, four RK steps, on the host's cores."""
    import numpy as np
    import torch

    from oracle.dgsem import rk_step
    from oracle.mesh import Mesh
    from oracle.physics import Gas
    from paper_2606_18927_amd import workloads

    sub = workloads.Workload("tgv_n7_sample", "tgv", wl.N, (16, 16, 16), nsteps=4, noise=wl.noise,
                             seed=wl.seed)
    from oracle.basis import lgl
    xi, _ = lgl(sub.N)
    U, dt = workloads.make_state(sub, xi.numpy())
    mesh = Mesh(sub.N, sub.faces(), bc=sub.bc, T_wall=sub.T_wall)
    gas = Gas(sub.gamma, sub.R, sub.mu, sub.Pr)
    Ut = torch.as_tensor(U)
    t0 = time.perf_counter()
    rk_step(Ut, mesh, gas, dt, sub.nsteps)
    sec = time.perf_counter() - t0
    ns = sec * 1e9 / (mesh.n_dof * sub.nsteps * 5)
    return {"value": ns, "unit": "ns/DOF/stage", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"N=7 Taylor-Green, 16x16x16 periodic elements ({mesh.n_dof} DOF), "
                      f"{sub.nsteps} RK steps, {sec:.1f} s wall, float64 torch CPU",
            "host_cpu_count": os.cpu_count()}


def triad_gbs():
    import torch

    from paper_2606_18927_amd import dgsem
    n = 1 << 27
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.rand(n, dtype=torch.float64, device="cuda")
    for _ in range(3):
        dgsem.stream_triad(b, c, 1.5, a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        dgsem.stream_triad(b, c, 1.5, a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, b, c
    return 24.0 * n / sec / 1e9


def run_precision(wl, U, dt, precision, steps, warmup, repeats=False):
    import torch

    from paper_2606_18927_amd import dgsem
    S = dgsem.solver_for(wl, precision=precision)
    Ud = torch.as_tensor(U.reshape(-1)).cuda()
    S.set_state(Ud)
    ms, lift_ms, rk_ms, n_lift, n_rk = time_steps(S, dt, steps, warmup)
    dof = S.n_dof
    stages = steps * 5
    ns = ms * 1e6 / (dof * stages)
    reps = sorted(x * 1e6 / (dof * stages) for x in repeat_steps(S, dt, steps)) if repeats else None
    b = alg_bytes(precision, wl.N)
    rk_bytes = dof * (b["rk"] * (stages - steps) + b["rk_first"] * steps) / stages
    rk_avg_s = rk_ms / 1e3 / n_rk
    lift_avg_s = lift_ms / 1e3 / max(n_lift, 1)
    res = {
        "ns_per_dof_stage": ns, "ms_per_step": ms / steps, "dof": dof,
        "rk_kernel_ms": rk_ms / n_rk, "face_kernel_ms": lift_ms / max(n_lift, 1),
        "rk_kernel_gbs": rk_bytes / rk_avg_s / 1e9,
        "face_kernel_gbs": dof * b["face"] / lift_avg_s / 1e9,
        "step_alg_bytes_per_dof": b["face"] + (b["rk"] * (stages - steps) + b["rk_first"] * steps) / stages,
        "step_alg_gbs": dof * (b["face"] * stages + b["rk"] * (stages - steps) + b["rk_first"] * steps)
        / (ms / 1e3) / 1e9,
        "rk_bytes_per_launch": rk_bytes,
    }
    if reps:
        res["repeats_ns_per_dof_stage"] = {"n": len(reps), "min": reps[0], "median": reps[len(reps) // 2],
                                           "max": reps[-1]}
    del S
    torch.cuda.empty_cache()
    return res, Ud


def run_small_graph(steps: int, warmup: int):
    """The launch-bound small case (N = 3 Taylor-Green on 4^3 elements, 4,096
    DOF, ten launches per RK step): steps pairs of RK steps launched with
    dg_rk_step, then replayed from a HIP graph of two steps
    (dg_rk_graph_build / dg_rk_graph_launch)."""
    import torch

    from paper_2606_18927_amd import dgsem, workloads

    wl = workloads.WORKLOADS["tgv_n3_4x4x4"]
    xi, _ = dgsem.lgl(wl.N)
    U, dt = workloads.make_state(wl, xi)
    Ud = torch.as_tensor(U.reshape(-1)).cuda()
    S = dgsem.solver_for(wl)
    S.set_state(Ud)

    def timed(run):
        run(warmup)
        S.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(S.stream)
        run(steps)
        b.record(S.stream)
        S.sync()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    def eager(k):
        for _ in range(k):
            S.rk_step(dt, 2)

    t_eager = timed(eager)
    S.rk_graph_build(dt, 2)
    t_graph = timed(lambda k: S.rk_graph_launch(k))
    per = lambda ms: ms * 1e6 / (S.n_dof * 2 * steps * 5)  # noqa: E731
    res = {"workload": wl.name, "dof": S.n_dof, "rk_steps": 2 * steps,
           "eager_ns_per_dof_stage": per(t_eager), "graph_ns_per_dof_stage": per(t_graph),
           "eager_us_per_step": t_eager * 1e3 / (2 * steps), "graph_us_per_step": t_graph * 1e3 / (2 * steps),
           "speedup": t_eager / t_graph}
    del S
    return res


def run_adjoint(steps: int, K: int):
    """Adjoint/forward time ratio on the N=5, 48x32x48 stretched channel as
    configured: a mixed-precision forward RK rollout of `steps` steps, then the
    checkpointed FP64 adjoint of the final kinetic energy (forward with a
    checkpoint every K steps, the last segment's stages recorded, the other
    segments recomputed once, reverse steps) against the plain forward of the
    same steps.  The gradient is compared per conserved variable with the
    all-FP64 (forward and adjoint) gradient of the same rollout."""
    import numpy as np
    import torch

    from paper_2606_18927_amd import dgsem, workloads
    from paper_2606_18927_amd.autograd import kinetic_energy_gradient

    wl = workloads.WORKLOADS["channel_n5_48x32x48"]
    xi, _ = dgsem.lgl(wl.N)
    U, dt = workloads.make_state(wl, xi)
    S = dgsem.solver_for(wl, with_adjoint=True)
    Ud = torch.as_tensor(U.reshape(-1)).cuda()
    del U
    S.set_state(Ud)
    S.rk_step(dt, 2)
    S.sync()
    ev = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))  # noqa: E731
    a, b = ev()
    S.set_state(Ud)
    a.record(S.stream)
    S.rk_step(dt, steps)
    b.record(S.stream)
    S.sync()
    torch.cuda.synchronize()
    t_fwd = a.elapsed_time(b)
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    base_mem = torch.cuda.memory_allocated()
    a, b = ev()
    a.record(S.stream)
    J, g = kinetic_energy_gradient(S, Ud, dt, steps, checkpoint_every=K)
    b.record(S.stream)
    torch.cuda.synchronize()
    t_adj = a.elapsed_time(b)
    peak_extra = torch.cuda.max_memory_allocated() - base_mem
    print(f"[bench] adjoint {steps} steps, K = {K}: forward {t_fwd:.0f} ms, forward + adjoint {t_adj:.0f} ms",
          file=sys.stderr, flush=True)
    dof = S.n_dof
    ws_gb = S.workspace_bytes / 1e9
    del S
    torch.cuda.empty_cache()
    # the all-FP64 reference gradient of the same rollout
    S64 = dgsem.solver_for(wl, with_adjoint=True, precision="fp64")
    J64, g64 = kinetic_energy_gradient(S64, Ud, dt, steps, checkpoint_every=K)
    torch.cuda.synchronize()
    gv, rv = g.view(5, -1), g64.view(5, -1)
    grad_err = ((gv - rv).norm(dim=1) / rv.norm(dim=1)).cpu().numpy()
    grad_max = ((gv - rv).abs().amax(dim=1) / rv.abs().amax(dim=1)).cpu().numpy()
    del S64, g64, g
    torch.cuda.empty_cache()
    # kernel level: one right-hand side vs one vector-Jacobian product (FP64),
    # for both flux pairs
    lam = torch.randn_like(Ud)

    def rhs_vs_vjp(flux):
        Sf = dgsem.solver_for(wl, with_adjoint=True, precision="fp64", flux=flux)
        out = Sf.state_like()
        for _ in range(2):
            Sf.eval_rhs(Ud, out)
            Sf.eval_rhs_vjp(Ud, lam, out)
        reps = 5
        a, b = ev()
        a.record(Sf.stream)
        for _ in range(reps):
            Sf.eval_rhs(Ud, out)
        b.record(Sf.stream)
        c, d = ev()
        c.record(Sf.stream)
        for _ in range(reps):
            Sf.eval_rhs_vjp(Ud, lam, out)
        d.record(Sf.stream)
        Sf.sync()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps, c.elapsed_time(d) / reps

    t_rhs, t_vjp = rhs_vs_vjp("kg_llf")
    t_rhs_ec, t_vjp_ec = rhs_vs_vjp("ec_roe")
    state_gb = 5 * dof * 8 / 1e9
    res = {"workload": wl.name, "dof": dof, "steps": steps, "checkpoint_every": K,
           "forward_precision": "mixed", "adjoint_precision": "fp64",
           "forward_ms": t_fwd, "forward_ns_per_dof_stage": t_fwd * 1e6 / (dof * steps * 5),
           "adjoint_total_ms": t_adj, "adjoint_forward_ratio": t_adj / t_fwd,
           "memory_gb": {"workspace": ws_gb, "checkpoints": (-(-steps // K) - 1) * state_gb,
                         "recorded_stages_one_segment": K * 25 * dof * 8 / 1e9,
                         "peak_beyond_state_and_workspace": peak_extra / 1e9},
           "gradient_vs_fp64": {"rel_l2_per_variable": [float(x) for x in grad_err],
                                "rel_max_per_variable": [float(x) for x in grad_max],
                                "J_rel_diff": abs(J.item() - J64.item()) / abs(J64.item())},
           "eval_rhs_fp64_ms": t_rhs, "eval_rhs_vjp_fp64_ms": t_vjp, "vjp_rhs_ratio": t_vjp / t_rhs,
           "ec_roe": {"eval_rhs_fp64_ms": t_rhs_ec, "eval_rhs_vjp_fp64_ms": t_vjp_ec,
                      "vjp_rhs_ratio": t_vjp_ec / t_rhs_ec},
           "J": J.item()}
    torch.cuda.empty_cache()
    return res


def run_freestream(steps: int, warmup: int):
    """The paper's throughput workload (a uniform free stream in the periodic
    box, N = 7; its PID does not depend on the solution) on the 32^3 mesh,
    FP64: a context row beside the Taylor-Green value."""
    from paper_2606_18927_amd import dgsem, workloads
    wl = workloads.WORKLOADS["freestream_n7_32x32x32"]
    xi, _ = dgsem.lgl(wl.N)
    U, dt = workloads.make_state(wl, xi)
    r, _ = run_precision(wl, U, dt, "fp64", steps, warmup)
    return _leg(wl.name, r)


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2606_18927_amd import dgsem, workloads

    wl = workloads.WORKLOADS[args.workload]
    xi, _ = dgsem.lgl(wl.N)
    U, dt = workloads.make_state(wl, xi)
    print(f"[bench] {wl.name}: {wl.n_dof} DOF, dt={dt:.4e}, steps={args.steps}, warmup={args.warmup}",
          file=sys.stderr, flush=True)

    fp64, Ud = run_precision(wl, U, dt, "fp64", args.steps, args.warmup, repeats=True)
    rp = fp64["repeats_ns_per_dof_stage"]
    print(f"[bench] fp64 {fp64['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage (5 more runs: min {rp['min']*1e3:.1f}, "
          f"median {rp['median']*1e3:.1f})", file=sys.stderr, flush=True)
    mixed = None
    if not args.no_mixed:
        try:
            mixed, _ = run_precision(wl, U, dt, "mixed", args.steps, args.warmup, repeats=True)
            print(f"[bench] mixed {mixed['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage", file=sys.stderr, flush=True)
        except dgsem.DgsemError as e:
            mixed = {"error": str(e)}
    ec = None
    if not args.no_ec and wl.name == "tgv_n7_32x32x32":
        # the paper's production flux pair on the same workload, FP64
        wl_ec = workloads.WORKLOADS["tgv_n7_32x32x32_ec"]
        r, _ = run_precision(wl_ec, U, dt, "fp64", args.steps, args.warmup)
        ec = {"workload": wl_ec.name, "flux": "ec_roe", "ns_per_dof_stage": r["ns_per_dof_stage"],
              "ms_per_step": r["ms_per_step"], "rk_kernel_ms": r["rk_kernel_ms"],
              "face_kernel_ms": r["face_kernel_ms"], "step_alg_gbs": r["step_alg_gbs"],
              "step_frac": r["step_alg_gbs"] / HBM_PEAK_GBS}
        print(f"[bench] ec_roe {ec['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage", file=sys.stderr, flush=True)
        if not args.no_mixed:
            rm, _ = run_precision(wl_ec, U, dt, "mixed", args.steps, args.warmup)
            ec["mixed"] = {k: rm[k] for k in ("ns_per_dof_stage", "ms_per_step", "rk_kernel_ms",
                                              "face_kernel_ms", "step_alg_gbs")}
            print(f"[bench] ec_roe mixed {rm['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage", file=sys.stderr,
                  flush=True)
    suth = wall = None
    if not args.no_physics and wl.name == "tgv_n7_32x32x32":
        wl_s = workloads.WORKLOADS["tgv_n7_32x32x32_sutherland"]
        try:
            r, _ = run_precision(wl_s, U, dt, "fp64", args.steps, args.warmup)
            suth = _leg(wl_s.name, r)
            print(f"[bench] sutherland {suth['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage", file=sys.stderr,
                  flush=True)
        except dgsem.DgsemError as e:
            suth = {"error": str(e)}
        try:
            wall = run_wall_model(args.steps, args.warmup)
            print(f"[bench] wall model channel {wall['wall_model']['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage "
                  f"(mixed {wall['wall_model_mixed']['ns_per_dof_stage']*1e3:.1f}; "
                  f"isothermal {wall['isothermal_constant_mu']['ns_per_dof_stage']*1e3:.1f}); "
                  f"k_wall_stress {wall['k_wall_stress']['ms_per_launch']*1e3:.1f} us", file=sys.stderr,
                  flush=True)
            print(f"[bench] production physics (ec_roe + wall model + Sutherland) "
                  f"{wall['production_ec_roe']['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage, mixed "
                  f"{wall['production_ec_roe_mixed']['ns_per_dof_stage']*1e3:.1f}", file=sys.stderr, flush=True)
        except dgsem.DgsemError as e:
            wall = {"error": str(e)}
    curved = None
    if not args.no_curved and wl.name == "tgv_n7_32x32x32":
        try:
            curved = run_curved(args.steps, args.warmup)
            print(f"[bench] curved {curved['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage, k_rhs_curv "
                  f"{curved['rk_kernel_ms']*1e3:.0f} us ({curved['rk_frac']*100:.0f} % of HBM)", file=sys.stderr,
                  flush=True)
            cec = run_curved(args.steps, args.warmup, flux="ec_roe")
            curved["ec_roe"] = {k: cec[k] for k in ("ns_per_dof_stage", "ms_per_step", "rk_kernel_ms",
                                                     "face_kernel_ms", "step_frac")}
            print(f"[bench] curved ec_roe {cec['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage", file=sys.stderr,
                  flush=True)
            cmx = run_curved(args.steps, args.warmup, precision="mixed")
            curved["mixed"] = {k: cmx[k] for k in ("ns_per_dof_stage", "ms_per_step", "rk_kernel_ms",
                                                   "face_kernel_ms", "rk_kernel_gbs", "step_frac", "rk_traffic",
                                                   "rk_traffic_over_algorithmic")}
            print(f"[bench] curved mixed {cmx['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage", file=sys.stderr,
                  flush=True)
            cem = run_curved(args.steps, args.warmup, flux="ec_roe", precision="mixed")
            curved["ec_roe"]["mixed"] = {k: cem[k] for k in ("ns_per_dof_stage", "ms_per_step", "rk_kernel_ms",
                                                             "face_kernel_ms", "step_frac")}
            print(f"[bench] curved ec_roe mixed {cem['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage",
                  file=sys.stderr, flush=True)
        except dgsem.DgsemError as e:
            curved = {"error": str(e)}
    small = None
    if wl.name == "tgv_n7_32x32x32":
        small = run_small_graph(100, 5)
        print(f"[bench] {small['workload']}: {small['eager_us_per_step']:.1f} us/step launched, "
              f"{small['graph_us_per_step']:.1f} us/step from a HIP graph", file=sys.stderr, flush=True)
    freestream = None
    if wl.name == "tgv_n7_32x32x32":
        freestream = run_freestream(args.steps, args.warmup)
        print(f"[bench] free stream {freestream['ns_per_dof_stage']*1e3:.1f} ps/DOF/stage", file=sys.stderr,
              flush=True)
    adjoint = None
    if not args.no_adjoint:
        adjoint = run_adjoint(args.adjoint_steps, 25)
        print(f"[bench] adjoint/forward {adjoint['adjoint_forward_ratio']:.2f} "
              f"(gradient vs FP64 rel L2 max {max(adjoint['gradient_vs_fp64']['rel_l2_per_variable']):.1e}); "
              f"vjp/rhs kg_llf {adjoint['vjp_rhs_ratio']:.2f}, ec_roe {adjoint['ec_roe']['vjp_rhs_ratio']:.2f}",
              file=sys.stderr, flush=True)
    triad = triad_gbs()
    print(f"[bench] triad {triad:.0f} GB/s", file=sys.stderr, flush=True)
    cpu = None if args.no_cpu else cpu_baseline(wl)

    value = fp64["ns_per_dof_stage"]
    traffic = counted_traffic() if wl.name == "tgv_n7_32x32x32" else None
    dof = fp64["dof"]
    rk_s = fp64["rk_kernel_ms"] / 1e3
    alg_rk_bytes = RHS_STAGE_BYTES_PER_DOF * dof          # per launch
    achieved = alg_rk_bytes / rk_s / 1e9
    counted_flops = counted_traffic(COUNTED_FLOPS) if wl.name == "tgv_n7_32x32x32" else None
    step_s_per_stage = value * 1e-9 * dof                 # seconds per RK stage
    alg_tflops = ALG_FLOPS_PER_DOF_STAGE * dof / step_s_per_stage / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ns/DOF/stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp64["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Taylor-Green state + 1% velocity noise)",
        "config": {"workload": wl.name, "N": wl.N, "elements": list(wl.nelem), "dof": wl.n_dof,
                   "rk_stages_per_step": 5, "precision": "fp64"},
        "dof_stage_per_s": 1e9 / value,
        "repeats_ns_per_dof_stage": fp64["repeats_ns_per_dof_stage"],
        "roofline": {
            "bound": "hbm",
            "kernel": "k_rhs (fused right-hand side + RK stage)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_dof": RHS_STAGE_BYTES_PER_DOF,
            "alg_bytes_per_launch": alg_rk_bytes,
            "kernel_ms": fp64["rk_kernel_ms"],
            "traffic_unit": "bytes per launch (rocprofv3 TCC_EA0_RDREQ_{32,64,128}B + WRITE_SIZE)",
            "traffic_gbs": None if traffic is None else traffic / rk_s / 1e9,
            "own_bytes_per_launch": fp64["rk_bytes_per_launch"],
            "own_bytes_gbs": fp64["rk_kernel_gbs"],
            "frac_own_bytes": fp64["rk_kernel_gbs"] / HBM_PEAK_GBS,
            "traffic_over_own_bytes": None if traffic is None else traffic / fp64["rk_bytes_per_launch"],
            "face_kernel_ms": fp64["face_kernel_ms"],
            "face_kernel_gbs": fp64["face_kernel_gbs"],
            "step_alg_bytes_per_dof": STORED_GRADIENT_BYTES_PER_DOF,
            "step_frac": STORED_GRADIENT_BYTES_PER_DOF / value / HBM_PEAK_GBS,
            "step_own_bytes_per_dof": fp64["step_alg_bytes_per_dof"],
            "step_frac_own_bytes": fp64["step_alg_gbs"] / HBM_PEAK_GBS,
            "triad_gbs": triad,
            "step_frac_of_triad": STORED_GRADIENT_BYTES_PER_DOF / value / triad,
        },
        "fp64_compute": {
            "alg_flop_per_dof_stage": ALG_FLOPS_PER_DOF_STAGE,
            "achieved_tflops": alg_tflops,
            "peak_tflops": FP64_PEAK_TFLOPS,
            "frac": alg_tflops / FP64_PEAK_TFLOPS,
            "counted_flop_per_dof_stage": counted_flops,
            "counted_frac": None if counted_flops is None else
            counted_flops * dof / step_s_per_stage / 1e12 / FP64_PEAK_TFLOPS,
        },
        "cpu_baseline": cpu,
        "mixed": mixed,
        "ec_roe": ec,
        "sutherland": suth,
        "curved": curved,
        "wall_model": wall,
        "adjoint": adjoint,
        "small_case_graph": small,
        "freestream_context": freestream,
        "context_mi300a_pid_ns": {"range": [2.457, 4.260], "note": "paper Table 1, 32 APUs, N=7 free stream"},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
