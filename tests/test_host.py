"""Host-side logic (CPU): the bench contract, the algorithmic byte counts the
roofline is priced on, the seeded inputs (warped meshes and states), and the
binding's behaviour when the library is missing."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2606_18927_amd import dgsem, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    b = bench.alg_bytes("fp64", 7)
    # per stage: face kernel 64, fused kernel 184 (144 on stage 1): 240 on average
    assert b["face"] == 64 and b["rk"] == 184 and b["rk_first"] == 144
    assert b["face"] + (4 * b["rk"] + b["rk_first"]) / 5 == 240
    m = bench.alg_bytes("mixed", 7)
    assert m["face"] + (4 * m["rk"] + m["rk_first"]) / 5 == 216
    c = bench.curved_alg_bytes(7)
    assert c["rk"] == 264 and c["rk_first"] == 224
    assert c["face"] == pytest.approx(40 + 80 * 296 / 512 + 24)
    assert c["face"] + (4 * c["rk"] + c["rk_first"]) / 5 == pytest.approx(366.25)


def test_warped_nodes_periodic_and_shared_faces():
    N, n = 5, (3, 2, 4)
    xi, _ = dgsem.lgl(N)
    X = workloads.warped_nodes(xi, n, amp=0.07)
    assert X.shape == (3, n[2], n[1], n[0], N + 1, N + 1, N + 1)
    # neighbours along x share their face nodes bitwise
    assert np.array_equal(X[:, :, :, :-1, :, :, N], X[:, :, :, 1:, :, :, 0])
    assert np.array_equal(X[:, :, :-1, :, :, N, :], X[:, :, 1:, :, :, 0, :])
    assert np.array_equal(X[:, :-1, :, :, N, :, :], X[:, 1:, :, :, 0, :, :])
    # across the periodic end the face differs by the period in x and to
    # rounding in y, z
    L = 2 * np.pi
    a, b = X[:, :, :, -1, :, :, N], X[:, :, :, 0, :, :, 0]
    assert np.allclose(a[0] - b[0], L, rtol=0, atol=1e-14)
    assert np.allclose(a[1:], b[1:], rtol=0, atol=1e-14)
    # amp = 0 is the uniform tensor mesh
    X0 = workloads.warped_nodes(xi, n, amp=0.0)
    faces = tuple(L * np.arange(k + 1) / k for k in n)
    ref = workloads.node_coords(xi, faces)
    for d in range(3):
        assert np.allclose(X0[d], ref[d], rtol=0, atol=1e-14)


def test_curved_workload_state():
    wl = workloads.WORKLOADS["tgv_n3_4x4x4_curved"]
    xi, _ = dgsem.lgl(wl.N)
    U, dt = workloads.make_state(wl, xi)
    X = wl.nodes(xi)
    assert U.shape == (5,) + X.shape[1:] and dt > 0
    # the Taylor-Green fields are evaluated at the displaced nodes
    p0 = 1.0 / (wl.gamma * wl.Ma ** 2)
    u = np.sin(X[0]) * np.cos(X[1]) * np.cos(X[2])
    assert np.allclose(U[1] / U[0], u, rtol=0, atol=1e-14)
    p = p0 + (np.cos(2 * X[0]) + np.cos(2 * X[1])) * (np.cos(2 * X[2]) + 2.0) / 16.0
    assert np.allclose(U[0], p / wl.R, rtol=1e-15, atol=0)
    assert workloads.WORKLOADS["tgv_n3_4x4x4"].nodes(xi) is None


def test_mesh_spec_from_nodes():
    X = np.zeros((3, 4, 3, 2, 4, 4, 4))
    spec = dgsem.MeshSpec(3, None, nodes=X)
    assert spec.nelem == (2, 3, 4)


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(dgsem, "_lib", None)
    monkeypatch.setattr(dgsem, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libdgsem.so"))
    with pytest.raises(dgsem.DgsemError) as ei:
        dgsem.lib()
    assert ei.value.status == dgsem.DG_ESTATE


def test_segments_recorded_in_the_forward_pass():
    """The checkpointed adjoint records the trailing segments that fit the
    stage-memory budget (K 25 n_dof doubles each), at least one, at most all."""
    from types import SimpleNamespace

    from paper_2606_18927_amd.autograd import _segments_to_record
    S = SimpleNamespace(n_dof=1000)
    per = 25 * 25 * 1000 * 8  # K = 25
    assert _segments_to_record(S, 50, 25, None) == 1
    assert _segments_to_record(S, 50, 25, 0) == 1
    assert _segments_to_record(S, 50, 25, 2 * per) == 2
    assert _segments_to_record(S, 50, 25, 10 * per) == 2
    assert _segments_to_record(S, 51, 25, 10 * per) == 3
    assert _segments_to_record(S, 60, 25, 2 * per + per // 2) == 2
