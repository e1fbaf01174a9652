"""dg_eval_rhs_noalloc (the right-hand side with its scratch in a static
device array) against dg_eval_rhs through the C ABI (GPU).

Two calls in a row on different contexts, the second on a smaller mesh (so
the tables and scratch left by the first call must not leak into it), then
the first again; each must equal dg_eval_rhs bit for bit (the same kernels
run in the same order) and the oracle to the FP64 parity bound.  A context
that never bound a workspace works too; the status word reports a negative
density; a mesh beyond the scratch size is rejected on the host.
"""

import ctypes

import numpy as np
import pytest
import torch

from oracle.dgsem import rhs
from oracle.mesh import Mesh
from oracle.physics import Gas
from paper_2606_18927_amd import dgsem

from _cases import random_faces, random_state
from _gpu import need_gpu, rel_l2, say

pytestmark = pytest.mark.gpu


def _case(N, n, bc, seed, mixed=False):
    rng = np.random.default_rng(seed)
    faces = tuple(random_faces(n[d], -1.0, 1.0, rng) if bc[d] == "wall" else random_faces(n[d], 0.0, 2.0 + d, rng)
                  for d in range(3))
    mesh = Mesh(N, faces, bc=bc, T_wall=1.1)
    g = Gas(gamma=1.4, R=1.0 / (1.4 * 0.01), mu=0.01, Pr=0.72)
    U = random_state(mesh, g.gamma, g.R, rng, vel_amp=1.0, p_mean=1.0 / (1.4 * 0.01), p_amp=0.05)
    S = dgsem.Solver(dgsem.MeshSpec(N, faces, bc, 1.1), g.gamma, g.R, g.mu, g.Pr,
                     precision="mixed" if mixed else "fp64")
    return mesh, g, U.numpy(), S


def _noalloc(S, Ud, status=None):
    out = S.state_like()
    st = dgsem.lib().dg_eval_rhs_noalloc(S._ctx, Ud.data_ptr(), out.data_ptr(), 0.0,
                                         0 if status is None else status.data_ptr())
    assert st == dgsem.DG_OK, dgsem.lib().dg_last_error(S._ctx)
    torch.cuda.synchronize()
    return out


def test_noalloc_matches_eval_rhs_two_calls_second_smaller():
    need_gpu()
    cases = [("N=5 6x5x4, walls in y, FP64", 5, (6, 5, 4), ("periodic", "wall", "periodic"), 1, False),
             ("N=3 3x2x2 periodic, mixed", 3, (3, 2, 2), ("periodic",) * 3, 2, True)]
    built = [(_case(N, n, bc, seed, mixed), tag, 1e-4 if mixed else 1e-12)
             for tag, N, n, bc, seed, mixed in cases]
    for (mesh, g, U, S), tag, bound in built + built[:1]:
        say("case", tag)
        Ud = torch.as_tensor(U.reshape(-1)).cuda()
        ref_gpu = S.eval_rhs(Ud)
        S.sync()
        got = _noalloc(S, Ud)
        assert torch.equal(got, ref_gpu)
        ref = rhs(torch.as_tensor(U), mesh, g).numpy()
        e = rel_l2(got.cpu().numpy().reshape(ref.shape), ref)
        say("  rel L2 vs oracle", e)
        assert np.all(e < bound)


def _raw_ctx(N, faces, bc, g):
    """A context from dg_init_mesh alone: no workspace is ever bound."""
    L = dgsem.lib()
    desc = dgsem.MeshDesc()
    desc.N = N
    keep = [np.ascontiguousarray(f, dtype=np.float64) for f in faces]
    for d in range(3):
        desc.nelem[d] = len(faces[d]) - 1
        desc.faces[d] = keep[d].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        desc.bc[d] = dgsem.BC[bc[d]]
    desc.T_wall = 1.1
    desc.wm_node = 1
    phys = dgsem.Physics(g.gamma, g.R, g.mu, g.Pr, 1, 0, 0, 0, 0, 0.0, 0.0)
    ctx = ctypes.c_void_p()
    st = L.dg_init_mesh(ctypes.byref(desc), ctypes.byref(phys), torch.cuda.current_stream().cuda_stream,
                        ctypes.byref(ctx))
    assert st == dgsem.DG_OK
    return ctx, keep


def test_noalloc_without_workspace_and_status():
    need_gpu()
    mesh, g, U, S = _case(3, (4, 3, 5), ("wall", "periodic", "periodic"), 3)
    Ud = torch.as_tensor(U.reshape(-1)).cuda()
    ref_gpu = S.eval_rhs(Ud)
    S.sync()
    ctx, keep = _raw_ctx(3, mesh.faces, mesh.bc, g)
    L = dgsem.lib()
    try:
        out = torch.empty_like(Ud)
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        assert L.dg_eval_rhs_noalloc(ctx, Ud.data_ptr(), out.data_ptr(), 0.0, status.data_ptr()) == dgsem.DG_OK
        torch.cuda.synchronize()
        assert torch.equal(out, ref_gpu)
        assert status.item() == 0
        bad = Ud.clone()
        bad[5] = -1.0  # a negative density
        assert L.dg_eval_rhs_noalloc(ctx, bad.data_ptr(), out.data_ptr(), 0.0, status.data_ptr()) == dgsem.DG_OK
        torch.cuda.synchronize()
        assert status.item() == 1
    finally:
        L.dg_free(ctx)


def test_noalloc_rejects_a_mesh_beyond_the_scratch():
    need_gpu()
    g = Gas(gamma=1.4, R=1.0, mu=0.01, Pr=0.72)
    faces = tuple(np.linspace(0.0, 1.0, 49) for _ in range(3))
    ctx, keep = _raw_ctx(7, faces, ("periodic",) * 3, g)
    L = dgsem.lib()
    try:
        x = torch.zeros(1, dtype=torch.float64, device="cuda")
        assert L.dg_eval_rhs_noalloc(ctx, x.data_ptr(), x.data_ptr(), 0.0, 0) == dgsem.DG_EINVAL
        assert b"too large" in L.dg_last_error(ctx)
    finally:
        L.dg_free(ctx)
