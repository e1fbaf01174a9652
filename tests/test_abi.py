"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/dgsem.h declares, and its host-only entry points (LGL tables, argument
validation, workspace sizing) behave as documented."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2606_18927_amd import dgsem
from oracle.basis import lgl as oracle_lgl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgsem.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(dgsem.LIB_PATH):
        pytest.fail("libdgsem.so is not built (python -m paper_2606_18927_amd.build)")
    return dgsem.lib()


def test_library_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(dgsem.exported_symbols())


def test_version(L):
    assert dgsem.version().startswith("dgsem-gfx950")


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7, 9, 12])
def test_host_lgl_matches_independent_oracle_basis(L, N):
    xi, w = dgsem.lgl(N)
    xo, wo = oracle_lgl(N)
    assert np.allclose(xi, xo.numpy(), atol=2e-16 * 4, rtol=0)
    assert np.allclose(w, wo.numpy(), atol=1e-15, rtol=0)


def _desc(N=3, n=(2, 2, 2), faces=None, bc=(0, 0, 0), T_wall=1.0):
    desc = dgsem.MeshDesc()
    desc.N = N
    keep = []
    for d in range(3):
        f = np.ascontiguousarray(faces[d] if faces else np.linspace(0, 1, n[d] + 1))
        keep.append(f)
        desc.nelem[d] = n[d]
        desc.faces[d] = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        desc.bc[d] = bc[d]
    desc.T_wall = T_wall
    return desc, keep


def _init(L, desc, phys):
    ctx = ctypes.c_void_p()
    st = L.dg_init_mesh(ctypes.byref(desc), ctypes.byref(phys), None, ctypes.byref(ctx))
    return st, ctx


def _phys(**kw):
    base = dict(gamma=1.4, R=1.0, mu=0.01, Pr=0.72, viscous=1, precision=0, central_only=0, flux=0,
                viscosity=0, T_ref=0.0, S=0.0)
    base.update(kw)
    return dgsem.Physics(base["gamma"], base["R"], base["mu"], base["Pr"], base["viscous"],
                         base["precision"], base["central_only"], base["flux"], base["viscosity"],
                         base["T_ref"], base["S"])


def test_init_mesh_validation_errors(L):
    d, keep = _desc()
    st, ctx = _init(L, d, _phys())
    assert st == dgsem.DG_OK
    L.dg_free(ctx)
    d, keep = _desc(N=4)
    assert _init(L, d, _phys())[0] == dgsem.DG_EUNSUPPORTED
    # flux choice: the entropy-conserving / Roe pair in FP64 and mixed precision
    # (not without the reference state); unknown values are rejected
    d, keep = _desc()
    for prec in (0, 1):
        st, ctx = _init(L, d, _phys(flux=1, precision=prec))
        assert st == dgsem.DG_OK
        L.dg_free(ctx)
    assert _init(L, d, _phys(flux=1, precision=2))[0] == dgsem.DG_EUNSUPPORTED
    assert _init(L, d, _phys(flux=2))[0] == dgsem.DG_EINVAL
    # viscosity law: Sutherland's needs T_ref > 0 and S >= 0
    st, ctx = _init(L, d, _phys(viscosity=1, T_ref=1.0, S=0.38))
    assert st == dgsem.DG_OK
    L.dg_free(ctx)
    st, ctx = _init(L, d, _phys(viscosity=1, T_ref=1.0, S=0.38, precision=1))  # mixed precision too
    assert st == dgsem.DG_OK
    L.dg_free(ctx)
    for bad in (dict(viscosity=2), dict(viscosity=1, T_ref=0.0, S=0.38), dict(viscosity=1, T_ref=1.0, S=-1.0),
                dict(viscosity=1, T_ref=float("inf"), S=0.38)):
        assert _init(L, d, _phys(**bad))[0] == dgsem.DG_EINVAL, bad
    # a constant-viscosity context ignores T_ref and S
    st, ctx = _init(L, d, _phys(T_ref=-1.0, S=-1.0))
    assert st == dgsem.DG_OK
    L.dg_free(ctx)
    d, keep = _desc(faces=(np.array([0.0, 0.5, 0.4]), np.linspace(0, 1, 3), np.linspace(0, 1, 3)))
    assert _init(L, d, _phys())[0] == dgsem.DG_EINVAL          # non-monotone faces
    d, keep = _desc(bc=(0, 7, 0))
    assert _init(L, d, _phys())[0] == dgsem.DG_EINVAL          # unknown boundary kind
    d, keep = _desc(bc=(0, 1, 0), T_wall=0.0)
    assert _init(L, d, _phys())[0] == dgsem.DG_EINVAL          # wall needs T_wall > 0
    d, keep = _desc()
    for bad in (dict(gamma=1.0), dict(R=0.0), dict(mu=-1.0), dict(Pr=0.0), dict(precision=3)):
        assert _init(L, d, _phys(**bad))[0] == dgsem.DG_EINVAL, bad
    d, keep = _desc(n=(0, 2, 2))
    assert _init(L, d, _phys())[0] == dgsem.DG_EINVAL
    assert L.dg_init_mesh(None, None, None, None) == dgsem.DG_EINVAL


def test_workspace_size_and_state_errors(L):
    d, keep = _desc(N=7, n=(3, 2, 5))
    st, ctx = _init(L, d, _phys())
    assert st == dgsem.DG_OK
    n = ctypes.c_longlong()
    assert L.dg_n_dof(ctx, ctypes.byref(n)) == dgsem.DG_OK and n.value == 30 * 512
    fwd, adj = ctypes.c_size_t(), ctypes.c_size_t()
    L.dg_workspace_bytes(ctx, 0, ctypes.byref(fwd))
    L.dg_workspace_bytes(ctx, 1, ctypes.byref(adj))
    dof = n.value
    # three states (U ping-pong and G) plus the face viscous fluxes
    # (6 faces x 4 components x 64 face nodes per 512-node element = 3 per DOF)
    assert fwd.value >= (15 + 3) * dof * 8 and fwd.value < (15 + 3) * dof * 8 + 64 * 1024
    assert adj.value > fwd.value
    # no workspace bound yet: device calls are refused before any HIP call
    assert L.dg_rk_step(ctx, 0.0, 1e-3, 1) == dgsem.DG_ESTATE
    assert L.dg_eval_rhs(ctx, None, None, 0.0) == dgsem.DG_ESTATE
    assert L.dg_rk_record_stages(ctx, None, 0.0, 1e-3, 1, None) == dgsem.DG_ESTATE
    assert L.dg_rk_step_vjp_stages(ctx, None, 0.0, 1e-3, None, None) == dgsem.DG_ESTATE
    assert b"workspace" in L.dg_last_error(ctx)
    L.dg_free(ctx)
    # mixed precision halves the face-flux storage
    st, ctx = _init(L, d, _phys(precision=1))
    mixed = ctypes.c_size_t()
    L.dg_workspace_bytes(ctx, 0, ctypes.byref(mixed))
    assert fwd.value - mixed.value >= 3 * dof * 4 - 4096
    L.dg_free(ctx)


def test_wall_face_count(L):
    """dg_wall_faces is host-only: 2 nb nc per wall direction."""
    n = ctypes.c_longlong()
    for bc, expected in (((0, 0, 0), 0), ((0, 1, 0), 2 * 3 * 5), ((1, 1, 1), 2 * (2 * 5 + 3 * 5 + 3 * 2))):
        d, keep = _desc(n=(3, 2, 5), bc=bc)
        st, ctx = _init(L, d, _phys())
        assert st == dgsem.DG_OK
        assert L.dg_wall_faces(ctx, ctypes.byref(n)) == dgsem.DG_OK and n.value == expected
        # device call without a workspace is refused before any HIP call
        assert L.dg_wall_stress(ctx, None, 1, None) == dgsem.DG_ESTATE
        L.dg_free(ctx)


def test_curved_mesh_validation(L):
    """Curved elements (node coordinates given): periodic or isothermal-wall
    ends, FP64 (either flux pair); faces may be absent; non-finite
    coordinates are rejected.  Host only."""
    from paper_2606_18927_amd.workloads import warped_nodes
    N, n = 3, (2, 2, 2)
    X = np.ascontiguousarray(warped_nodes(dgsem.lgl(N)[0], n)).reshape(-1)

    def desc(bc=(0, 0, 0), nodes=X, with_faces=False):
        d, keep = _desc(N=N, n=n, bc=bc)
        if not with_faces:
            for k in range(3):
                d.faces[k] = ctypes.POINTER(ctypes.c_double)()
        d.nodes = nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return d, keep

    d, keep = desc()
    st, ctx = _init(L, d, _phys())
    assert st == dgsem.DG_OK
    size = ctypes.c_size_t()
    assert L.dg_workspace_bytes(ctx, 0, ctypes.byref(size)) == dgsem.DG_OK
    L.dg_free(ctx)
    d0, keep0 = _desc(N=N, n=n)
    plain = ctypes.c_size_t()
    st, ctx = _init(L, d0, _phys())
    L.dg_workspace_bytes(ctx, 0, ctypes.byref(plain))
    L.dg_free(ctx)
    nd = 8 * 64
    nfn = 2 * (N + 1) ** 2 + (N - 1) * 4 * N  # boundary nodes per element
    # metric terms: 10 values per DOF, and again per boundary node
    assert size.value >= plain.value + 10 * nd * 8 + 10 * 8 * nfn * 8
    d, keep = desc()
    st, ctx = _init(L, d, _phys(precision=1))  # mixed precision with the Kennedy-Gruber pair
    assert st == dgsem.DG_OK
    mixed = ctypes.c_size_t()
    assert L.dg_workspace_bytes(ctx, 0, ctypes.byref(mixed)) == dgsem.DG_OK
    L.dg_free(ctx)
    # the FP32 copy of the metric terms (10 values per DOF) exists only in
    # mixed precision, whose face fluxes are FP32 (half the FP64 ones)
    ff64 = 8 * 6 * 4 * (N + 1) ** 2 * 8
    assert mixed.value >= size.value + 10 * nd * 4 - ff64 // 2 - 4096
    assert mixed.value <= size.value + 10 * nd * 4 + 4096
    d, keep = desc()  # the entropy-conserving pair in mixed precision
    st, ctx = _init(L, d, _phys(precision=1, flux=1))
    assert st == dgsem.DG_OK
    L.dg_free(ctx)
    assert _init(L, d, _phys(precision=2, flux=1))[0] == dgsem.DG_EUNSUPPORTED  # not without the reference
    d, keep = desc(bc=(0, 1, 0))  # isothermal walls are fine
    st, ctx = _init(L, d, _phys())
    assert st == dgsem.DG_OK
    L.dg_free(ctx)
    d, keep = desc(bc=(0, 2, 0))  # the wall model is not
    d.wm_node = 1
    assert _init(L, d, _phys())[0] == dgsem.DG_EUNSUPPORTED
    Xn = X.copy()
    Xn[17] = np.nan
    d, keep = desc(nodes=Xn)
    assert _init(L, d, _phys())[0] == dgsem.DG_EINVAL
    # faces are still required without node coordinates
    d, keep = _desc(N=N, n=n)
    d.faces[1] = ctypes.POINTER(ctypes.c_double)()
    assert _init(L, d, _phys())[0] == dgsem.DG_EINVAL
