"""Split-form DGSEM right-hand side, BR1 lifting and low-storage RK of the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Semi-discrete form (paper Sec. 2.2: split-form DG on LGL nodes; Sec. 4: viscous
Navier-Stokes of an ideal gas) on an affine hexahedral element with reference
coordinates xi in [-1, 1]^3, scales s_d = 2/width_d, LGL weights w and
derivative matrix D.  Written for direction x; y and z are the same along
their own line index.

Lifting (BR1, strong form) of the primitive gradients q in (u, v, w, T):

    g_x[i] = s_x ( sum_m D_im q_m + delta_iN (q*_R - q_N) / w_N
                                  - delta_i0 (q*_L - q_0) / w_0 ),

with q* the mean of the two sides' primitive values at a shared face node
(readings: the lifted set is (u, v, w, T); the face value averages the
primitives, not the conservative states) and q* = (0, 0, 0, T_wall) at a wall.

Right-hand side (strong form, reading: the strong form is used; on LGL nodes it
equals the weak form up to rounding through the summation-by-parts property):

    Ut[i] = - sum_d s_d ( 2 sum_m D_im f#_d(U_i, U_m) - sum_m D_im f_v,d(U_m, g_m)
                          + delta_iN ((F*_c - F*_v)_R - (f_d - f_v,d)(U_N)) / w_N
                          - delta_i0 ((F*_c - F*_v)_L - (f_d - f_v,d)(U_0)) / w_0 ),

with F*_c the local Lax-Friedrichs flux (Kennedy-Gruber central part) and
F*_v = (f_v,d(U_L, g_L) + f_v,d(U_R, g_R)) / 2 (BR1 central viscous flux, each
side with its own lifted gradients).  At a wall the face flux is the wall flux
of ``physics``.

Time integration (paper Sec. 4: fourth-order low-storage RK; the coefficients
are those of Carpenter & Kennedy's five-stage fourth-order 2N-storage scheme):

    for s = 1..5:   G <- A_s G + dt L(U);   U <- U + B_s G,   with G = 0 at step start.

Objective: volume-averaged kinetic energy with LGL collocation quadrature,
J(U) = sum_nodes w_i w_j w_k J_e |m|^2 / (2 rho) / sum_nodes w_i w_j w_k J_e.

Element traversal and summation follow index order; no blocking or fusion.
"""

from __future__ import annotations

from fractions import Fraction

import torch

from .basis import diff_matrix, lgl
from .mesh import ELEM_AXIS, NODE_AXIS, WALL, WALL_MODEL, Mesh
from .physics import (FLUXES, Gas, Prim, ec_flux, euler_flux, kg_flux, llf_flux, primitives,
                      roe_flux, viscous_flux, wall_convective_flux)

__all__ = ["from_flat", "to_flat", "lift", "rhs", "lsrk", "rk_step", "kinetic_energy",
           "RK_A", "RK_B", "RK_C"]

# Carpenter & Kennedy (1994) RK4(5) 2N-storage coefficients
RK_A = tuple(float(x) for x in (
    Fraction(0),
    Fraction(-567301805773, 1357537059087),
    Fraction(-2404267990393, 2016746695238),
    Fraction(-3550918686646, 2091501179385),
    Fraction(-1275806237668, 842570457699)))
RK_B = tuple(float(x) for x in (
    Fraction(1432997174477, 9575080441755),
    Fraction(5161836677717, 13612068292357),
    Fraction(1720146321549, 2090206949498),
    Fraction(3134564353537, 4481467310338),
    Fraction(2277821191437, 14882151754819)))
RK_C = tuple(float(x) for x in (
    Fraction(0),
    Fraction(1432997174477, 9575080441755),
    Fraction(2526269341429, 6820363962896),
    Fraction(2006345519317, 3224310063776),
    Fraction(2802321613138, 2924317926251)))


def from_flat(U_flat: torch.Tensor, mesh: Mesh) -> torch.Tensor:
    """Canonical flat layout [v][e][node] -> (5, nz, ny, nx, k, j, i)."""
    return U_flat.reshape((U_flat.shape[0],) + mesh.shape)


def to_flat(U: torch.Tensor) -> torch.Tensor:
    return U.reshape(U.shape[0], -1)


# ----------------------------------------------------------------- line tools

def _apply_D(q: torch.Tensor, D: torch.Tensor, na: int) -> torch.Tensor:
    """sum_m D[i, m] q[.., m, ..] along node axis na."""
    return (q.movedim(na, -1) @ D.to(q.dtype).T).movedim(-1, na)


def _at_node(plane: torch.Tensor, na: int, idx: int, NP: int) -> torch.Tensor:
    """Nodal field equal to `plane` on node index idx along axis na, zero elsewhere."""
    onehot = torch.zeros(NP, dtype=torch.float64)
    onehot[idx] = 1.0
    shape = [1] * (plane.dim() + 1)
    shape[na] = NP
    return plane.unsqueeze(na) * onehot.to(plane.dtype).reshape(shape)


def _end_mask(plane: torch.Tensor, ea: int, last: bool) -> torch.Tensor:
    n = plane.shape[ea]
    m = torch.zeros(n, dtype=torch.bool)
    m[n - 1 if last else 0] = True
    shape = [1] * plane.dim()
    shape[ea] = n
    return m.reshape(shape)


def _wall_plane(t: torch.Tensor, like: torch.Tensor, d: int, ea: int) -> torch.Tensor:
    """Wall-face values t[eb, ea, b, a] (face nodes (a, b) = (j, k), (i, k), (i, j)
    and wall elements (ea, eb) = (ey, ez), (ex, ez), (ex, ey) for d = x, y, z)
    placed on a face plane shaped like `like`: (nz, ny, nx, ...) without the
    direction-d element and node axes selected, broadcast along the d element axis."""
    # the plane tensors keep the element axes (nz, ny, nx) and two node axes
    # ordered (k, j, i) without the d one; e.g. d = 1: (nz, ny, nx, k, i)
    out = torch.zeros_like(like)
    if d == 0:      # like: (nz, ny, nx, k, j); t[ez, ey, k, j]
        val = t.permute(0, 1, 2, 3)[:, :, None, :, :]
    elif d == 1:    # like: (nz, ny, nx, k, i); t[ez, ex, k, i]
        val = t[:, None, :, :, :]
    else:           # like: (nz, ny, nx, j, i); t[ey, ex, j, i]
        val = t[None, :, :, :, :]
    return out + val


def _prim_plane(P: Prim, na: int, idx: int) -> Prim:
    s = lambda x: x.select(na, idx)  # noqa: E731
    return Prim(s(P.rho), tuple(s(x) for x in P.vel), s(P.p), s(P.T), s(P.e), s(P.E))


def _prim_roll(P: Prim, shift: int, ea: int) -> Prim:
    r = lambda x: torch.roll(x, shift, ea)  # noqa: E731
    return Prim(r(P.rho), tuple(r(x) for x in P.vel), r(P.p), r(P.T), r(P.e), r(P.E))


def _prim_line(P: Prim, na: int, slot: int) -> Prim:
    """Move the node axis to the end and open a pair axis: slot -2 -> index i, -1 -> m."""
    def f(x):
        x = x.movedim(na, -1)
        return x.unsqueeze(-1) if slot == -2 else x.unsqueeze(-2)
    return Prim(f(P.rho), tuple(f(x) for x in P.vel), f(P.p), f(P.T), f(P.e), f(P.E))


# -------------------------------------------------------------------- lifting

def lift(U: torch.Tensor, mesh: Mesh, gas: Gas):
    """BR1 lifted gradients grad[q][d] of q in (u, v, w, T), each a nodal field."""
    N, NP = mesh.N, mesh.NP
    D = diff_matrix(N)
    _, w = lgl(N)
    P = primitives(U, gas)
    q = [P.vel[0], P.vel[1], P.vel[2], P.T]
    q_wall = [0.0, 0.0, 0.0, mesh.T_wall]
    grad = [[None] * 3 for _ in range(4)]
    for d in range(3):
        ea, na = ELEM_AXIS[d], NODE_AXIS[d]
        s = mesh.scale(d).to(U.dtype)
        for c in range(4):
            vol = _apply_D(q[c], D, na)
            lo, hi = q[c].select(na, 0), q[c].select(na, N)
            star_lo = 0.5 * (lo + torch.roll(hi, 1, ea))    # lower neighbour's last plane
            star_hi = 0.5 * (hi + torch.roll(lo, -1, ea))   # upper neighbour's first plane
            if mesh.bc[d] == WALL:
                wv = torch.full_like(lo, q_wall[c])
                star_lo = torch.where(_end_mask(lo, ea, last=False), wv, star_lo)
                star_hi = torch.where(_end_mask(hi, ea, last=True), wv, star_hi)
            elif mesh.bc[d] == WALL_MODEL:
                # slip, adiabatic wall: the own value with the normal velocity removed
                wlo = torch.zeros_like(lo) if c == d else lo
                whi = torch.zeros_like(hi) if c == d else hi
                star_lo = torch.where(_end_mask(lo, ea, last=False), wlo, star_lo)
                star_hi = torch.where(_end_mask(hi, ea, last=True), whi, star_hi)
            surf = (_at_node(star_hi - hi, na, N, NP) / w[N]
                    - _at_node(star_lo - lo, na, 0, NP) / w[0])
            grad[c][d] = s * (vol + surf)
    return grad


# --------------------------------------------------------------------- RHS

def rhs(U: torch.Tensor, mesh: Mesh, gas: Gas, *, viscous: bool = True,
        central_only: bool = False, source=None, flux: str = "kg_llf") -> torch.Tensor:
    """L(U) of the split-form DGSEM (module docstring).  U: (5, *mesh.shape).
    flux: "kg_llf" (Kennedy-Gruber volume flux, Lax-Friedrichs surface flux) or
    "ec_roe" (Chandrashekar volume flux, Roe surface flux with the Harten-Hyman
    correction, ``physics``)."""
    if flux not in FLUXES:
        raise ValueError(f"flux must be one of {FLUXES}")
    ec = flux == "ec_roe"
    N, NP = mesh.N, mesh.NP
    D = diff_matrix(N)
    _, w = lgl(N)
    P = primitives(U, gas)
    grad = lift(U, mesh, gas) if viscous else None
    Ut = [torch.zeros_like(U[0]) for _ in range(5)]
    for d in range(3):
        ea, na = ELEM_AXIS[d], NODE_AXIS[d]
        s = mesh.scale(d).to(U.dtype)

        # volume integral: two-point flux differencing along the d-lines
        Pi, Pm = _prim_line(P, na, -2), _prim_line(P, na, -1)
        fsharp = ec_flux(Pi, Pm, d, gas) if ec else kg_flux(Pi, Pm, d)
        Dd = D.to(U.dtype)
        vol_c = [(2.0 * (Dd * f).sum(-1)).movedim(-1, na) for f in fsharp]

        fc = euler_flux(P, d)
        if viscous:
            fv = viscous_flux(P.vel, grad, d, gas, P.T)
            vol_v = [_apply_D(f, D, na) for f in fv]
        else:
            fv = [torch.zeros_like(U[0]) for _ in range(5)]
            vol_v = fv

        # own physical flux on the element's first and last planes
        own_lo = [(fc[v] - fv[v]).select(na, 0) for v in range(5)]
        own_hi = [(fc[v] - fv[v]).select(na, N) for v in range(5)]

        # numerical flux on each element's upper face (L = own, R = upper neighbour)
        P_hi, P_lo = _prim_plane(P, na, N), _prim_plane(P, na, 0)
        P_R = _prim_roll(P_lo, -1, ea)
        U_hi = [U[v].select(na, N) for v in range(5)]
        U_R = [torch.roll(U[v].select(na, 0), -1, ea) for v in range(5)]
        Fc = roe_flux(P_hi, P_R, d, gas, central_only) if ec else \
            llf_flux(P_hi, P_R, U_hi, U_R, d, gas, central_only)
        Fv_L = [fv[v].select(na, N) for v in range(5)]
        Fv_R = [torch.roll(fv[v].select(na, 0), -1, ea) for v in range(5)]
        F_hi = [Fc[v] - 0.5 * (Fv_L[v] + Fv_R[v]) for v in range(5)]
        # the lower face of an element is the upper face of its lower neighbour
        F_lo = [torch.roll(F_hi[v], 1, ea) for v in range(5)]

        if mesh.bc[d] == WALL_MODEL:
            # slip, adiabatic wall: pressure-only convective flux; viscous flux
            # with the modelled wall shear stress (sign: the stress on the fluid
            # below an upper wall is the negative), the own normal viscous stress,
            # and no energy flux (adiabatic, stationary wall)
            from .wallmodel import wall_stress_field
            tau = torch.as_tensor(wall_stress_field(U, mesh, gas, mesh.wm_node, gas.mu_of))
            wall_index = [dd for dd in range(3) if mesh.bc[dd] != "periodic"]
            base = 0
            for dd in wall_index:
                if dd == d:
                    break
                others = [c for c in range(3) if c != dd]
                base += 2 * mesh.nelem[others[0]] * mesh.nelem[others[1]]
            others = [c for c in range(3) if c != d]
            na_e, nb_e = mesh.nelem[others[0]], mesh.nelem[others[1]]
            for plane_P, idx, F, last in ((P_lo, 0, F_lo, False), (P_hi, N, F_hi, True)):
                side = 1 if last else 0
                # (faces, 3, NP, NP) of this wall, face index = ea + na_e eb, node (a, b)
                t = tau[base + side * na_e * nb_e: base + (side + 1) * na_e * nb_e].reshape(nb_e, na_e, 3, NP, NP)
                sgn = -1.0 if last else 1.0
                fwc = wall_convective_flux(plane_P, d)
                if viscous:
                    g_plane = [[grad[c][b].select(na, idx) for b in range(3)] for c in range(4)]
                    fvo = viscous_flux(plane_P.vel, g_plane, d, gas, plane_P.T)
                fwv = [torch.zeros_like(plane_P.p) for _ in range(5)]
                for c in range(3):
                    if not viscous:
                        continue
                    if c == d:
                        fwv[1 + c] = fvo[1 + c]
                    else:
                        fwv[1 + c] = sgn * _wall_plane(t[:, :, c], plane_P.p, d, ea)
                mask = _end_mask(plane_P.p, ea, last)
                for v in range(5):
                    F[v] = torch.where(mask, fwc[v] - fwv[v], F[v])
        if mesh.bc[d] == WALL:
            zero = torch.zeros_like(U[0])
            for plane_P, idx, F, last in ((P_lo, 0, F_lo, False), (P_hi, N, F_hi, True)):
                g_plane = [[grad[c][b].select(na, idx) for b in range(3)] for c in range(4)] \
                    if viscous else None
                fwc = wall_convective_flux(plane_P, d)
                if viscous:
                    zv = zero.select(na, idx)
                    fwv = viscous_flux((zv, zv, zv), g_plane, d, gas, plane_P.T)
                else:
                    fwv = [torch.zeros_like(plane_P.p)] * 5
                mask = _end_mask(plane_P.p, ea, last)
                for v in range(5):
                    F[v] = torch.where(mask, fwc[v] - fwv[v], F[v])

        for v in range(5):
            surf = (_at_node(F_hi[v] - own_hi[v], na, N, NP) / w[N]
                    - _at_node(F_lo[v] - own_lo[v], na, 0, NP) / w[0])
            Ut[v] = Ut[v] - s * (vol_c[v] - vol_v[v] + surf)
    out = torch.stack(Ut)
    if source is not None:
        out = out + source
    return out


# ---------------------------------------------------------------------- RK

def lsrk(L, U, dt: float, nsteps: int = 1, t0: float = 0.0):
    """Five-stage low-storage RK: for each stage G <- A_s G + dt L(U, t_s); U <- U + B_s G."""
    t = t0
    for _ in range(nsteps):
        G = torch.zeros_like(U)
        for s in range(5):
            G = RK_A[s] * G + dt * L(U, t + RK_C[s] * dt)
            U = U + RK_B[s] * G
        t = t + dt
    return U


def rk_step(U: torch.Tensor, mesh: Mesh, gas: Gas, dt: float, nsteps: int = 1,
            *, t0: float = 0.0, source_fn=None, **opts) -> torch.Tensor:
    """Advance U by nsteps RK steps of the DGSEM operator (optional source S(t))."""
    def L(V, t):
        src = source_fn(t) if source_fn is not None else None
        return rhs(V, mesh, gas, source=src, **opts)
    return lsrk(L, U, dt, nsteps, t0)


# ----------------------------------------------------------------- objective

def kinetic_energy(U: torch.Tensor, mesh: Mesh) -> torch.Tensor:
    """Volume-averaged kinetic energy sum(wJ |m|^2/(2 rho)) / sum(wJ)."""
    wq = mesh.quadrature_weights().to(U.dtype)
    ke = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / U[0]
    return (wq * ke).sum() / wq.sum()
