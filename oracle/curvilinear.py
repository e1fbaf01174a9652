"""Split-form DGSEM on curvilinear hexahedra (test infrastructure only).

The paper's production meshes are curved hexahedra (Sec. 4: the Rotor 67
blade passage); it states no formulas for the curved-element operator.  This
module writes the standard curvilinear split-form DGSEM from its published
definitions, in the notation of the Cartesian operator (``dgsem``):

* geometry: element e maps the reference cube [-1, 1]^3 to physical space by
  the degree-N interpolant of its node coordinates X at the LGL nodes
  (isoparametric); the connectivity is that of the structured tensor mesh
  (neighbours ex +- 1, ey +- 1, ez +- 1); each direction periodic or closed
  at both ends by an isothermal no-slip wall;
* metric terms (reading: Kopriva's conservative curl form, which makes the
  discrete metric identities sum_i d/dxi^i (J a^i_n) = 0 hold and gives both
  elements of a face the same normal):
      J a^i_n = -1/2 [ curl_xi ( X_l grad_xi X_m - X_m grad_xi X_l ) ]_i,
      (n, m, l) cyclic over (x, y, z), every xi-derivative the collocation
      derivative D of the nodal product; the form is invariant under a
      translation of X, and it is evaluated (reading) with each element's
      coordinates taken relative to its first node, so that its rounding is
      that of the element's size rather than of the coordinates' magnitude;
  J = det(dX_n / dxi^j) with dX/dxi from D (reading);
* lifting (BR1, strong form; reading: chain rule with the node's own metric):
      J grad q = sum_i J a^i ( sum_m D_im q_m + delta_iN (q*_R - q_N) / w_N
                                            - delta_i0 (q*_L - q_0) / w_0 ),
  q* the mean of the two sides' primitives at a shared face node, and
  (0, 0, 0, T_wall) at a wall;
* right-hand side (strong form):
      J Ut = - sum_i ( 2 sum_m D_im F#^i(U_a, U_m) - sum_m D_im Fv^i_m
                       + delta_iN ((F* - Fv*)_R - (F^i - Fv^i)(U_N)) / w_N
                       - delta_i0 ((F* - Fv*)_L - (F^i - Fv^i)(U_0)) / w_0 ),
  along each xi^i line, with
    - the contravariant Kennedy-Gruber two-point flux with averaged metrics
      F#^i(A, B) = sum_d f#_d(A, B) (J a^i_d(A) + J a^i_d(B)) / 2;
    - contravariant physical fluxes F^i = sum_d f_d J a^i_d and
      Fv^i = sum_d f_v,d J a^i_d at each node (own metrics);
    - the surface flux across a xi^i face, computed once per face with the
      normal vector s = J a^i of the element below the face at the face node
      (pointing towards +xi^i; reading: one normal per face, so the flux
      leaving one element enters the other exactly even where the two
      elements' face nodes differ in rounding, as at a periodic seam): local
      Lax-Friedrichs
      F* = sum_d f#_d(L, R) s_d - lambda/2 |s| (U_R - U_L),
      lambda = max(|u_L . n| + c_L, |u_R . n| + c_R), n = s / |s|;
      BR1 central viscous flux Fv* = (Fv^i(L) + Fv^i(R)) / 2;
    - at a wall face, with the own face node's normal s: the pressure-only
      convective flux (0, p s, 0) and the viscous flux contracted with s for
      zero velocity and the interior gradients (the Cartesian wall of
      ``physics`` with e_d replaced by s).
With ``flux = "ec_roe"`` (the paper's production pair, Sec. 4) the volume flux
is Chandrashekar's flux contracted with the averaged metric terms,
sum_d f#EC_d(A, B) (J a^i_d(A) + J a^i_d(B)) / 2, and the surface flux is
Roe's flux across the face normal n = s / |s| scaled by |s|:
F* = sum_d f#EC_d(L, R) s_d - |s| / 2 sum_k |lambda_k| alpha_k r_k, with the
waves of Roe's linearisation along n (acoustic u~.n -+ a~, entropy and shear
u~.n, the shear jump being the tangential part [[u]] - ([[u]].n) n) and the
Harten-Hyman correction of the acoustic waves; walls keep the pressure-only
flux.
On an affine box the metric terms are J a^i = J s_i e_i and everything above
reduces to the Cartesian operator.  ``metric_form = "cross"`` computes
J a^i = dX/dxi^j x dX/dxi^k directly instead: a negative control whose
metric identities hold only to truncation error, so free streams are not
preserved on curved elements.
"""

from __future__ import annotations

from dataclasses import dataclass

import torch

from .basis import diff_matrix, lgl
from .dgsem import _apply_D, _at_node, _end_mask, _prim_line, _prim_plane, _prim_roll, lsrk
from .mesh import ELEM_AXIS, NODE_AXIS, PERIODIC, WALL
from .physics import (FLUXES, Gas, ec_flux, euler_flux, harten_hyman_abs, kg_flux, primitives, rabs, rmax,
                      viscous_flux)

__all__ = ["CurvMesh", "metrics", "lift", "rhs", "rk_step", "llf_flux_metric", "roe_waves_normal",
           "roe_flux_metric"]


@dataclass
class CurvMesh:
    N: int
    X: torch.Tensor          # (3, nz, ny, nx, N+1, N+1, N+1) node coordinates
    metric_form: str = "curl"
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    T_wall: float = 1.0

    def __post_init__(self):
        for b in self.bc:
            if b not in (PERIODIC, WALL):
                raise ValueError(f"curved elements take periodic or wall ends, not {b!r}")
        self.X = torch.as_tensor(self.X, dtype=torch.float64)
        if self.X.dim() != 7 or self.X.shape[0] != 3 or any(s != self.N + 1 for s in self.X.shape[4:]):
            raise ValueError("X must be shaped (3, nz, ny, nx, N+1, N+1, N+1)")
        if self.metric_form not in ("curl", "cross"):
            raise ValueError("metric_form must be 'curl' or 'cross'")

    @property
    def NP(self) -> int:
        return self.N + 1

    @property
    def shape(self):
        return tuple(self.X.shape[1:])

    @property
    def nelem(self):
        nz, ny, nx = self.X.shape[1:4]
        return (nx, ny, nz)

    @property
    def n_dof(self) -> int:
        return self.X[0].numel()

    def quadrature_weights(self) -> torch.Tensor:
        """w_i w_j w_k J at every node (J from ``metrics``)."""
        _, w = lgl(self.N)
        w = w.to(torch.float64)
        wk = w.reshape(-1, 1, 1) * w.reshape(1, -1, 1) * w.reshape(1, 1, -1)
        _, J = metrics(self)
        return wk * J


def metrics(mesh: CurvMesh):
    """(Ja, J): Ja[i][n] = J a^i_n (i: reference direction, n: physical
    component), each a nodal field; J the Jacobian determinant."""
    D = diff_matrix(mesh.N)
    X = mesh.X - mesh.X[..., :1, :1, :1]  # relative to each element's node (0, 0, 0)
    dX = [[_apply_D(X[n], D, NODE_AXIS[j]) for j in range(3)] for n in range(3)]  # dX[n][j] = dX_n/dxi^j
    J = (dX[0][0] * (dX[1][1] * dX[2][2] - dX[1][2] * dX[2][1])
         - dX[0][1] * (dX[1][0] * dX[2][2] - dX[1][2] * dX[2][0])
         + dX[0][2] * (dX[1][0] * dX[2][1] - dX[1][1] * dX[2][0]))
    Ja = [[None] * 3 for _ in range(3)]
    for n in range(3):
        m, l = (n + 1) % 3, (n + 2) % 3
        if mesh.metric_form == "curl":
            V = [X[l] * dX[m][j] - X[m] * dX[l][j] for j in range(3)]
            for i in range(3):
                a, b = (i + 1) % 3, (i + 2) % 3
                Ja[i][n] = -0.5 * (_apply_D(V[b], D, NODE_AXIS[a]) - _apply_D(V[a], D, NODE_AXIS[b]))
        else:
            for i in range(3):
                a, b = (i + 1) % 3, (i + 2) % 3
                Ja[i][n] = dX[m][a] * dX[l][b] - dX[l][a] * dX[m][b]
    return Ja, J


def lift(U: torch.Tensor, mesh: CurvMesh, gas: Gas, geo=None):
    """BR1 lifted gradients grad[q][d] of q in (u, v, w, T) on the curved mesh."""
    N, NP = mesh.N, mesh.NP
    D = diff_matrix(N)
    _, w = lgl(N)
    Ja, J = metrics(mesh) if geo is None else geo
    P = primitives(U, gas)
    q = [P.vel[0], P.vel[1], P.vel[2], P.T]
    gxi = [[None] * 3 for _ in range(4)]  # reference-space gradients with the lifting terms
    for i in range(3):
        ea, na = ELEM_AXIS[i], NODE_AXIS[i]
        for c in range(4):
            vol = _apply_D(q[c], D, na)
            lo, hi = q[c].select(na, 0), q[c].select(na, N)
            star_lo = 0.5 * (lo + torch.roll(hi, 1, ea))
            star_hi = 0.5 * (hi + torch.roll(lo, -1, ea))
            if mesh.bc[i] == WALL:
                wv = torch.full_like(lo, (0.0, 0.0, 0.0, mesh.T_wall)[c])
                star_lo = torch.where(_end_mask(lo, ea, last=False), wv, star_lo)
                star_hi = torch.where(_end_mask(hi, ea, last=True), wv, star_hi)
            surf = (_at_node(star_hi - hi, na, N, NP) / w[N]
                    - _at_node(star_lo - lo, na, 0, NP) / w[0])
            gxi[c][i] = vol + surf
    return [[(Ja[0][d] * gxi[c][0] + Ja[1][d] * gxi[c][1] + Ja[2][d] * gxi[c][2]) / J for d in range(3)]
            for c in range(4)]


def llf_flux_metric(L, R, UL, UR, s, gas: Gas, central_only: bool = False):
    """Local Lax-Friedrichs flux across a face with normal vector s (not unit):
    sum_d f#_d(L, R) s_d - lambda/2 |s| (U_R - U_L)."""
    f = [sum(kg_flux(L, R, d)[v] * s[d] for d in range(3)) for v in range(5)]
    if central_only:
        return f
    smag = torch.sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2])
    un_L = (L.vel[0] * s[0] + L.vel[1] * s[1] + L.vel[2] * s[2]) / smag
    un_R = (R.vel[0] * s[0] + R.vel[1] * s[1] + R.vel[2] * s[2]) / smag
    c_L = torch.sqrt(gas.gamma * L.p / L.rho)
    c_R = torch.sqrt(gas.gamma * R.p / R.rho)
    lam = rmax(rabs(un_L) + c_L, rabs(un_R) + c_R)
    return [f[v] - 0.5 * lam * smag * (UR[v] - UL[v]) for v in range(5)]


def roe_waves_normal(L, R, n, gas: Gas):
    """Roe's wave decomposition across a face with unit normal n (L on the side
    n points away from): (lambda, alpha, r) lists with
    U_R - U_L = sum_k alpha_k r_k.  Shear waves are one entry with alpha = 1
    and r = rho~ (0, [[u_t]], u~ . [[u_t]]), [[u_t]] = [[u]] - ([[u]] . n) n."""
    g = gas.gamma
    sl, sr = torch.sqrt(L.rho), torch.sqrt(R.rho)
    wl, wr = sl / (sl + sr), sr / (sl + sr)
    u = [wl * L.vel[c] + wr * R.vel[c] for c in range(3)]
    H = wl * (L.E + L.p) / L.rho + wr * (R.E + R.p) / R.rho
    q2 = sum(u[c] * u[c] for c in range(3))
    a2 = (g - 1.0) * (H - 0.5 * q2)
    a = torch.sqrt(a2)
    rho = sl * sr
    un = sum(u[c] * n[c] for c in range(3))
    drho = R.rho - L.rho
    dp = R.p - L.p
    du = [R.vel[c] - L.vel[c] for c in range(3)]
    dun = sum(du[c] * n[c] for c in range(3))
    dut = [du[c] - dun * n[c] for c in range(3)]
    one = torch.ones_like(a)
    zero = torch.zeros_like(a)
    lam = [un - a, un, un, un + a]
    alpha = [(dp - rho * a * dun) / (2.0 * a2), drho - dp / a2, one, (dp + rho * a * dun) / (2.0 * a2)]
    r = [[one] + [u[c] - a * n[c] for c in range(3)] + [H - un * a],
         [one] + u + [0.5 * q2],
         [zero] + [rho * dut[c] for c in range(3)] + [rho * sum(u[c] * dut[c] for c in range(3))],
         [one] + [u[c] + a * n[c] for c in range(3)] + [H + un * a]]
    return lam, alpha, r


def roe_flux_metric(L, R, s, gas: Gas, central_only: bool = False):
    """Roe's flux with the Harten-Hyman correction across a face with normal
    vector s (not unit): sum_d f#EC_d(L, R) s_d - |s|/2 sum_k |lambda_k| alpha_k r_k."""
    f = [sum(ec_flux(L, R, d, gas)[v] * s[d] for d in range(3)) for v in range(5)]
    if central_only:
        return f
    smag = torch.sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2])
    n = [s[c] / smag for c in range(3)]
    lam, alpha, r = roe_waves_normal(L, R, n, gas)
    absl = [torch.abs(x) for x in lam]
    unL = sum(L.vel[c] * n[c] for c in range(3))
    unR = sum(R.vel[c] * n[c] for c in range(3))
    cL, cR = L.c(gas), R.c(gas)
    absl[0] = harten_hyman_abs(lam[0], unL - cL, unR - cR)
    absl[3] = harten_hyman_abs(lam[3], unL + cL, unR + cR)
    return [f[v] - 0.5 * smag * sum(absl[k] * alpha[k] * r[k][v] for k in range(4)) for v in range(5)]


def rhs(U: torch.Tensor, mesh: CurvMesh, gas: Gas, *, viscous: bool = True,
        central_only: bool = False, source=None, flux: str = "kg_llf") -> torch.Tensor:
    """L(U) of the curvilinear split-form DGSEM (module docstring)."""
    if flux not in FLUXES:
        raise ValueError(f"flux must be one of {FLUXES}")
    ec = flux == "ec_roe"
    N, NP = mesh.N, mesh.NP
    D = diff_matrix(N).to(U.dtype)
    _, w = lgl(N)
    Ja, J = metrics(mesh)
    P = primitives(U, gas)
    grad = lift(U, mesh, gas, (Ja, J)) if viscous else None
    fv_d = [viscous_flux(P.vel, grad, d, gas, P.T) for d in range(3)] if viscous else None
    fc_d = [euler_flux(P, d) for d in range(3)]
    acc = [torch.zeros_like(U[0]) for _ in range(5)]
    for i in range(3):
        ea, na = ELEM_AXIS[i], NODE_AXIS[i]
        Jai = Ja[i]

        # volume: contravariant two-point flux with averaged metrics
        Pa, Pm = _prim_line(P, na, -2), _prim_line(P, na, -1)
        Ma = [Jai[d].movedim(na, -1).unsqueeze(-1) for d in range(3)]
        Mm = [Jai[d].movedim(na, -1).unsqueeze(-2) for d in range(3)]
        fsharp = [ec_flux(Pa, Pm, d, gas) if ec else kg_flux(Pa, Pm, d) for d in range(3)]
        F2 = [sum(fsharp[d][v] * (0.5 * (Ma[d] + Mm[d])) for d in range(3)) for v in range(5)]
        vol_c = [(2.0 * (D * F2[v]).sum(-1)).movedim(-1, na) for v in range(5)]

        # contravariant physical fluxes at the nodes (own metrics)
        Fc = [sum(fc_d[d][v] * Jai[d] for d in range(3)) for v in range(5)]
        if viscous:
            Fv = [sum(fv_d[d][v] * Jai[d] for d in range(3)) for v in range(5)]
            vol_v = [_apply_D(Fv[v], D, na) for v in range(5)]
        else:
            Fv = [torch.zeros_like(U[0]) for _ in range(5)]
            vol_v = Fv
        own_lo = [(Fc[v] - Fv[v]).select(na, 0) for v in range(5)]
        own_hi = [(Fc[v] - Fv[v]).select(na, N) for v in range(5)]

        # numerical flux on each element's upper face (L = own, R = upper neighbour)
        s = [Jai[d].select(na, N) for d in range(3)]
        P_hi = _prim_plane(P, na, N)
        P_R = _prim_roll(_prim_plane(P, na, 0), -1, ea)
        U_hi = [U[v].select(na, N) for v in range(5)]
        U_R = [torch.roll(U[v].select(na, 0), -1, ea) for v in range(5)]
        Fs = roe_flux_metric(P_hi, P_R, s, gas, central_only) if ec else \
            llf_flux_metric(P_hi, P_R, U_hi, U_R, s, gas, central_only)
        Fv_L = [Fv[v].select(na, N) for v in range(5)]
        Fv_R = [torch.roll(Fv[v].select(na, 0), -1, ea) for v in range(5)]
        F_hi = [Fs[v] - 0.5 * (Fv_L[v] + Fv_R[v]) for v in range(5)]
        F_lo = [torch.roll(F_hi[v], 1, ea) for v in range(5)]
        if mesh.bc[i] == WALL:
            for idx, F, last in ((0, F_lo, False), (N, F_hi, True)):
                Pw = _prim_plane(P, na, idx)
                sw = [Jai[d].select(na, idx) for d in range(3)]
                zero = torch.zeros_like(Pw.p)
                fw = [zero] + [Pw.p * sw[a] for a in range(3)] + [zero]
                if viscous:
                    g_plane = [[grad[c][b].select(na, idx) for b in range(3)] for c in range(4)]
                    fvw = [viscous_flux((zero, zero, zero), g_plane, d, gas, Pw.T) for d in range(3)]
                    fw = [fw[v] - sum(fvw[d][v] * sw[d] for d in range(3)) for v in range(5)]
                mask = _end_mask(Pw.p, ea, last)
                for v in range(5):
                    F[v] = torch.where(mask, fw[v], F[v])
        for v in range(5):
            surf = (_at_node(F_hi[v] - own_hi[v], na, N, NP) / w[N]
                    - _at_node(F_lo[v] - own_lo[v], na, 0, NP) / w[0])
            acc[v] = acc[v] + vol_c[v] - vol_v[v] + surf
    out = torch.stack([-a / J for a in acc])
    if source is not None:
        out = out + source
    return out


def rk_step(U: torch.Tensor, mesh: CurvMesh, gas: Gas, dt: float, nsteps: int = 1, *,
            t0: float = 0.0, source_fn=None, **opts) -> torch.Tensor:
    """Advance U by nsteps steps of the five-stage low-storage RK scheme."""
    def L(V, t):
        src = source_fn(t) if source_fn is not None else None
        return rhs(V, mesh, gas, source=src, **opts)
    return lsrk(L, U, dt, nsteps, t0)
