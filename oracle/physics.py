"""Gas model and fluxes of the oracle (test infrastructure only).

Paper Sec. 4: the working fluid is an ideal gas and the scheme is a split-form
DG discretisation with viscous fluxes.  The default configuration uses the
readings below, each written from its published definition; the paper's own
production choices (Chandrashekar entropy-conserving volume flux, Roe/Harten
surface flux, Sutherland viscosity) are options described further down and
in the viscous-flux item:

* ideal gas:   p = (gamma - 1) (E - rho |u|^2 / 2),   T = p / (rho R),
               c = sqrt(gamma p / rho),   e = E / rho;
* Euler flux along direction d:
               f_d = (rho u_d, rho u u_d + p delta_1d, rho v u_d + p delta_2d,
                      rho w u_d + p delta_3d, (E + p) u_d);
* Kennedy-Gruber two-point volume flux, {{x}} = (x_a + x_b) / 2:
               f#_d = ({{rho}}{{u_d}}, {{rho}}{{u_d}}{{u}} + {{p}} delta_1d, ...,
                       {{rho}}{{u_d}}{{e}} + {{p}}{{u_d}});
* Newtonian/Fourier viscous flux,
  tau = mu (grad u + grad u^T - 2/3 (div u) I), kappa = mu gamma R / ((gamma-1) Pr):
               f_v,d = (0, tau_1d, tau_2d, tau_3d, u_a tau_ad + kappa dT/dx_d),
  with mu constant, or (Sec. 4 names Sutherland's law for the working fluid)
  mu(T) = mu_ref (T / T_ref)^(3/2) (T_ref + S) / (T + S), mu_ref the
  viscosity at T_ref and S Sutherland's temperature, both in the units of T;
  mu and kappa are taken at the temperature of the node whose gradients form
  the flux (at a wall: the interior face node);
* local Lax-Friedrichs (Rusanov) surface flux whose central part is the
  Kennedy-Gruber flux: F* = f#_d(U_L, U_R) - lambda/2 (U_R - U_L),
  lambda = max(|u_d,L| + c_L, |u_d,R| + c_R);
* isothermal no-slip wall: convective flux (0, p_int n, 0) with the interior
  pressure; lifting wall value (u, v, w, T) = (0, 0, 0, T_wall); viscous flux
  f_v with zero wall velocity and the interior gradients.

All functions are complex-step safe: |z| and max(a, b) take the branch chosen
by the real part (ties go to the first argument).

The paper's production scheme (Sec. 4: an entropy-conserving split form with
Chandrashekar's flux, Roe's Riemann solver with Harten's entropy correction)
is the second flux choice, written from the published definitions (real
arithmetic only; readings listed with the functions):

* logarithmic mean x_ln(a, b) = (a - b) / (ln a - ln b), x_ln(a, a) = a;
* Chandrashekar's kinetic-energy-preserving, entropy-conserving two-point flux
  with beta = rho / (2 p), {{x}} the arithmetic mean and ln the log mean:
      F_rho = rho_ln {{u_d}},
      F_m   = F_rho {{u}} + delta_d p_hat,   p_hat = {{rho}} / (2 {{beta}}),
      F_E   = F_rho (1 / (2 (gamma - 1) beta_ln) - {{|u|^2}} / 2) + {{u}} . F_m,
  which satisfies Tadmor's condition [[v]] . F = [[rho u_d]] for the entropy
  variables v of the entropy -rho s / (gamma - 1), s = ln(p rho^-gamma);
* Roe's linearisation at the Roe average (sqrt(rho) weighted u and H,
  rho~ = sqrt(rho_L rho_R), a~^2 = (gamma - 1)(H~ - |u~|^2 / 2)) as waves
  lambda_k alpha_k r_k: acoustic waves u~_d -+ a~ with
  alpha = ([[p]] -+ rho~ a~ [[u_d]]) / (2 a~^2) and r = (1, u~ -+ a~ e_d,
  H~ -+ u~_d a~); the entropy wave u~_d with alpha = [[rho]] - [[p]] / a~^2 and
  r = (1, u~, |u~|^2 / 2); the shear waves u~_d with rho~ [[u_t]] and
  r = (0, t, u~ . t) for the tangential jump;
* Harten's entropy correction (reading: the Harten-Hyman form) on the two
  acoustic waves: |lambda| is replaced by (lambda^2 + delta^2) / (2 delta) when
  |lambda| < delta, delta = max(0, lambda(Roe) - lambda(L), lambda(R) - lambda(Roe));
* surface flux (reading: the central part is the volume flux, as in the
  Lax-Friedrichs choice): F* = F_EC(U_L, U_R) - (1/2) sum_k |lambda_k| alpha_k r_k.
"""

from __future__ import annotations

from dataclasses import dataclass

import torch

__all__ = ["Gas", "primitives", "euler_flux", "kg_flux", "viscous_flux",
           "llf_flux", "wall_convective_flux", "rabs", "rmax", "ln_mean", "ec_flux",
           "entropy_variables", "roe_waves", "harten_hyman_abs", "roe_flux", "FLUXES"]

FLUXES = ("kg_llf", "ec_roe")


@dataclass(frozen=True)
class Gas:
    gamma: float = 1.4
    R: float = 1.0
    mu: float = 0.0
    Pr: float = 0.72
    sutherland: bool = False  # mu(T) by Sutherland's law, mu being its value at T_ref
    T_ref: float = 1.0
    S: float = 0.0

    @property
    def kappa(self) -> float:
        return self.mu * self.gamma * self.R / ((self.gamma - 1.0) * self.Pr)

    def mu_of(self, T):
        """Dynamic viscosity at temperature T (a number or a tensor)."""
        if not self.sutherland:
            return self.mu
        return self.mu * (T / self.T_ref) ** 1.5 * (self.T_ref + self.S) / (T + self.S)

    def kappa_of(self, T):
        """Heat conductivity mu(T) c_p / Pr at temperature T."""
        return self.mu_of(T) * self.gamma * self.R / ((self.gamma - 1.0) * self.Pr)

    @property
    def cv(self) -> float:
        return self.R / (self.gamma - 1.0)


def _re(z: torch.Tensor) -> torch.Tensor:
    return torch.real(z) if z.is_complex() else z


def rabs(z: torch.Tensor) -> torch.Tensor:
    """|z| for real z, and its analytic continuation sign(Re z) z for complex z."""
    return z * torch.sign(_re(z))


def rmax(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """max(a, b) choosing by real part; ties go to a."""
    return torch.where(_re(a) >= _re(b), a, b)


class Prim:
    """Primitive variables at a set of nodes (all tensors of one shape)."""

    __slots__ = ("rho", "vel", "p", "T", "e", "E")

    def __init__(self, rho, vel, p, T, e, E):
        self.rho, self.vel, self.p, self.T, self.e, self.E = rho, vel, p, T, e, E

    def c(self, gas: Gas):
        return torch.sqrt(gas.gamma * self.p / self.rho)


def primitives(U, gas: Gas) -> Prim:
    """Ideal-gas recovery of (rho, u, v, w, p, T, e) from U = (rho, rho u, rho v, rho w, E)."""
    rho, mx, my, mz, E = U[0], U[1], U[2], U[3], U[4]
    u, v, w = mx / rho, my / rho, mz / rho
    p = (gas.gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w))
    T = p / (rho * gas.R)
    e = E / rho
    return Prim(rho, (u, v, w), p, T, e, E)


def conservative(P: Prim):
    rho = P.rho
    return [rho, rho * P.vel[0], rho * P.vel[1], rho * P.vel[2], P.E]


def euler_flux(P: Prim, d: int):
    ud = P.vel[d]
    f = [P.rho * ud]
    for a in range(3):
        fa = P.rho * P.vel[a] * ud
        if a == d:
            fa = fa + P.p
        f.append(fa)
    f.append((P.E + P.p) * ud)
    return f


def kg_flux(A: Prim, B: Prim, d: int):
    """Kennedy-Gruber two-point flux f#_d(A, B) (symmetric in A, B)."""
    avg = lambda x, y: 0.5 * (x + y)  # noqa: E731
    rho = avg(A.rho, B.rho)
    ud = avg(A.vel[d], B.vel[d])
    p = avg(A.p, B.p)
    e = avg(A.e, B.e)
    mass = rho * ud
    f = [mass]
    for a in range(3):
        fa = mass * avg(A.vel[a], B.vel[a])
        if a == d:
            fa = fa + p
        f.append(fa)
    f.append(mass * e + p * ud)
    return f


def viscous_flux(vel, grad, d: int, gas: Gas, T=None):
    """f_v,d for velocity vel = (u, v, w) and grad[q][b] = d q / d x_b, q in (u, v, w, T);
    T (needed with Sutherland's law) is the temperature at which mu and kappa are taken."""
    if gas.sutherland and T is None:
        raise ValueError("Sutherland's law needs the temperature")
    mu = gas.mu_of(T)
    kappa = gas.kappa_of(T)
    div = grad[0][0] + grad[1][1] + grad[2][2]
    tau = []
    for a in range(3):
        t = mu * (grad[a][d] + grad[d][a])
        if a == d:
            t = t - (2.0 / 3.0) * mu * div
        tau.append(t)
    energy = vel[0] * tau[0] + vel[1] * tau[1] + vel[2] * tau[2] + kappa * grad[3][d]
    zero = torch.zeros_like(tau[0])
    return [zero, tau[0], tau[1], tau[2], energy]


def llf_flux(L: Prim, R: Prim, UL, UR, d: int, gas: Gas, central_only: bool = False):
    """Local Lax-Friedrichs flux with the Kennedy-Gruber flux as its central part."""
    f = kg_flux(L, R, d)
    if central_only:
        return f
    lam = rmax(rabs(L.vel[d]) + L.c(gas), rabs(R.vel[d]) + R.c(gas))
    return [f[v] - 0.5 * lam * (UR[v] - UL[v]) for v in range(5)]


def wall_convective_flux(P: Prim, d: int):
    """Convective flux through an impermeable wall: only the interior pressure acts."""
    zero = torch.zeros_like(P.p)
    f = [zero]
    for a in range(3):
        f.append(P.p if a == d else zero)
    f.append(zero)
    return f


# ------------------------------------------------------- entropy-conserving / Roe

def ln_mean(a, b):
    """Logarithmic mean of positive a, b.  With f = (a - b) / (a + b) the identity
    ln(a / b) = 2 atanh(f) gives x_ln = (a + b) / (2 F), F = atanh(f) / f; for
    f^2 < 1e-4 F is its Taylor series 1 + f^2/3 + f^4/5 + f^6/7 (the first
    dropped term, f^8/9, is below 1.2e-17)."""
    s = a + b
    f = (a - b) / s
    u = f * f
    small = _re(u) < 1e-4
    fs = torch.where(small, torch.ones_like(f), f)
    F = torch.where(small, 1.0 + u / 3.0 + u * u / 5.0 + u * u * u / 7.0, torch.atanh(fs) / fs)
    return s / (2.0 * F)


def _beta(P: Prim):
    return P.rho / (2.0 * P.p)


def ec_flux(A: Prim, B: Prim, d: int, gas: Gas):
    """Chandrashekar's entropy-conserving two-point flux f#_d(A, B) (symmetric)."""
    avg = lambda x, y: 0.5 * (x + y)  # noqa: E731
    ba, bb = _beta(A), _beta(B)
    rho_ln = ln_mean(A.rho, B.rho)
    beta_ln = ln_mean(ba, bb)
    p_hat = avg(A.rho, B.rho) / (2.0 * avg(ba, bb))
    u = [avg(A.vel[c], B.vel[c]) for c in range(3)]
    q2 = avg(sum(A.vel[c] * A.vel[c] for c in range(3)), sum(B.vel[c] * B.vel[c] for c in range(3)))
    F1 = rho_ln * u[d]
    Fm = [F1 * u[c] + (p_hat if c == d else 0.0) for c in range(3)]
    F5 = F1 * (1.0 / (2.0 * (gas.gamma - 1.0) * beta_ln) - 0.5 * q2) + sum(Fm[c] * u[c] for c in range(3))
    return [F1] + Fm + [F5]


def entropy_variables(P: Prim, gas: Gas):
    """v = dU/dU of the entropy -rho s / (gamma - 1), s = ln(p rho^-gamma)."""
    s = torch.log(P.p) - gas.gamma * torch.log(P.rho)
    beta = _beta(P)
    q2 = sum(P.vel[c] * P.vel[c] for c in range(3))
    return [(gas.gamma - s) / (gas.gamma - 1.0) - beta * q2] + \
        [2.0 * beta * P.vel[c] for c in range(3)] + [-2.0 * beta]


def roe_waves(L: Prim, R: Prim, d: int, gas: Gas):
    """Roe's wave decomposition across a face with normal e_d, L = lower side:
    (lambda, alpha, r) lists with U_R - U_L = sum_k alpha_k r_k and
    f_d(U_R) - f_d(U_L) = sum_k lambda_k alpha_k r_k.  Shear waves are one
    entry with alpha = 1 and r = rho~ (0, [[u_t]], u~ . [[u_t]])."""
    g = gas.gamma
    sl, sr = torch.sqrt(L.rho), torch.sqrt(R.rho)
    wl, wr = sl / (sl + sr), sr / (sl + sr)
    u = [wl * L.vel[c] + wr * R.vel[c] for c in range(3)]
    H = wl * (L.E + L.p) / L.rho + wr * (R.E + R.p) / R.rho
    q2 = sum(u[c] * u[c] for c in range(3))
    a2 = (g - 1.0) * (H - 0.5 * q2)
    a = torch.sqrt(a2)
    rho = sl * sr
    un = u[d]
    drho = R.rho - L.rho
    dp = R.p - L.p
    du = [R.vel[c] - L.vel[c] for c in range(3)]
    dut = [du[c] - (du[d] if c == d else 0.0) for c in range(3)]
    one = torch.ones_like(a)
    zero = torch.zeros_like(a)

    def vec(first, vel, last):
        return [first] + vel + [last]

    lam = [un - a, un, un, un + a]
    alpha = [(dp - rho * a * du[d]) / (2.0 * a2), drho - dp / a2, one, (dp + rho * a * du[d]) / (2.0 * a2)]
    r = [vec(one, [u[c] - (a if c == d else 0.0) for c in range(3)], H - un * a),
         vec(one, u, 0.5 * q2),
         vec(zero, [rho * dut[c] for c in range(3)], rho * sum(u[c] * dut[c] for c in range(3))),
         vec(one, [u[c] + (a if c == d else 0.0) for c in range(3)], H + un * a)]
    return lam, alpha, r


def harten_hyman_abs(lam, lam_L, lam_R):
    """|lambda| with the entropy correction: (lambda^2 + delta^2) / (2 delta) where
    |lambda| < delta = max(0, lambda - lambda_L, lambda_R - lambda).  Comparisons
    take the real part and |.| is sign(Re z) z, so complex steps pass through."""
    delta = rmax(rmax(lam - lam_L, lam_R - lam), torch.zeros_like(lam))
    small = _re(rabs(lam)) < _re(delta)
    dsafe = torch.where(small, delta, torch.ones_like(delta))
    return torch.where(small, (lam * lam + delta * delta) / (2.0 * dsafe), rabs(lam))


def roe_flux(L: Prim, R: Prim, d: int, gas: Gas, central_only: bool = False, entropy_fix: bool = True):
    """F* = f#_EC(L, R) - (1/2) sum_k |lambda_k| alpha_k r_k (Roe dissipation with
    the Harten-Hyman correction of the acoustic waves)."""
    f = ec_flux(L, R, d, gas)
    if central_only:
        return f
    lam, alpha, r = roe_waves(L, R, d, gas)
    absl = [rabs(x) for x in lam]
    if entropy_fix:
        cL, cR = L.c(gas), R.c(gas)
        absl[0] = harten_hyman_abs(lam[0], L.vel[d] - cL, R.vel[d] - cR)
        absl[3] = harten_hyman_abs(lam[3], L.vel[d] + cL, R.vel[d] + cR)
    return [f[v] - 0.5 * sum(absl[k] * alpha[k] * r[k][v] for k in range(4)) for v in range(5)]
