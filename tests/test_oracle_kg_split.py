"""Pin of the Kennedy-Gruber flux's mass and energy terms by the split form it
stands for (CPU only).

Split-form DG on LGL nodes (paper Sec. 2.2) differentiates a two-point flux
along each line: 2 sum_m D_im f#(U_i, U_m).  With a derivative matrix whose
rows sum to zero, the means of products expand into discrete product rules
(the flux-differencing identities of Gassner, Winters and Kopriva):

  2 sum_m D_im {{a}}        = (D a)_i
  2 sum_m D_im {{a}}{{b}}   = ( D(ab) + a Db + b Da )_i / 2
  2 sum_m D_im {{a}}{{b}}{{c}}
        = ( D(abc) + a D(bc) + b D(ac) + c D(ab) + bc Da + ac Db + ab Dc )_i / 4

The Kennedy-Gruber split of the Euler fluxes is, component by component,
  mass      {{rho}}{{u_d}}                    -> the (rho, u_d) double product rule,
  momentum  {{rho}}{{u_d}}{{u_a}} + {{p}} e_d  -> the (rho, u_d, u_a) triple rule + D p,
  energy    {{rho}}{{u_d}}{{e}} + {{p}}{{u_d}} -> the (rho, u_d, e) triple rule
                                                + the (p, u_d) double rule, e = E / rho.
The right-hand sides are built here from nodal products and plain matrix-vector
products with D, independently of the oracle's two-point flux, which supplies
the left-hand sides.  Plausible misreadings of the flux -- {{rho u_d}} as the
mass flux, {{E}}{{u_d}} in the energy, or the total-enthalpy form
{{rho}}{{u_d}}{{H}} -- give different discrete operators; the negative controls
check that the identity tells them apart.
"""

import numpy as np
import pytest
import torch

from oracle import physics as ph
from oracle.basis import diff_matrix
from oracle.physics import Gas

GAMMA = 1.4


def _line_state(N, rng, n_lines=16):
    """Random primitive data on n_lines lines of N+1 nodes: (n_lines, N+1) each."""
    shape = (n_lines, N + 1)
    rho = 1.0 + 0.3 * rng.uniform(-1, 1, shape)
    vel = tuple(rng.uniform(-1, 1, shape) for _ in range(3))
    p = 1.0 + 0.3 * rng.uniform(-1, 1, shape)
    E = p / (GAMMA - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    U = torch.tensor(np.stack([rho, rho * vel[0], rho * vel[1], rho * vel[2], E]))
    return ph.primitives(U, Gas(gamma=GAMMA, R=1.0, mu=0.0, Pr=0.72))


def _pairs(P):
    """(own node i, line node m) views: values broadcast to (n_lines, N+1, N+1)."""
    def own(x):
        return x.unsqueeze(-1).expand(*x.shape, x.shape[-1])

    def line(x):
        return x.unsqueeze(-2).expand(*x.shape[:-1], x.shape[-1], x.shape[-1])

    Pi = ph.Prim(own(P.rho), tuple(own(v) for v in P.vel), own(P.p), own(P.T), own(P.e), own(P.E))
    Pm = ph.Prim(line(P.rho), tuple(line(v) for v in P.vel), line(P.p), line(P.T), line(P.e),
                 line(P.E))
    return Pi, Pm


def _flux_difference(f_pairs, D):
    """2 sum_m D_im f(i, m) for a pair field (n_lines, i, m)."""
    return 2.0 * (D * f_pairs).sum(-1)


def _Dx(D, x):
    return x @ D.T


def _double(D, a, b):
    return 0.5 * (_Dx(D, a * b) + a * _Dx(D, b) + b * _Dx(D, a))


def _triple(D, a, b, c):
    return 0.25 * (_Dx(D, a * b * c) + a * _Dx(D, b * c) + b * _Dx(D, a * c) + c * _Dx(D, a * b)
                   + b * c * _Dx(D, a) + a * c * _Dx(D, b) + a * b * _Dx(D, c))


def _split_form(P, d, D):
    """The Kennedy-Gruber product-rule split of the five Euler flux divergences."""
    ud = P.vel[d]
    out = [_double(D, P.rho, ud)]
    for a in range(3):
        t = _triple(D, P.rho, ud, P.vel[a])
        if a == d:
            t = t + _Dx(D, P.p)
        out.append(t)
    out.append(_triple(D, P.rho, ud, P.e) + _double(D, P.p, ud))
    return out


def _scale(ref):
    return max(float(r.abs().max()) for r in ref)


@pytest.mark.parametrize("N", [3, 5, 7])
def test_row_sums_vanish(N):
    D = diff_matrix(N)
    assert float(D.sum(1).abs().max()) < 1e-13 * float(D.abs().max())


@pytest.mark.parametrize("N", [3, 5, 7])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_kg_flux_differencing_is_the_kennedy_gruber_split(N, d):
    rng = np.random.default_rng(100 * N + d)
    D = diff_matrix(N)
    P = _line_state(N, rng)
    Pi, Pm = _pairs(P)
    got = [_flux_difference(f, D) for f in ph.kg_flux(Pi, Pm, d)]
    want = _split_form(P, d, D)
    sc = _scale(want)
    for v in range(5):
        err = float((got[v] - want[v]).abs().max())
        assert err < 1e-13 * sc, (v, err, sc)


@pytest.mark.parametrize("N", [3, 5, 7])
def test_misread_mass_and_energy_terms_fail_the_split(N):
    """Negative controls: each variant differs from the split form by far more
    than rounding, so the identity above would catch it in the oracle."""
    d = 0
    rng = np.random.default_rng(7 + N)
    D = diff_matrix(N)
    P = _line_state(N, rng)
    Pi, Pm = _pairs(P)
    want = _split_form(P, d, D)
    sc = _scale(want)
    avg = lambda x, y: 0.5 * (x + y)  # noqa: E731
    rho_ud = lambda A: A.rho * A.vel[d]  # noqa: E731
    # {{rho u_d}} as the mass flux
    mass_cons = avg(rho_ud(Pi), rho_ud(Pm))
    # {{E}}{{u_d}} + {{p}}{{u_d}} as the energy flux
    energy_E = avg(Pi.E, Pm.E) * avg(Pi.vel[d], Pm.vel[d]) + avg(Pi.p, Pm.p) * avg(Pi.vel[d], Pm.vel[d])
    # {{rho}}{{u_d}}{{H}}, H = (E + p) / rho, as the energy flux
    H = lambda A: (A.E + A.p) / A.rho  # noqa: E731
    energy_H = avg(Pi.rho, Pm.rho) * avg(Pi.vel[d], Pm.vel[d]) * avg(H(Pi), H(Pm))
    for f, v in ((mass_cons, 0), (energy_E, 4), (energy_H, 4)):
        err = float((_flux_difference(f, D) - want[v]).abs().max())
        assert err > 1e-6 * sc, (v, err)
