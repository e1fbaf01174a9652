"""Pins of the oracle's LGL basis and low-storage RK coefficients (CPU only).

Every check compares against something other than the oracle itself: closed
forms, a printed table, exact polynomial calculus, or the classical RK order
conditions.
"""

import math
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle.basis import diff_matrix, lagrange_eval, lgl
from oracle.dgsem import RK_A, RK_B, RK_C, lsrk

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ LGL nodes

CLOSED = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", sorted(CLOSED))
def test_lgl_closed_forms(N):
    x, w = lgl(N)
    xr, wr = CLOSED[N]
    assert np.allclose(x.numpy(), xr, atol=1e-15, rtol=0)
    assert np.allclose(w.numpy(), wr, atol=1e-15, rtol=0)


def test_lgl_against_printed_lobatto_table():
    rows = [line.split() for line in open(os.path.join(GOLDEN, "lobatto_abramowitz_stegun_25_6.txt"))
            if line.strip() and not line.startswith("#")]
    for n, xs, ws in rows:
        N = int(n) - 1
        x, w = lgl(N)
        xv, wv = float(xs), float(ws)
        k = int(np.argmin(np.abs(x.numpy() - xv)))
        assert abs(x[k].item() - xv) < 2e-15 + 1e-15
        assert abs(w[k].item() - wv) < 1e-14
        k2 = int(np.argmin(np.abs(x.numpy() + xv)))  # symmetric partner
        assert abs(x[k2].item() + xv) < 2e-15 and abs(w[k2].item() - wv) < 1e-14


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_lgl_quadrature_exact_to_degree_2N_minus_1(N):
    x, w = lgl(N)
    assert abs(w.sum().item() - 2.0) < 1e-14
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((w * x ** k).sum().item() - exact) < 1e-14
    # and not for degree 2N (Lobatto rules stop at 2N-1)
    k = 2 * N
    assert abs((w * x ** k).sum().item() - 2.0 / (k + 1)) > 1e-6


# ----------------------------------------------------------- derivative matrix

@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 9])
def test_D_differentiates_polynomials_exactly(N):
    x, _ = lgl(N)
    D = diff_matrix(N)
    for k in range(N + 1):
        f = x ** k
        df = k * x ** (k - 1) if k > 0 else torch.zeros_like(x)
        assert torch.allclose(D @ f, df, atol=5e-13 * max(1, N * N), rtol=0)
    assert (D @ torch.ones(N + 1, dtype=torch.float64)).abs().max() < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_D_is_derivative_of_lagrange_basis(N):
    """D_im = l_m'(xi_i): compare with a centred difference of the Lagrange basis."""
    x, _ = lgl(N)
    h = 1e-5
    Lp = lagrange_eval(N, x.numpy() + h)
    Lm = lagrange_eval(N, x.numpy() - h)
    fd = (Lp - Lm) / (2 * h)
    assert torch.allclose(diff_matrix(N), fd, atol=1e-6 * N * N, rtol=0)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_D_summation_by_parts(N):
    _, w = lgl(N)
    Q = torch.diag(w) @ diff_matrix(N)
    B = torch.zeros(N + 1, N + 1, dtype=torch.float64)
    B[0, 0], B[N, N] = -1.0, 1.0
    assert torch.allclose(Q + Q.T, B, atol=1e-14, rtol=0)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_D_diagonal_matches_closed_form(N):
    """The negative-sum diagonal equals the exact diagonal -N(N+1)/4, 0, ..., 0, N(N+1)/4."""
    d = torch.diagonal(diff_matrix(N))
    want = torch.zeros(N + 1, dtype=torch.float64)
    want[0], want[N] = -N * (N + 1) / 4.0, N * (N + 1) / 4.0
    assert torch.allclose(d, want, atol=1e-13 * N * N, rtol=0)
    assert (diff_matrix(N).sum(1)).abs().max() < 4e-16 * N * N


def test_lagrange_cardinal():
    x, _ = lgl(5)
    assert torch.allclose(lagrange_eval(5, x.numpy()), torch.eye(6, dtype=torch.float64), atol=1e-14)


# ------------------------------------------------------------------------- RK

def _butcher():
    """Butcher tableau of the 2N-storage scheme (exact rationals)."""
    A = [Fraction(0), Fraction(-567301805773, 1357537059087), Fraction(-2404267990393, 2016746695238),
         Fraction(-3550918686646, 2091501179385), Fraction(-1275806237668, 842570457699)]
    B = [Fraction(1432997174477, 9575080441755), Fraction(5161836677717, 13612068292357),
         Fraction(1720146321549, 2090206949498), Fraction(3134564353537, 4481467310338),
         Fraction(2277821191437, 14882151754819)]
    s = 5
    # G_j = sum_{l<=j} (prod_{m=l+1..j} A_m) k_l ;  U_i = U_0 + sum_{j<=i} B_j G_j
    coef = [[Fraction(0)] * s for _ in range(s)]  # coef[j][l]: weight of k_l in G_j
    for j in range(s):
        for l in range(j + 1):
            p = Fraction(1)
            for m in range(l + 1, j + 1):
                p *= A[m]
            coef[j][l] = p
    a = [[Fraction(0)] * s for _ in range(s)]
    for i in range(1, s):           # stage i evaluates at U_{i-1} = U0 + sum_{j<i} B_j G_j
        for l in range(s):
            a[i][l] = sum(B[j] * coef[j][l] for j in range(i))
    b = [sum(B[j] * coef[j][l] for j in range(s)) for l in range(s)]
    c = [sum(a[i]) for i in range(s)]
    return a, b, c


def test_rk_coefficients_match_float_tables():
    a, b, c = _butcher()
    assert RK_A[0] == 0.0
    for i in range(5):
        assert abs(float(c[i]) - RK_C[i]) < 1e-15


def test_rk_fourth_order_conditions():
    a, b, c = _butcher()
    s = range(5)
    conds = [
        (sum(b), 1),
        (sum(b[i] * c[i] for i in s), Fraction(1, 2)),
        (sum(b[i] * c[i] ** 2 for i in s), Fraction(1, 3)),
        (sum(b[i] * a[i][j] * c[j] for i in s for j in s), Fraction(1, 6)),
        (sum(b[i] * c[i] ** 3 for i in s), Fraction(1, 4)),
        (sum(b[i] * c[i] * a[i][j] * c[j] for i in s for j in s), Fraction(1, 8)),
        (sum(b[i] * a[i][j] * c[j] ** 2 for i in s for j in s), Fraction(1, 12)),
        (sum(b[i] * a[i][j] * a[j][k] * c[k] for i in s for j in s for k in s), Fraction(1, 24)),
    ]
    for got, want in conds:
        assert abs(float(got - want)) < 1e-15


def test_rk_observed_order_four():
    """y' = i w y integrated to t = 1: error ratio under halving dt -> 2^4."""
    w = 3.0
    y0 = torch.tensor([1.0 + 0j], dtype=torch.complex128)
    errs = []
    for n in (10, 20, 40):
        y = lsrk(lambda y, t: 1j * w * y, y0, 1.0 / n, n)
        errs.append(abs(complex(y[0]) - complex(np.exp(1j * w))))
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(3.8 < r < 4.3 for r in rates), rates


def test_rk_nonautonomous_stage_times():
    """y' = t^3 is integrated exactly by a fourth-order method (stage times C)."""
    y = lsrk(lambda y, t: torch.full_like(y, t ** 3), torch.zeros(1, dtype=torch.float64), 0.25, 4)
    assert abs(y.item() - 0.25) < 1e-15
