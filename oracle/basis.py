"""Legendre-Gauss-Lobatto basis of the oracle (test infrastructure only).

The paper's scheme collocates on Legendre-Gauss-Lobatto (LGL) nodes (Sec. 2.2,
split-form DG "evaluated at Legendre-Gauss-Lobatto nodes").  The paper prints
neither the nodes nor the derivative matrix, so both follow their textbook
definitions:

* nodes: xi_0 = -1, xi_N = +1 and the N-1 roots of P_N'(xi) (P_N the Legendre
  polynomial of degree N);
* weights: w_i = 2 / (N (N+1) P_N(xi_i)^2);
* derivative matrix: D_im = l_m'(xi_i) for the Lagrange polynomials l_m of the
  nodes; the off-diagonal entries are written in the classical closed form for
  LGL points
      D_im = P_N(xi_i) / (P_N(xi_m) (xi_i - xi_m))     (i != m),
  and the diagonal by the negative-sum rule D_ii = -sum_{m != i} D_im.
  Reading: the exact D annihilates constants (its diagonal is -N(N+1)/4,
  0, ..., 0, +N(N+1)/4); the negative-sum diagonal keeps that property in
  floating point, which fixes the discrete operator to rounding on nearly
  constant data (low-Mach pressure), where rounded closed-form diagonals leave
  row sums of a few ulps that dominate the result.

The off-diagonal construction differs in method from any barycentric/Newton
construction so that an independent implementation is pinned against it.
"""

from __future__ import annotations

import numpy as np
import torch
from numpy.polynomial import legendre as npleg

__all__ = ["lgl", "diff_matrix", "lagrange_eval"]


def _legendre_coeffs(N: int) -> np.ndarray:
    c = np.zeros(N + 1)
    c[N] = 1.0
    return c


def lgl(N: int):
    """Return (nodes, weights) of the (N+1)-point LGL rule as float64 tensors."""
    if N < 1:
        raise ValueError("LGL rule needs N >= 1")
    cN = _legendre_coeffs(N)
    dcN = npleg.legder(cN)
    inner = np.sort(np.real(npleg.legroots(dcN))) if N >= 2 else np.zeros(0)
    # polish the interior roots of P_N' with Newton steps on P_N' itself
    d2cN = npleg.legder(dcN)
    for _ in range(3):
        if inner.size:
            inner = inner - npleg.legval(inner, dcN) / npleg.legval(inner, d2cN)
    x = np.concatenate(([-1.0], inner, [1.0]))
    PN = npleg.legval(x, cN)
    w = 2.0 / (N * (N + 1) * PN ** 2)
    return torch.tensor(x, dtype=torch.float64), torch.tensor(w, dtype=torch.float64)


def diff_matrix(N: int) -> torch.Tensor:
    """LGL nodal derivative matrix D[i, m] = l_m'(xi_i) (see module doc)."""
    x, _ = lgl(N)
    x = x.numpy()
    PN = npleg.legval(x, _legendre_coeffs(N))
    D = np.zeros((N + 1, N + 1))
    for i in range(N + 1):
        for m in range(N + 1):
            if i != m:
                D[i, m] = PN[i] / (PN[m] * (x[i] - x[m]))
    for i in range(N + 1):
        D[i, i] = -sum(D[i, m] for m in range(N + 1) if m != i)
    return torch.tensor(D, dtype=torch.float64)


def lagrange_eval(N: int, xs) -> torch.Tensor:
    """Matrix L[k, m] = l_m(xs[k]) of the LGL Lagrange basis (used by tests)."""
    x, _ = lgl(N)
    x = x.numpy()
    xs = np.asarray(xs, dtype=np.float64)
    L = np.ones((xs.size, N + 1))
    for m in range(N + 1):
        for q in range(N + 1):
            if q != m:
                L[:, m] *= (xs - x[q]) / (x[m] - x[q])
    return torch.tensor(L, dtype=torch.float64)
