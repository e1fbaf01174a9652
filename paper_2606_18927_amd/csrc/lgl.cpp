// Host construction of the Legendre-Gauss-Lobatto basis (paper Sec. 2.2:
// collocation on LGL nodes).
//
// Nodes: -1, +1 and the roots of P_N', found by Newton's method on P_N' with
// the second derivative from Legendre's equation
//   (1 - x^2) P_N'' = 2 x P_N' - N (N+1) P_N,
// started from the Chebyshev-Gauss-Lobatto points -cos(pi j / N).
// Weights: w_j = 2 / (N (N+1) P_N(x_j)^2).
// Derivative matrix: barycentric form D_im = (b_m / b_i) / (x_i - x_m) with
// b_i = 1 / prod_{m != i} (x_i - x_m), and the diagonal by the negative-sum
// rule D_ii = -sum_{m != i} D_im, which makes rows of D annihilate constants
// to rounding.
#include <cmath>
#include <vector>

#include "dg_internal.hpp"

namespace dg {

namespace {

// P_N(x) and P_N'(x) by the three-term recurrence.
void legendre(int N, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (N == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 1; k < N; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    const double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  P = p1;
  dP = d1;
}

}  // namespace

void lgl_nodes_weights(int N, std::vector<double>& xi, std::vector<double>& w) {
  xi.assign(N + 1, 0.0);
  w.assign(N + 1, 0.0);
  xi[0] = -1.0;
  xi[N] = 1.0;
  const double nn1 = N * (N + 1.0);
  for (int j = 1; j < N; ++j) {
    double x = -std::cos(M_PI * j / N);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(N, x, P, dP);
      const double d2P = (2.0 * x * dP - nn1 * P) / (1.0 - x * x);
      const double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < 1e-16 * (1.0 + std::fabs(x))) break;
    }
    xi[j] = x;
  }
  // exact symmetry of the rule
  for (int j = 0; j <= N / 2; ++j) {
    const double a = 0.5 * (xi[N - j] - xi[j]);
    xi[j] = -a;
    xi[N - j] = a;
  }
  if (N % 2 == 0) xi[N / 2] = 0.0;
  for (int j = 0; j <= N; ++j) {
    double P, dP;
    legendre(N, xi[j], P, dP);
    w[j] = 2.0 / (nn1 * P * P);
  }
}

void lgl_diff_matrix(const std::vector<double>& xi, std::vector<double>& D) {
  const int NP = static_cast<int>(xi.size());
  std::vector<double> b(NP, 1.0);
  for (int i = 0; i < NP; ++i) {
    double prod = 1.0;
    for (int m = 0; m < NP; ++m)
      if (m != i) prod *= (xi[i] - xi[m]);
    b[i] = 1.0 / prod;
  }
  D.assign(NP * NP, 0.0);
  for (int i = 0; i < NP; ++i) {
    double diag = 0.0;
    for (int m = 0; m < NP; ++m) {
      if (m == i) continue;
      const double v = (b[m] / b[i]) / (xi[i] - xi[m]);
      D[i * NP + m] = v;
      diag -= v;
    }
    D[i * NP + i] = diag;
  }
}

}  // namespace dg
