// Algebraic equilibrium wall-stress model (paper Sec. 3: the GPU wall model
// runs one thread per wall-face degree of freedom).  Per wall-face node: the
// state at the interface node n_wm on the wall-normal line, the wall-parallel
// velocity, its Van Driest transform for an adiabatic wall (Crocco-Busemann
// temperature, recovery factor r), and the friction velocity from Spalding's
// law (quartic variant, kappa = 0.4, C = 0.1108) by a Newton iteration that
// starts below the root:
//   F(x) = h x / nu_w - f(u_VD / x),   f(u+) = u+ + C (exp(k) - sum_{n<5} k^n/n!),
//   k = kappa u+.  F is increasing and concave in x, so Newton steps from any
//   point with F <= 0 increase monotonically to the root.
// Output per wall face: tau[(face * 3 + c) * NF + ab], the wall-stress vector
// rho_w u_tau^2 t along the wall-parallel velocity direction t.  The wall
// viscosity is the gas model's at T_w (constant, or Sutherland's law).
#include "dg_device.hpp"

namespace dg {
namespace {

constexpr double kKappa = 0.4;
constexpr double kSpaldingC = 0.1108;

// f(u+) and f'(u+) of Spalding's law, k = kappa u+:
//   f = u+ + C T5(k),  f' = 1 + C kappa T4(k),  Tm(k) = exp(k) - sum_{n<m} k^n/n!
// T5 for k <= 5 as the series sum_{n>=5} k^n/n! (no cancellation near 0; the
// 40 terms n = 5..44 reach below 1e-25 of the sum), multiplying by the
// reciprocals 1/n instead of dividing; T4 = T5 + k^4/24.  Above 5 from exp(k).
template <int n>
__device__ inline void tail_terms(double k, double& t, double& s) {
  if constexpr (n < 45) {
    s += t;
    t *= k * (1.0 / (n + 1));
    tail_terms<n + 1>(k, t, s);
  }
}

__device__ inline void spalding_f(double up, double& f, double& df) {
  const double k = kKappa * up;
  const double k2 = k * k, k4 = k2 * k2;
  double t5, t4;
  if (k > 5.0) {
    const double e = exp(k);
    const double p3 = 1.0 + k * (1.0 + k * (0.5 + k * (1.0 / 6.0)));
    t4 = e - p3;
    t5 = t4 - k4 * (1.0 / 24.0);
  } else {
    double t = k4 * k * (1.0 / 120.0), s = 0.0;
    tail_terms<5>(k, t, s);
    t5 = s;
    t4 = s + k4 * (1.0 / 24.0);
  }
  f = up + kSpaldingC * t5;
  df = 1.0 + kSpaldingC * kKappa * t4;
}

// F(x) and F'(x); F = -inf where exp(kappa u+) would overflow (far below the root)
__device__ inline void spalding_residual(double x, double u, double h, double nu, double& F,
                                         double& dF) {
  const double up = u / x;
  if (kKappa * up > 700.0) {
    F = -INFINITY;
    dF = 0.0;
    return;
  }
  double f, df;
  spalding_f(up, f, df);
  F = h * x / nu - f;
  dF = h / nu + df * up / x;
}

__device__ inline double solve_u_tau(double u, double h, double nu) {
  if (!(u > 0.0)) return 0.0;
  double F, dF;
  double lo = sqrt(nu * u / h);  // u+ <= y+ bounds the root from below
  spalding_residual(lo, u, h, nu, F, dF);
  if (F >= 0.0) return lo;
  double hi = 2.0 * lo;
  for (int it = 0; it < 200; ++it) {
    spalding_residual(hi, u, h, nu, F, dF);
    if (F > 0.0) break;
    lo = hi;
    hi *= 2.0;
  }
  for (int it = 0; it < 200; ++it) {
    spalding_residual(lo, u, h, nu, F, dF);
    if (isfinite(F)) break;
    lo = sqrt(lo * hi);
  }
  double x = lo;
  for (int it = 0; it < 100; ++it) {
    spalding_residual(x, u, h, nu, F, dF);
    const double dx = -F / dF;
    x += dx;
    if (!(dx > 4e-16 * x)) break;
  }
  return x;
}

__global__ __launch_bounds__(256) void k_wall_stress(const double* __restrict__ U,
                                                     double* __restrict__ tau, DevMesh mesh,
                                                     DevPhys ph, int N, int n_wm, double xi_wm1,
                                                     double recovery, long long n_tasks) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n_tasks) return;
  const int NP = N + 1, NF = NP * NP, NN = NF * NP;
  const long long w = t / NF;
  const int ab = static_cast<int>(t - w * NF);
  // wall face w -> (direction d, side, element indices a, b of the wall plane)
  int d = 0;
  long long base = 0, M = 0;
  for (d = 0; d < 3; ++d) {
    if (mesh.bc[d] == DG_BC_PERIODIC) continue;
    const int na = d == 0 ? mesh.n[1] : mesh.n[0];
    const int nb = d == 2 ? mesh.n[1] : mesh.n[2];
    M = static_cast<long long>(na) * nb;
    if (w < base + 2 * M) break;
    base += 2 * M;
  }
  const long long r = w - base;
  const int side = r < M ? 0 : 1;
  const long long q = r - side * M;
  const int na = d == 0 ? mesh.n[1] : mesh.n[0];
  const int ea = static_cast<int>(q % na), eb = static_cast<int>(q / na);
  const int nd = d == 0 ? mesh.n[0] : (d == 1 ? mesh.n[1] : mesh.n[2]);
  const int ed = side == 0 ? 0 : nd - 1;
  const int ex = d == 0 ? ed : ea, ey = d == 1 ? ed : (d == 0 ? ea : eb), ez = d == 2 ? ed : eb;
  const int an = ab % NP, bn = ab / NP;
  const int line = side == 0 ? n_wm : N - n_wm;  // interface node index along d
  const int i = d == 0 ? line : an, j = d == 1 ? line : (d == 0 ? an : bn), k = d == 2 ? line : bn;
  const long long e = ex + static_cast<long long>(mesh.n[0]) * (ey + static_cast<long long>(mesh.n[1]) * ez);
  const long long stride = mesh.nE * NN;
  double s[5];
  load_state(U, stride, e * NN + i + NP * (j + NP * k), s);
  const Prim P = primitives(s, ph);
  double ut[3] = {P.u, P.v, P.w};
  ut[d] = 0.0;  // wall-parallel part (the normal is +-e_d)
  const double u_par = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
  double* out = tau + w * 3 * NF + ab;
  if (!(u_par > 0.0)) {
    for (int c = 0; c < 3; ++c) out[c * NF] = 0.0;
    return;
  }
  // Van Driest transform, adiabatic wall: T_w = T + r u^2 / (2 c_p),
  // u_VD = a asin(u / a), a^2 = 2 c_p T_w / r
  const double cp = ph.gamma * ph.R / ph.gm1;
  const double T_w = P.T + recovery * u_par * u_par / (2.0 * cp);
  const double a = sqrt(2.0 * cp * T_w / recovery);
  const double u_vd = a * asin(u_par / a);
  const double rho_w = P.p / (ph.R * T_w);
  const double nu_w = ph.mu * viscosity_ratio(ph, T_w) / rho_w;
  const double sd = d == 0 ? mesh.s[0][ex] : (d == 1 ? mesh.s[1][ey] : mesh.s[2][ez]);
  const double h = xi_wm1 / sd;  // (xi_nwm + 1) width / 2
  const double u_tau = solve_u_tau(u_vd, h, nu_w);
  const double tw = rho_w * u_tau * u_tau / u_par;
  for (int c = 0; c < 3; ++c) out[c * NF] = tw * ut[c];
}

}  // namespace

hipError_t launch_wall_stress(int N, const DevMesh& m, const DevPhys& p, const double* U, int n_wm,
                              double xi_wm1, double recovery, double* tau, hipStream_t s) {
  const long long tasks = wall_faces(m) * (N + 1) * (N + 1);
  if (tasks == 0) return hipSuccess;
  const long long blocks = (tasks + 255) / 256;
  hipLaunchKernelGGL(k_wall_stress, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, U, tau, m, p,
                     N, n_wm, xi_wm1, recovery, tasks);
  return hipGetLastError();
}

}  // namespace dg
