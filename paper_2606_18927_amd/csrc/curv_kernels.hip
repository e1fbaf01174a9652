// Split-form DGSEM on curvilinear hexahedra (FP64 or mixed precision,
// structured meshes with periodic or isothermal no-slip wall ends).
//
// Geometry (the paper's production meshes are curved, Sec. 4): each element's
// map is the degree-N interpolant of its node coordinates.  The metric terms
// J a^i_n are Kopriva's conservative curl form,
//   J a^i_n = -1/2 [curl_xi (X_l grad_xi X_m - X_m grad_xi X_l)]_i, (n, m, l) cyclic,
// with the collocation derivative D for every xi-derivative, so the discrete
// metric identities hold and both elements of a face see the same normal;
// J = det(dX/dxi).  k_metrics computes them once per mesh into
//   geo[c][e][node], c = 3 i + n: J a^i_n; c = 9: 1 / J; then the same ten
//   fields in FP32 (read by the mixed-precision sweeps).
// Operator per stage (one workgroup per element, one lane per node; face
// lanes = one lane per face node):
//   k_face_flux_curv  BR1 gradients at the face nodes (chain rule with the
//                     node's metrics: J grad q = sum_i J a^i (D_i q + lifting
//                     term)) and the contravariant normal viscous flux
//                     Fv^i = sum_d f_v,d J a^i_d of every face, to ffv;
//   k_rhs_curv        gradients of every node, per direction i the
//                     contravariant Kennedy-Gruber two-point flux with
//                     averaged metrics sum_d f#_d (J a^i_d(A) + J a^i_d(B)) / 2
//                     and the viscous flux Fv^i, Lax-Friedrichs across each
//                     face with its normal J a^i (that of the element below
//                     the face, shared by both sides), Ut = -(1/J)(...),
//                     fused RK update.
#include "dg_device.hpp"

namespace dg {
namespace {

template <int N>
struct CurvCfg {
  static constexpr int NP = N + 1, NF = NP * NP, NN = NF * NP;
  static constexpr int LANES = NN > 6 * NF ? NN : 6 * NF;
  static constexpr int BS = (LANES + 63) / 64 * 64;
};

// sum_m D[idx][m] f(node with the dir-coordinate replaced by m), f an LDS field
// indexed i + NP (j + NP k)
template <int N, typename R>
__device__ inline R dline(const R* f, const double (*sD)[N + 2], int dir, int i, int j, int k) {
  constexpr int NP = N + 1;
  const int idx = dir == 0 ? i : (dir == 1 ? j : k);
  const int base = dir == 0 ? NP * (j + NP * k) : (dir == 1 ? i + NP * NP * k : i + NP * j);
  const int step = dir == 0 ? 1 : (dir == 1 ? NP : NP * NP);
  R a = R(0);
#pragma unroll
  for (int m = 0; m < NP; ++m) a += static_cast<R>(sD[idx][m]) * f[base + step * m];
  return a;
}

// Chandrashekar's flux contracted with the metric vector M (the average of the
// two nodes' J a^i in the volume, the face normal on a face): with
// a, b = (rho, u, v, w, beta, |u|^2), beta = rho / (2 p), U~ = {{u}} . M,
//   F_rho = rho_ln U~,  F_m = F_rho {{u}} + p^ M,  p^ = {{rho}} / (2 {{beta}}),
//   F_E = F_rho (1 / (2 (gamma - 1) beta_ln) - {{|u|^2}} / 2) + {{u}} . F_m.
__device__ inline void ec_flux_contra(const double a[6], const double b[6], double M0, double M1, double M2,
                                      double gm1, double f[5]) {
  double rho_ln, inv_beta_ln, p_hat;
  ec_means(a[0], b[0], a[4], b[4], rho_ln, inv_beta_ln, p_hat);
  const double u = 0.5 * (a[1] + b[1]), v = 0.5 * (a[2] + b[2]), w = 0.5 * (a[3] + b[3]);
  const double q2 = 0.5 * (a[5] + b[5]);
  const double F1 = rho_ln * (u * M0 + v * M1 + w * M2);
  f[0] = F1;
  f[1] = F1 * u + p_hat * M0;
  f[2] = F1 * v + p_hat * M1;
  f[3] = F1 * w + p_hat * M2;
  f[4] = F1 * (0.5 / gm1 * inv_beta_ln - 0.5 * q2) + f[1] * u + f[2] * v + f[3] * w;
}

// The same pair in FP32 relative to the element's reference state (mixed
// precision): a, b = (rho, u, v, w, beta - beta_ref, |u|^2, pi) with
// pi = rho (p - p_ref) / p; with sb = beta_a + beta_b,
//   p^ - p_ref = (pi_a + pi_b) / (2 sb),
//   1 / beta_ln - 1 / beta_ref = (2 (F - 1) - (dbeta_a + dbeta_b) / beta_ref) / sb,
// F = atanh f / f of the beta pair (its series less the leading 1 below
// f^2 = 1e-2), so no FP32 difference of O(p_ref) terms is formed.
// f = f#_EC - (0, p_ref M, F1 e_ref + p_ref U_c) with U_c = {{u}} . M and
// e_ref = kap / beta_ref; uc returns U_c.  The p_ref M part sums to the
// discrete divergence of the metric terms (zero by the metric identities);
// the energy part is added back in FP64 by the caller.
__device__ inline void ec_flux_contra_ref(const float a[7], const float b[7], float M0, float M1, float M2,
                                          float kap, float beta_ref, float ibr, float f[5], float& uc) {
  const float sr = a[0] + b[0], sdb = a[4] + b[4];
  const float sb = 2.0f * beta_ref + sdb;
  const float x = __builtin_amdgcn_rcpf(sr * sb);
  const float ir = sb * x, ib = sr * x;
  const float fr = (a[0] - b[0]) * ir, fb = (a[4] - b[4]) * ib;
  const float ur = fr * fr, ub = fb * fb;
  float G = 1.0f - ur * (1.0f / 3.0f + ur * (4.0f / 45.0f + ur * (44.0f / 945.0f)));
  float Fs = ub * (1.0f / 3.0f + ub * (0.2f + ub * (1.0f / 7.0f)));
  if (ur >= 1e-2f) G = fr / atanhf(fr);
  if (ub >= 1e-2f) Fs = atanhf(fb) / fb - 1.0f;
  const float u = 0.5f * (a[1] + b[1]), v = 0.5f * (a[2] + b[2]), w = 0.5f * (a[3] + b[3]);
  uc = u * M0 + v * M1 + w * M2;
  const float F1 = 0.5f * sr * G * uc;
  const float dp = 0.5f * (a[6] + b[6]) * ib;
  const float dib = (2.0f * Fs - sdb * ibr) * ib;
  const float X = kap * dib - 0.25f * (a[5] + b[5]) + (u * u + v * v + w * w);
  f[0] = F1;
  f[1] = F1 * u + dp * M0;
  f[2] = F1 * v + dp * M1;
  f[3] = F1 * w + dp * M2;
  f[4] = F1 * X + dp * uc;
}

// Roe's dissipation sum_k |lambda_k| alpha_k r_k across a face with unit
// normal n (L on the side n points away from; primitives (rho, u, v, w, p)
// and total energies E), linearised at the Roe average (sqrt(rho)-weighted u
// and H = (E + p) / rho, rho~ = sqrt(rho_L rho_R), a~^2 = (gamma - 1)(H~ - |u~|^2/2)):
// acoustic waves u~.n -+ a~ with alpha = ([[p]] -+ rho~ a~ [[u.n]]) / (2 a~^2),
// r = (1, u~ -+ a~ n, H~ -+ (u~.n) a~) and Harten-Hyman |lambda|; the entropy
// wave u~.n with alpha = [[rho]] - [[p]] / a~^2, r = (1, u~, |u~|^2 / 2); the
// shear wave u~.n with rho~ (0, [[u]]_t, u~ . [[u]]_t), [[u]]_t = [[u]] - [[u.n]] n.
__device__ inline void roe_dissipation_normal(const double L[5], double EL, const double R[5], double ER,
                                              const double n[3], double gamma, double D[5]) {
  const double sl = sqrt(L[0]), sr = sqrt(R[0]);
  const double isum = 1.0 / (sl + sr);
  const double wl = sl * isum, wr = sr * isum;
  double ut[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) ut[c] = wl * L[1 + c] + wr * R[1 + c];
  const double H = wl * (EL + L[4]) / L[0] + wr * (ER + R[4]) / R[0];
  const double q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  const double a2 = (gamma - 1.0) * (H - 0.5 * q2);
  const double a = sqrt(a2);
  const double rho = sl * sr;
  const double un = ut[0] * n[0] + ut[1] * n[1] + ut[2] * n[2];
  const double dp = R[4] - L[4];
  double du[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) du[c] = R[1 + c] - L[1 + c];
  const double dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  const double al1 = (dp - rho * a * dun) / (2.0 * a2);
  const double al5 = (dp + rho * a * dun) / (2.0 * a2);
  const double al2 = (R[0] - L[0]) - dp / a2;
  const double unl = L[1] * n[0] + L[2] * n[1] + L[3] * n[2], unr = R[1] * n[0] + R[2] * n[1] + R[3] * n[2];
  const double cl = sqrt(gamma * L[4] / L[0]), cr = sqrt(gamma * R[4] / R[0]);
  const double l1 = hh_abs(un - a, unl - cl, unr - cr);
  const double l5 = hh_abs(un + a, unl + cl, unr + cr);
  const double l2 = fabs(un);
  const double t1 = l1 * al1, t5 = l5 * al5, t2 = l2 * al2, ts = l2 * rho;
  double udt = 0.0;
  D[0] = t1 + t2 + t5;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double sh = du[c] - dun * n[c];
    udt += ut[c] * sh;
    D[1 + c] = (t1 + t2 + t5) * ut[c] + (t5 - t1) * a * n[c] + ts * sh;
  }
  D[4] = t1 * (H - un * a) + t2 * (0.5 * q2) + t5 * (H + un * a) + ts * udt;
}

// ---------------------------------------------------------------- metrics
template <int N>
__global__ __launch_bounds__(CurvCfg<N>::BS) void k_metrics(const double* __restrict__ X,
                                                           double* __restrict__ geo,
                                                           double* __restrict__ geoF, bool with_f32,
                                                           DevBasis basis, long long nE,
                                                           int* __restrict__ status) {
  using C = CurvCfg<N>;
  constexpr int NP = C::NP, NN = C::NN;
  __shared__ double sD[NP][N + 2];
  __shared__ double sX[3][NN];
  __shared__ double sdX[9][NN];  // dX_n / dxi^j at 3 n + j
  __shared__ double sV[3][NN];
  const int tid = threadIdx.x;
  const long long e = blockIdx.x;
  const long long stride = nE * NN;
  const bool active = tid < NN;
  const int i = tid % NP, j = (tid / NP) % NP, k = tid / (NP * NP);
  if (tid < NP * NP) sD[tid / NP][tid % NP] = basis.D[tid];
  // coordinates relative to the element's node (0, 0, 0): the curl form is
  // translation invariant, and its rounding then scales with the element's
  // size instead of the magnitude of the coordinates
  if (active) {
#pragma unroll
    for (int n = 0; n < 3; ++n) sX[n][tid] = X[n * stride + e * NN + tid] - X[n * stride + e * NN];
  }
  __syncthreads();
  double dX[9];
  if (active) {
#pragma unroll
    for (int n = 0; n < 3; ++n)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        dX[3 * n + d] = dline<N>(sX[n], sD, d, i, j, k);
        sdX[3 * n + d][tid] = dX[3 * n + d];
      }
  }
  __syncthreads();
  double Ja[9];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    const int m = (n + 1) % 3, l = (n + 2) % 3;
    if (active) {
#pragma unroll
      for (int d = 0; d < 3; ++d)
        sV[d][tid] = sX[l][tid] * sdX[3 * m + d][tid] - sX[m][tid] * sdX[3 * l + d][tid];
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int a = (r + 1) % 3, b = (r + 2) % 3;
        Ja[3 * r + n] = -0.5 * (dline<N>(sV[b], sD, a, i, j, k) - dline<N>(sV[a], sD, b, i, j, k));
      }
    }
    __syncthreads();
  }
  if (active) {
    const double J = dX[0] * (dX[4] * dX[8] - dX[5] * dX[7]) - dX[1] * (dX[3] * dX[8] - dX[5] * dX[6]) +
                     dX[2] * (dX[3] * dX[7] - dX[4] * dX[6]);
    if (!(J > 0.0)) status[0] = 1;
    const long long o = e * NN + tid;
#pragma unroll
    for (int c = 0; c < 9; ++c) geo[c * stride + o] = Ja[c];
    geo[9 * stride + o] = 1.0 / J;
    // boundary nodes once more, contiguous per element (face node number t)
    if (i == 0 || i == N || j == 0 || j == N || k == 0 || k == N) {
      constexpr int NFN = n_face_nodes<N>();
      const long long of = e * NFN + face_node_index<N>(i, j, k);
#pragma unroll
      for (int c = 0; c < 9; ++c) geoF[c * nE * NFN + of] = Ja[c];
      geoF[9 * nE * NFN + of] = 1.0 / J;
    }
    // FP32 copy for the mixed-precision sweeps, after the ten FP64 fields
    // (the workspace holds it only in mixed-precision contexts)
    if (with_f32) {
      float* const g32 = reinterpret_cast<float*>(geo + 10 * stride);
#pragma unroll
      for (int c = 0; c < 9; ++c) g32[c * stride + o] = static_cast<float>(Ja[c]);
      g32[9 * stride + o] = static_cast<float>(1.0 / J);
    }
  }
}

// Own-side contravariant viscous flux along metric vector M from the stress:
// (sum_d M_d tau_0d, sum_d M_d tau_1d, sum_d M_d tau_2d, u . (those) + M . qT)
template <typename R>
__device__ inline void contra_viscous(R u, R v, R w, const R tau[6], const R qT[3], R M0, R M1, R M2,
                                      R f[4]) {
  f[0] = M0 * tau[0] + M1 * tau[3] + M2 * tau[4];
  f[1] = M0 * tau[3] + M1 * tau[1] + M2 * tau[5];
  f[2] = M0 * tau[4] + M1 * tau[5] + M2 * tau[2];
  f[3] = u * f[0] + v * f[1] + w * f[2] + M0 * qT[0] + M1 * qT[1] + M2 * qT[2];
}

// Stress (t00, t11, t22, t01, t02, t12) and heat flux of physical gradients g[3 q + d]
template <typename R>
__device__ inline void stress64(const R g[12], R mu, R kappa, R tau[6], R qT[3]) {
  const R dd = R(2.0 / 3.0) * (g[0] + g[4] + g[8]);
  tau[0] = mu * (g[0] + g[0] - dd);
  tau[1] = mu * (g[4] + g[4] - dd);
  tau[2] = mu * (g[8] + g[8] - dd);
  tau[3] = mu * (g[1] + g[3]);
  tau[4] = mu * (g[2] + g[6]);
  tau[5] = mu * (g[5] + g[7]);
  qT[0] = kappa * g[9];
  qT[1] = kappa * g[10];
  qT[2] = kappa * g[11];
}

// Physical gradients of q = (u, v, w, T) at node (i, j, k): reference
// derivatives plus the lifting terms of the faces the node lies on, then
// grad q = (1/J) sum_r J a^r gxi_r.  sq[c] are LDS fields of q; corr[f][c][ab]
// the lifting terms (q* - q)(+-1/w) of face f.
template <int N, typename R>
__device__ inline void curv_gradients(const R* const sq[4], const double (*sD)[N + 2],
                                      const R (*corr)[4][(N + 1) * (N + 1)], int i, int j, int k,
                                      const R Ja[9], R invJ, R g[12]) {
  constexpr int NP = N + 1;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    R gx[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) gx[r] = dline<N, R>(sq[c], sD, r, i, j, k);
    if (i == 0) gx[0] += corr[0][c][j + NP * k];
    if (i == N) gx[0] += corr[1][c][j + NP * k];
    if (j == 0) gx[1] += corr[2][c][i + NP * k];
    if (j == N) gx[1] += corr[3][c][i + NP * k];
    if (k == 0) gx[2] += corr[4][c][i + NP * j];
    if (k == N) gx[2] += corr[5][c][i + NP * j];
#pragma unroll
    for (int d = 0; d < 3; ++d) g[3 * c + d] = invJ * (Ja[d] * gx[0] + Ja[3 + d] * gx[1] + Ja[6 + d] * gx[2]);
  }
}

// Metric field c at node idx in the sweep precision: the FP64 field, or its
// FP32 copy stored after the ten FP64 fields.
template <typename R>
__device__ inline R geo_at(const double* geo, long long stride, int c, long long idx) {
  if constexpr (sizeof(R) == sizeof(float))
    return reinterpret_cast<const float*>(geo + 10 * stride)[c * stride + idx];
  else
    return geo[c * stride + idx];
}

// ---------------------------------------------------------- face viscous flux
// (R = float in mixed precision: the fluxes are formed in FP64 and stored in FP32)
template <int N, typename R>
__global__ __launch_bounds__(CurvCfg<N>::BS) void k_face_flux_curv(const double* __restrict__ U,
                                                                  R* __restrict__ ffv, DevMesh mesh,
                                                                  DevPhys ph, DevBasis basis) {
  using C = CurvCfg<N>;
  constexpr int NP = C::NP, NF = C::NF, NN = C::NN;
  __shared__ double sD[NP][N + 2];
  __shared__ double sq[4][NN];
  __shared__ double corr[6][4][NF];
  const int tid = threadIdx.x;
  const long long nE = mesh.nE;
  const long long stride = nE * NN;
  const long long e = xcd_remap(blockIdx.x, gridDim.x);
  int ex, ey, ez;
  elem_coords(e, mesh, ex, ey, ez);
  if (tid < NP * NP) sD[tid / NP][tid % NP] = basis.D[tid];
  constexpr int NFN = n_face_nodes<N>();
  static_assert(NFN <= CurvCfg<N>::BS, "one lane per boundary node");
  double Ja[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, invJ = 0.0;
  if (tid < NFN) {
    const long long fs = nE * NFN, of = e * NFN + tid;
#pragma unroll
    for (int c = 0; c < 9; ++c) Ja[c] = mesh.geoF[c * fs + of];
    invJ = mesh.geoF[9 * fs + of];
  }
  if (tid < NN) {
    double s[5];
    load_state(U, stride, e * NN + tid, s);
    const Prim P = primitives(s, ph);
    sq[0][tid] = P.u;
    sq[1][tid] = P.v;
    sq[2][tid] = P.w;
    sq[3][tid] = P.T;
  }
  // face lanes fetch the neighbour's face node now and take their own values
  // from LDS after the barrier
  double sn[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
  long long nb = -1;  // -1: the face is a wall
  if (tid < 6 * NF) {
    const FaceTask<N> ft(tid);
    nb = neighbour(mesh, ex, ey, ez, ft.d, ft.up);
    if (nb >= 0) load_state(U, stride, nb * NN + ft.nb_node(), sn);
  }
  __syncthreads();
  if (tid < 6 * NF) {
    const FaceTask<N> ft(tid);
    const int lo = ft.own_node();
    const double qo[4] = {sq[0][lo], sq[1][lo], sq[2][lo], sq[3][lo]};
    double qs[4] = {0.0, 0.0, 0.0, mesh.T_wall};  // isothermal no-slip wall
    if (nb >= 0) {
      const Prim Pn = primitives(sn, ph);
      qs[0] = 0.5 * (qo[0] + Pn.u);
      qs[1] = 0.5 * (qo[1] + Pn.v);
      qs[2] = 0.5 * (qo[2] + Pn.w);
      qs[3] = 0.5 * (qo[3] + Pn.T);
    }
    const double sc = ft.up ? basis.inv_w_end : -basis.inv_w_end;
#pragma unroll
    for (int c = 0; c < 4; ++c) corr[ft.f][c][ft.ab] = (qs[c] - qo[c]) * sc;
  }
  __syncthreads();
  // one lane per boundary node (face node number t = tid), with that node's
  // metric terms from the boundary-node copy (fetched before the barriers)
  if (tid >= NFN) return;
  int i, j, k;
  face_node_of<N>(tid, i, j, k);
  const int n = i + NP * (j + NP * k);
  const double* const q[4] = {sq[0], sq[1], sq[2], sq[3]};
  double g[12];
  curv_gradients<N, double>(q, sD, corr, i, j, k, Ja, invJ, g);
  const double r = viscosity_ratio(ph, sq[3][n]);
  double tau[6], qT[3];
  stress64<double>(g, ph.mu * r, ph.kappa * r, tau, qT);
  const double u = sq[0][n], v = sq[1][n], w = sq[2][n];
  R* out = ffv + e * (6 * 4 * NF);
  double f[4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int idx = d == 0 ? i : (d == 1 ? j : k);
    if (idx != 0 && idx != N) continue;
    const int ab = d == 0 ? j + NP * k : (d == 1 ? i + NP * k : i + NP * j);
    const int fi = 2 * d + (idx == N ? 1 : 0);
    contra_viscous<double>(u, v, w, tau, qT, Ja[3 * d], Ja[3 * d + 1], Ja[3 * d + 2], f);
#pragma unroll
    for (int c = 0; c < 4; ++c) out[(fi * 4 + c) * NF + ab] = static_cast<R>(f[c]);
  }
}

// ------------------------------------------------------- right-hand side / RK
// The Kennedy-Gruber instances fit 128 registers (four waves per SIMD); the
// FP64 entropy-conserving ones are bounded for three: at 128 they spilled
// 46-58 values per lane, and at degree 7 one workgroup per CU without spills
// is 17 % faster than two with them.  The mixed-precision entropy-conserving
// ones are bounded for four (degree 7: 6 values spilled, 1.85 ms against
// 2.63 ms with three waves and no spills).
// R = float: mixed precision: the LDS fields, gradients, metric terms of the
// sweeps and line sums in FP32, with p, e and T (entropy-conserving pair:
// beta and rho (p - p_ref) / p) relative to the element's first node;
// primitive recovery, lifting corrections, surface fluxes, 1/J scaling and
// the RK update in FP64.  The reference pressure's share of the momentum sums
// is the discrete divergence of the metric terms (zero by the metric
// identities) and is dropped; the energy's, e_ref sum D (rho U~)# + p_ref sum
// D U~#, is added back in FP64.
template <int N, typename R, bool RK, bool VISC, bool EC>
__global__ __launch_bounds__(CurvCfg<N>::BS) __attribute__((amdgpu_waves_per_eu(EC && sizeof(R) == sizeof(double) ? 3 : 4))) void k_rhs_curv(
    const double* __restrict__ U, const R* __restrict__ ffv, double* __restrict__ out,
    double* __restrict__ U_out, DevMesh mesh, DevPhys ph, DevBasis basis, Stage st,
    int* __restrict__ status) {
  using C = CurvCfg<N>;
  constexpr int NP = C::NP, NF = C::NF, NN = C::NN;
  constexpr bool MIXED = sizeof(R) == sizeof(float);
  // LDS fields per node: rho, u, v, w, p, e (p, e relative to the reference in
  // mixed precision); entropy-conserving pair: rho, u, v, w, beta, |u|^2, in
  // mixed precision beta - beta_ref and, seventh, rho (p - p_ref) / p
  constexpr int NSP = EC && MIXED ? 7 : 6;
  __shared__ double sD[NP][N + 2];
  __shared__ R sp[NSP][NN];
  __shared__ double sX[6][5][NF];         // own viscous face flux, then surface terms
  // phase-shared regions: (T, lifting terms) until the gradients are formed,
  // (viscous flux, metric of the sweep direction) in the sweeps
  constexpr int R1 = NN + 6 * 4 * NF, R2 = 4 * NN + 3 * NN;
  __shared__ R sbuf[R1 > R2 ? R1 : R2];
  R* sT = sbuf;
  R(*corr)[4][NF] = reinterpret_cast<R(*)[4][NF]>(sbuf + NN);
  R(*sfv)[NN] = reinterpret_cast<R(*)[NN]>(sbuf);
  R(*sM)[NN] = reinterpret_cast<R(*)[NN]>(sbuf + 4 * NN);

  const int tid = threadIdx.x;
  const long long nE = mesh.nE;
  const long long stride = nE * NN;
  const long long e = xcd_remap(blockIdx.x, gridDim.x);
  int ex, ey, ez;
  elem_coords(e, mesh, ex, ey, ez);
  const bool active = tid < NN;
  const bool face_lane = tid < 6 * NF;
  const int i = tid % NP, j = (tid / NP) % NP, k = tid / NF;
  if (tid < NP * NP) sD[tid / NP][tid % NP] = basis.D[tid];

  // P1: own state; face lanes fetch the neighbour's face node (registers are
  // the limit of this kernel: metric terms, the neighbour's state and the own
  // primitives are fetched again where they are used, from L2 and LDS)
  // mixed precision: the element's first node (with the entropy-conserving
  // pair e_ref is its internal energy p_ref / ((gamma - 1) rho_ref))
  double p_ref = 0.0, e_ref = 0.0, T_ref = 0.0, beta_ref = 0.0;
  if (active) {
    double u0[5];
    load_state(U, stride, e * NN + tid, u0);
    const Prim P = primitives(u0, ph);
    if (!(P.rho > 0.0) || !(P.p > 0.0)) status[0] = 1;
    if (MIXED && ph.mixed_ref) {
      double s0[5];
      load_state(U, stride, e * NN, s0);
      const Prim P0 = primitives(s0, ph);
      p_ref = P0.p;
      e_ref = EC ? P0.p / (ph.gm1 * P0.rho) : P0.e;
      T_ref = P0.T;
      beta_ref = 0.5 * P0.rho / P0.p;
    }
    sp[0][tid] = static_cast<R>(P.rho);
    sp[1][tid] = static_cast<R>(P.u);
    sp[2][tid] = static_cast<R>(P.v);
    sp[3][tid] = static_cast<R>(P.w);
    sp[4][tid] = static_cast<R>(EC ? 0.5 * P.rho / P.p - beta_ref : P.p - p_ref);
    sp[5][tid] = static_cast<R>(EC ? P.u * P.u + P.v * P.v + P.w * P.w : P.e - e_ref);
    if constexpr (EC && MIXED) sp[NSP - 1][tid] = static_cast<R>(P.rho * (P.p - p_ref) / P.p);
    if (VISC) sT[tid] = static_cast<R>(P.T - T_ref);
  }
  double sn[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
  double so[5] = {1.0, 0.0, 0.0, 0.0, 1.0};  // own face node (mixed precision)
  bool fwall1 = true;  // the face task's face is a wall (P1b)
  if (VISC && face_lane) {
    const FaceTask<N> ft(tid);
    const long long nb = neighbour(mesh, ex, ey, ez, ft.d, ft.up);
    fwall1 = nb < 0;
    if (!fwall1) load_state(U, stride, nb * NN + ft.nb_node(), sn);
    if (MIXED) load_state(U, stride, e * NN + ft.own_node(), so);
  }
  __syncthreads();

  // P1b: BR1 lifting terms of the face nodes
  if (VISC) {
    if (face_lane) {
      const FaceTask<N> ft(tid);
      const int lo = ft.own_node();
      double qo[4];
      if constexpr (MIXED) {
        const Prim Po = primitives(so, ph);
        qo[0] = Po.u;
        qo[1] = Po.v;
        qo[2] = Po.w;
        qo[3] = Po.T;
      } else {
        qo[0] = sp[1][lo];
        qo[1] = sp[2][lo];
        qo[2] = sp[3][lo];
        qo[3] = sT[lo];
      }
      double qs[4] = {0.0, 0.0, 0.0, mesh.T_wall};  // isothermal no-slip wall
      if (!fwall1) {
        const Prim Pn = primitives(sn, ph);
        qs[0] = 0.5 * (qo[0] + Pn.u);
        qs[1] = 0.5 * (qo[1] + Pn.v);
        qs[2] = 0.5 * (qo[2] + Pn.w);
        qs[3] = 0.5 * (qo[3] + Pn.T);
      }
      const double sc = ft.up ? basis.inv_w_end : -basis.inv_w_end;
#pragma unroll
      for (int c = 0; c < 4; ++c) corr[ft.f][c][ft.ab] = static_cast<R>((qs[c] - qo[c]) * sc);
    }
    __syncthreads();
  }

  // P2: gradients, stress and heat flux.  With the Kennedy-Gruber pair the
  // metric terms read here stay in registers for the sweeps (and, in FP64,
  // 1/J for the output): read again after P2 they miss in L2.  The
  // entropy-conserving instances and degree 3 have no registers to spare and
  // read them again.
  constexpr bool KEEP = VISC && !EC && N >= 5;
  R tau[6] = {0, 0, 0, 0, 0, 0}, qT[3] = {0, 0, 0};
  R Jr[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (VISC) {
    if (active) {
#pragma unroll
      for (int c = 0; c < 10; ++c) Jr[c] = geo_at<R>(mesh.geo, stride, c, e * NN + tid);
      const R* const q[4] = {sp[1], sp[2], sp[3], sT};
      R g[12];
      curv_gradients<N, R>(q, sD, corr, i, j, k, Jr, Jr[9], g);
      const double r = viscosity_ratio(ph, static_cast<double>(sT[tid]) + T_ref);
      stress64<R>(g, static_cast<R>(ph.mu * r), static_cast<R>(ph.kappa * r), tau, qT);
    }
    __syncthreads();
  }

  // P3: per direction, volume sweep of the two-point and viscous fluxes
  double ut[5] = {0, 0, 0, 0, 0};
#pragma unroll 1
  for (int d = 0; d < 3; ++d) {
    const int idx = d == 0 ? i : (d == 1 ? j : k);
    const int ab = d == 0 ? j + NP * k : (d == 1 ? i + NP * k : i + NP * j);
    R M0 = 0, M1 = 0, M2 = 0, A[NSP];
#pragma unroll
    for (int c = 0; c < NSP; ++c) A[c] = R(c == 0 || c == 4 || c == 5 ? 1 : 0);
    if (active) {
      const long long gi = e * NN + tid;
      if (KEEP) {
        M0 = d == 0 ? Jr[0] : (d == 1 ? Jr[3] : Jr[6]);
        M1 = d == 0 ? Jr[1] : (d == 1 ? Jr[4] : Jr[7]);
        M2 = d == 0 ? Jr[2] : (d == 1 ? Jr[5] : Jr[8]);
      } else {
        M0 = geo_at<R>(mesh.geo, stride, 3 * d, gi);
        M1 = geo_at<R>(mesh.geo, stride, 3 * d + 1, gi);
        M2 = geo_at<R>(mesh.geo, stride, 3 * d + 2, gi);
      }
#pragma unroll
      for (int c = 0; c < NSP; ++c) A[c] = sp[c][tid];
      sM[0][tid] = M0;
      sM[1][tid] = M1;
      sM[2][tid] = M2;
      if (VISC) {
        R f[4];
        contra_viscous<R>(A[1], A[2], A[3], tau, qT, M0, M1, M2, f);
#pragma unroll
        for (int c = 0; c < 4; ++c) sfv[c][tid] = f[c];
        if (idx == 0 || idx == N) {
          const int fi = 2 * d + (idx == N ? 1 : 0);
#pragma unroll
          for (int c = 0; c < 4; ++c) sX[fi][c][ab] = f[c];
        }
      }
    }
    __syncthreads();
    if (active) {
      const int base = d == 0 ? NP * (j + NP * k) : (d == 1 ? i + NF * k : i + NP * j);
      const int step = d == 0 ? 1 : (d == 1 ? NP : NF);
      R ac[5] = {0, 0, 0, 0, 0}, av[4] = {0, 0, 0, 0}, du = 0;
      if constexpr (EC && MIXED) {
        const float kap = static_cast<float>(0.5 / ph.gm1), br = static_cast<float>(beta_ref),
                    ibr = static_cast<float>(1.0 / beta_ref);
#pragma unroll 1
        for (int m = 0; m < NP; ++m) {
          const int nm = base + step * m;
          const float Dm = static_cast<float>(sD[idx][m]);
          const float m0 = 0.5f * (M0 + sM[0][nm]), m1 = 0.5f * (M1 + sM[1][nm]), m2 = 0.5f * (M2 + sM[2][nm]);
          float B[NSP];
#pragma unroll
          for (int c = 0; c < NSP; ++c) B[c] = sp[c][nm];
          float f[5], uc;
          ec_flux_contra_ref(A, B, m0, m1, m2, kap, br, ibr, f, uc);
#pragma unroll
          for (int v = 0; v < 5; ++v) ac[v] += Dm * f[v];
          du += Dm * uc;
          if (VISC) {
#pragma unroll
            for (int c = 0; c < 4; ++c) av[c] += Dm * sfv[c][nm];
          }
        }
      } else if constexpr (EC) {
        // not unrolled: the pair flux is long, and unrolled copies keep too
        // many values live
#pragma unroll 1
        for (int m = 0; m < NP; ++m) {
          const int nm = base + step * m;
          const double Dm = sD[idx][m];
          const double m0 = 0.5 * (M0 + sM[0][nm]), m1 = 0.5 * (M1 + sM[1][nm]), m2 = 0.5 * (M2 + sM[2][nm]);
          const double B6[6] = {sp[0][nm], sp[1][nm], sp[2][nm], sp[3][nm], sp[4][nm], sp[5][nm]};
          double f[5];
          ec_flux_contra(A, B6, m0, m1, m2, ph.gm1, f);
#pragma unroll
          for (int v = 0; v < 5; ++v) ac[v] += Dm * f[v];
          if (VISC) {
#pragma unroll
            for (int c = 0; c < 4; ++c) av[c] += Dm * sfv[c][nm];
          }
        }
      } else {
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const int nm = base + step * m;
          const R Dm = static_cast<R>(sD[idx][m]);
          const R h = R(0.5);
          const R m0 = h * (M0 + sM[0][nm]), m1 = h * (M1 + sM[1][nm]), m2 = h * (M2 + sM[2][nm]);
          const R rho = h * (A[0] + sp[0][nm]);
          const R uu = h * (A[1] + sp[1][nm]);
          const R vv = h * (A[2] + sp[2][nm]);
          const R ww = h * (A[3] + sp[3][nm]);
          const R pp = h * (A[4] + sp[4][nm]);
          const R ee = h * (A[5] + sp[5][nm]);
          const R Uc = uu * m0 + vv * m1 + ww * m2;
          const R mass = rho * Uc;
          ac[0] += Dm * mass;
          ac[1] += Dm * (mass * uu + pp * m0);
          ac[2] += Dm * (mass * vv + pp * m1);
          ac[3] += Dm * (mass * ww + pp * m2);
          ac[4] += Dm * (mass * ee + pp * Uc);
          if (MIXED) du += Dm * Uc;
          if (VISC) {
#pragma unroll
            for (int c = 0; c < 4; ++c) av[c] += Dm * sfv[c][nm];
          }
        }
      }
      ut[0] -= 2.0 * static_cast<double>(ac[0]);
#pragma unroll
      for (int c = 0; c < 4; ++c) ut[1 + c] -= 2.0 * static_cast<double>(ac[1 + c]) - static_cast<double>(av[c]);
      if (MIXED)
        ut[4] -= 2.0 * (e_ref * static_cast<double>(ac[0]) + p_ref * static_cast<double>(du));
    }
    // The entropy-conserving instances (one workgroup per CU) need no barrier
    // after the last sweep: P4 reads and writes only the face entries of sX,
    // which no sweep reads.  (The Kennedy-Gruber ones, two workgroups per CU,
    // measured slower without it and with the early fetch below.)
    if (!EC || d < 2) __syncthreads();
  }

  // entropy-conserving instances: G and the own state of the RK update,
  // fetched now so that their latency overlaps the surface phase
  double gA[5] = {0, 0, 0, 0, 0}, u0[5] = {0, 0, 0, 0, 0};
  if (EC && RK && active) {
    if (st.read_G) {
#pragma unroll
      for (int v = 0; v < 5; ++v) gA[v] = load_once(&out[v * stride + e * NN + tid]);
    }
    load_state(U, stride, e * NN + tid, u0);
  }

  // P4: surface terms (face lanes); the neighbour index is formed again here
  // rather than held through the sweeps
  if (face_lane) {
    const FaceTask<N> ft(tid);
    const long long nb = neighbour(mesh, ex, ey, ez, ft.d, ft.up);
    const int lo = ft.own_node();
    // one normal per face: that of the element below it (own on an upper face,
    // the neighbour's on a lower face), so the two sides' fluxes are exact
    // negatives even where the face nodes of the two elements differ in
    // rounding (the periodic seam)
    // (a wall face has no element on its other side: the own normal)
    const bool fwall = nb < 0;
    double s[3];
    const long long ge = (ft.up || fwall) ? e : nb;
    const int gn = (ft.up || fwall) ? lo : ft.nb_node();
    if constexpr (MIXED) {
      // the sweeps read the FP32 copy, so the FP64 rows are not in L2 here:
      // the boundary-node copy is the smaller fetch
      constexpr int NFN = n_face_nodes<N>();
      const long long gi = ge * NFN + face_node_index<N>(gn % NP, (gn / NP) % NP, gn / NF);
#pragma unroll
      for (int c = 0; c < 3; ++c) s[c] = mesh.geoF[(3 * ft.d + c) * (nE * NFN) + gi];
    } else {
      // FP64: the gradient phase read these rows, mostly still in L2
#pragma unroll
      for (int c = 0; c < 3; ++c) s[c] = mesh.geo[(3 * ft.d + c) * stride + ge * NN + gn];
    }
    // the neighbour's face node, fetched again (a state of its own, so that
    // the one of the lifting phase is not held through the sweeps)
    double sn[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
    if (!fwall) load_state(U, stride, nb * NN + ft.nb_node(), sn);
    const Prim Pn = primitives(sn, ph);
    double Fo[5], Fs[5], vo[3];  // own contravariant Euler flux, surface flux, own velocity
    if constexpr (EC) {
      // FP64: sp holds (rho, u, v, w, beta, |u|^2): p = rho / (2 beta), E from p
      // and |u|^2; mixed precision: the own face node in FP64, from U
      double A6[6], po, Eo;
      if constexpr (MIXED) {
        double s5[5];
        load_state(U, stride, e * NN + lo, s5);
        const Prim Po = primitives(s5, ph);
        A6[0] = Po.rho; A6[1] = Po.u; A6[2] = Po.v; A6[3] = Po.w;
        A6[4] = 0.5 * Po.rho / Po.p;
        A6[5] = Po.u * Po.u + Po.v * Po.v + Po.w * Po.w;
        po = Po.p;
        Eo = s5[4];
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) A6[c] = sp[c][lo];
        po = 0.5 * A6[0] / A6[4];
        Eo = po / ph.gm1 + 0.5 * A6[0] * A6[5];
      }
      vo[0] = A6[1];
      vo[1] = A6[2];
      vo[2] = A6[3];
      const double Uo = A6[1] * s[0] + A6[2] * s[1] + A6[3] * s[2];
      Fo[0] = A6[0] * Uo;
      Fo[1] = A6[0] * A6[1] * Uo + po * s[0];
      Fo[2] = A6[0] * A6[2] * Uo + po * s[1];
      Fo[3] = A6[0] * A6[3] * Uo + po * s[2];
      Fo[4] = (Eo + po) * Uo;
      if (fwall) {  // impermeable wall: the interior pressure only
        Fs[0] = 0.0;
        Fs[1] = po * s[0];
        Fs[2] = po * s[1];
        Fs[3] = po * s[2];
        Fs[4] = 0.0;
      } else {
        // central part: Chandrashekar's flux contracted with the face normal
        const double B6[6] = {Pn.rho, Pn.u, Pn.v, Pn.w, 0.5 * Pn.rho / Pn.p, Pn.u * Pn.u + Pn.v * Pn.v + Pn.w * Pn.w};
        ec_flux_contra(A6, B6, s[0], s[1], s[2], ph.gm1, Fs);
        if (!ph.central) {
          const double smag = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
          const double ism = 1.0 / smag;
          const double n[3] = {s[0] * ism, s[1] * ism, s[2] * ism};
          const double Po5[5] = {A6[0], A6[1], A6[2], A6[3], po}, Pn5[5] = {Pn.rho, Pn.u, Pn.v, Pn.w, Pn.p};
          double Dr[5];
          // L = own on an upper face, the neighbour on a lower face
          if (ft.up)
            roe_dissipation_normal(Po5, Eo, Pn5, sn[4], n, ph.gamma, Dr);
          else
            roe_dissipation_normal(Pn5, sn[4], Po5, Eo, n, ph.gamma, Dr);
#pragma unroll
          for (int v = 0; v < 5; ++v) Fs[v] -= 0.5 * smag * Dr[v];
        }
      }
    } else {
      double Ao[6];
      if constexpr (MIXED) {  // the own face node in FP64, from U
        double s5[5];
        load_state(U, stride, e * NN + lo, s5);
        const Prim Po = primitives(s5, ph);
        Ao[0] = Po.rho; Ao[1] = Po.u; Ao[2] = Po.v; Ao[3] = Po.w; Ao[4] = Po.p; Ao[5] = Po.e;
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) Ao[c] = sp[c][lo];
      }
      const double An[6] = {Pn.rho, Pn.u, Pn.v, Pn.w, Pn.p, Pn.e};
      const double so[5] = {Ao[0], Ao[0] * Ao[1], Ao[0] * Ao[2], Ao[0] * Ao[3], Ao[0] * Ao[5]};
      vo[0] = Ao[1];
      vo[1] = Ao[2];
      vo[2] = Ao[3];
      const double Uo = Ao[1] * s[0] + Ao[2] * s[1] + Ao[3] * s[2];
      Fo[0] = Ao[0] * Uo;
      Fo[1] = Ao[0] * Ao[1] * Uo + Ao[4] * s[0];
      Fo[2] = Ao[0] * Ao[2] * Uo + Ao[4] * s[1];
      Fo[3] = Ao[0] * Ao[3] * Uo + Ao[4] * s[2];
      Fo[4] = (Ao[0] * Ao[5] + Ao[4]) * Uo;
      // central part: the contravariant Kennedy-Gruber flux of the two sides
      const double rho = 0.5 * (Ao[0] + An[0]), uu = 0.5 * (Ao[1] + An[1]), vv = 0.5 * (Ao[2] + An[2]);
      const double ww = 0.5 * (Ao[3] + An[3]), pp = 0.5 * (Ao[4] + An[4]), ee = 0.5 * (Ao[5] + An[5]);
      const double Uc = uu * s[0] + vv * s[1] + ww * s[2];
      const double mass = rho * Uc;
      Fs[0] = mass;
      Fs[1] = mass * uu + pp * s[0];
      Fs[2] = mass * vv + pp * s[1];
      Fs[3] = mass * ww + pp * s[2];
      Fs[4] = mass * ee + pp * Uc;
      if (fwall) {  // impermeable wall: the interior pressure only
        Fs[0] = 0.0;
        Fs[1] = Ao[4] * s[0];
        Fs[2] = Ao[4] * s[1];
        Fs[3] = Ao[4] * s[2];
        Fs[4] = 0.0;
      } else if (!ph.central) {
        const double smag = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        const double co = sqrt(ph.gamma * Ao[4] / Ao[0]), cn = sqrt(ph.gamma * An[4] / An[0]);
        const double uno = Uo / smag, unn = (An[1] * s[0] + An[2] * s[1] + An[3] * s[2]) / smag;
        // L = own on an upper face, the neighbour on a lower face; ties go to L
        const double lo_l = ft.up ? fabs(uno) + co : fabs(unn) + cn;
        const double lo_r = ft.up ? fabs(unn) + cn : fabs(uno) + co;
        const double lam = lo_r > lo_l ? lo_r : lo_l;
        const double h = 0.5 * lam * smag * (ft.up ? 1.0 : -1.0);
#pragma unroll
        for (int v = 0; v < 5; ++v) Fs[v] -= h * (sn[v] - so[v]);
      }
    }
    double fvo[4] = {0, 0, 0, 0}, fvs[4] = {0, 0, 0, 0};
    if (VISC) {
#pragma unroll
      for (int c = 0; c < 4; ++c) fvo[c] = sX[ft.f][c][ft.ab];
      if (fwall) {
        // zero wall velocity with the interior gradients: the own stresses,
        // and of the energy flux only the heat flux
#pragma unroll
        for (int c = 0; c < 3; ++c) fvs[c] = fvo[c];
        fvs[3] = fvo[3] - (vo[0] * fvo[0] + vo[1] * fvo[1] + vo[2] * fvo[2]);
      } else {
        const R* src = ffv + nb * (6 * 4 * NF) + ((ft.f ^ 1) * 4) * NF + ft.ab;
#pragma unroll
        for (int c = 0; c < 4; ++c) fvs[c] = 0.5 * (fvo[c] + static_cast<double>(load_once(&src[c * NF])));
      }
    }
    const double sc = ft.up ? basis.inv_w_end : -basis.inv_w_end;
    double corr5[5];
    corr5[0] = sc * (Fs[0] - Fo[0]);
#pragma unroll
    for (int c = 0; c < 4; ++c) corr5[1 + c] = sc * ((Fs[1 + c] - fvs[c]) - (Fo[1 + c] - fvo[c]));
#pragma unroll
    for (int v = 0; v < 5; ++v) sX[ft.f][v][ft.ab] = corr5[v];
  }
  __syncthreads();

  // P5: surface terms, 1/J, output
  if (active) {
    const double invJ = KEEP && !MIXED ? static_cast<double>(Jr[9]) : mesh.geo[9 * stride + e * NN + tid];
    if (!EC && RK && st.read_G) {
#pragma unroll
      for (int v = 0; v < 5; ++v) gA[v] = load_once(&out[v * stride + e * NN + tid]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double c = 0.0;
      if (i == 0) c += sX[0][v][j + NP * k];
      if (i == N) c += sX[1][v][j + NP * k];
      if (j == 0) c += sX[2][v][i + NP * k];
      if (j == N) c += sX[3][v][i + NP * k];
      if (k == 0) c += sX[4][v][i + NP * j];
      if (k == N) c += sX[5][v][i + NP * j];
      ut[v] = invJ * (ut[v] - c);
    }
    const long long idx = e * NN + tid;
    if (RK) {
      if (!EC) load_state(U, stride, idx, u0);  // read again: holding it from P1 spills
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double gv = st.A * gA[v] + st.dt * ut[v];
        store_once(&out[v * stride + idx], gv);
        store_once(&U_out[v * stride + idx], u0[v] + st.B * gv);
      }
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) store_once(&out[v * stride + idx], ut[v]);
    }
  }
}

template <int N>
hipError_t metrics_n(const double* X, double* geo, double* geoF, bool with_f32, const DevBasis& b,
                     long long nE, int* status, hipStream_t s) {
  hipLaunchKernelGGL((k_metrics<N>), dim3(static_cast<unsigned>(nE)), dim3(CurvCfg<N>::BS), 0, s, X, geo,
                     geoF, with_f32, b, nE, status);
  return hipGetLastError();
}

template <int N, typename R>
hipError_t face_flux_curv_n(const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                            void* ffv, hipStream_t s) {
  hipLaunchKernelGGL((k_face_flux_curv<N, R>), dim3(static_cast<unsigned>(m.nE)), dim3(CurvCfg<N>::BS), 0, s,
                     U, static_cast<R*>(ffv), m, p, b);
  return hipGetLastError();
}

template <int N, typename R, bool RK>
hipError_t rhs_curv_n(const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                      const void* ffv_, double* out, double* U_out, const Stage& st, int* status,
                      hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(m.nE)), block(CurvCfg<N>::BS);
  const R* ffv = static_cast<const R*>(ffv_);
  if constexpr (sizeof(R) == sizeof(double)) {
    if (p.ec) {
      if (p.viscous)
        hipLaunchKernelGGL((k_rhs_curv<N, R, RK, true, true>), grid, block, 0, s, U, ffv, out, U_out, m, p, b,
                           st, status);
      else
        hipLaunchKernelGGL((k_rhs_curv<N, R, RK, false, true>), grid, block, 0, s, U, ffv, out, U_out, m, p, b,
                           st, status);
      return hipGetLastError();
    }
  } else {
    if (p.ec) {
      if (!p.mixed_ref) return hipErrorInvalidValue;  // rejected at init: needs the reference state
      if (p.viscous)
        hipLaunchKernelGGL((k_rhs_curv<N, R, RK, true, true>), grid, block, 0, s, U, ffv, out, U_out, m, p, b,
                           st, status);
      else
        hipLaunchKernelGGL((k_rhs_curv<N, R, RK, false, true>), grid, block, 0, s, U, ffv, out, U_out, m, p, b,
                           st, status);
      return hipGetLastError();
    }
  }
  if (p.viscous)
    hipLaunchKernelGGL((k_rhs_curv<N, R, RK, true, false>), grid, block, 0, s, U, ffv, out, U_out, m, p, b, st,
                       status);
  else
    hipLaunchKernelGGL((k_rhs_curv<N, R, RK, false, false>), grid, block, 0, s, U, ffv, out, U_out, m, p, b, st,
                       status);
  return hipGetLastError();
}

template <typename R, bool RK>
hipError_t rhs_curv_dispatch(int N, const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                             const void* ffv, double* out, double* U_out, const Stage& st, int* status,
                             hipStream_t s) {
  switch (N) {
    case 3: return rhs_curv_n<3, R, RK>(m, p, b, U, ffv, out, U_out, st, status, s);
    case 5: return rhs_curv_n<5, R, RK>(m, p, b, U, ffv, out, U_out, st, status, s);
    case 7: return rhs_curv_n<7, R, RK>(m, p, b, U, ffv, out, U_out, st, status, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_metrics(int N, const double* X, double* geo, double* geoF, bool with_f32,
                          const DevBasis& b, long long nE, int* status, hipStream_t s) {
  switch (N) {
    case 3: return metrics_n<3>(X, geo, geoF, with_f32, b, nE, status, s);
    case 5: return metrics_n<5>(X, geo, geoF, with_f32, b, nE, status, s);
    case 7: return metrics_n<7>(X, geo, geoF, with_f32, b, nE, status, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_face_flux_curv(int N, int precision, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                                 const double* U, void* ffv, hipStream_t s) {
  const bool f32 = precision != DG_FP64;
  switch (N) {
    case 3: return f32 ? face_flux_curv_n<3, float>(m, p, b, U, ffv, s) : face_flux_curv_n<3, double>(m, p, b, U, ffv, s);
    case 5: return f32 ? face_flux_curv_n<5, float>(m, p, b, U, ffv, s) : face_flux_curv_n<5, double>(m, p, b, U, ffv, s);
    case 7: return f32 ? face_flux_curv_n<7, float>(m, p, b, U, ffv, s) : face_flux_curv_n<7, double>(m, p, b, U, ffv, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rhs_curv(int N, int precision, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                           const double* U, const void* ffv, double* Ut, int* status, hipStream_t s) {
  const Stage st{0.0, 0.0, 0.0, 0};
  return precision != DG_FP64
             ? rhs_curv_dispatch<float, false>(N, m, p, b, U, ffv, Ut, nullptr, st, status, s)
             : rhs_curv_dispatch<double, false>(N, m, p, b, U, ffv, Ut, nullptr, st, status, s);
}

hipError_t launch_rk_stage_curv(int N, int precision, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                                const double* U, const void* ffv, double* G, double* U_out,
                                const Stage& st, int* status, hipStream_t s) {
  return precision != DG_FP64
             ? rhs_curv_dispatch<float, true>(N, m, p, b, U, ffv, G, U_out, st, status, s)
             : rhs_curv_dispatch<double, true>(N, m, p, b, U, ffv, G, U_out, st, status, s);
}

}  // namespace dg
