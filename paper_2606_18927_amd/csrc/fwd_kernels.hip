// Forward kernels of the split-form DGSEM operator for gfx950.
//
// One workgroup owns EPB whole elements ((N+1)^3 nodes each, one lane per
// node).  Per stage two kernels run:
//
//   k_lift : U (+ the neighbours' face planes of U)  ->  grad(u, v, w, T)
//            BR1 lifting (paper Sec. 2.2 scheme, viscous part of Sec. 4);
//   k_rhs  : U, grad (+ the neighbours' face planes)  ->  Ut, or the fused
//            low-storage RK update G <- A G + dt Ut, U' <- U + B G (Sec. 4).
//
// Data flow inside a workgroup (both kernels):
//   phase 1  each lane loads its node (SoA, coalesced), recovers the
//            primitives in FP64 and stages them in LDS;
//   phase 2  face tasks: one lane per face node of each of the 6 faces
//            (6 (N+1)^2 tasks per element) computes the surface correction
//            against the neighbour's face node (or the wall state) and
//            stores it in LDS, so the surface work is spread over the
//            workgroup instead of diverging inside the volume sweeps;
//   phase 3  tensor-product line sweeps along x, y and z over the LDS block
//            (derivative matrix D in LDS);
//   phase 4  the surface corrections of nodes on faces are added, the sum is
//            scaled by s_d = 2 / width_d and written (or fed to the RK update).
//
// Workgroup ids are remapped so that each of the 8 XCDs (own L2) works on one
// contiguous range of elements: face neighbours in x are consecutive element
// ids and then tend to hit in the same L2.
#include "dg_internal.hpp"

namespace dg {
namespace {

template <int N>
struct Cfg;
template <>
struct Cfg<3> {
  static constexpr int EPB = 4, BS = 256;
};
template <>
struct Cfg<5> {
  static constexpr int EPB = 1, BS = 256;
};
template <>
struct Cfg<7> {
  static constexpr int EPB = 1, BS = 512;
};

template <int N>
struct Geo {
  static constexpr int NP = N + 1, NF = NP * NP, NN = NF * NP;
  static constexpr int RS = NP + 1;        // padded x-row stride of the LDS block
  static constexpr int EB = RS * NP * NP;  // LDS doubles per element and field
  __device__ static constexpr int lds(int i, int j, int k) { return i + RS * (j + NP * k); }
};

// Workgroup b of nb -> element block, so that XCD x = b % 8 covers one
// contiguous range of blocks (bijective for any nb).
__device__ inline int xcd_remap(int b, int nb) {
  constexpr int X = 8;
  const int q = nb / X, r = nb % X;
  const int x = b % X, l = b / X;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

__device__ inline void elem_coords(long long e, const DevMesh& m, int& ex, int& ey, int& ez) {
  ex = static_cast<int>(e % m.n[0]);
  const long long t = e / m.n[0];
  ey = static_cast<int>(t % m.n[1]);
  ez = static_cast<int>(t / m.n[1]);
}

// Face neighbour of element (ex, ey, ez) across its lower (up = false) or
// upper face normal to d; -1 on a wall.
__device__ inline long long neighbour(const DevMesh& m, int ex, int ey, int ez, int d, bool up) {
  int c[3] = {ex, ey, ez};
  int v = c[d] + (up ? 1 : -1);
  if (v < 0 || v >= m.n[d]) {
    if (m.bc[d] != DG_BC_PERIODIC) return -1;
    v = (v + m.n[d]) % m.n[d];
  }
  c[d] = v;
  return c[0] + static_cast<long long>(m.n[0]) * (c[1] + static_cast<long long>(m.n[1]) * c[2]);
}

// Node (i, j, k) of face (d, up) with in-face coordinates (a, b).
template <int N>
__device__ inline void face_node(int d, bool up, int a, int b, int& i, int& j, int& k) {
  const int n = up ? N : 0;
  if (d == 0) {
    i = n; j = a; k = b;
  } else if (d == 1) {
    i = a; j = n; k = b;
  } else {
    i = a; j = b; k = n;
  }
}

struct Prim {
  double rho, u, v, w, p, e;
};

// Ideal-gas primitive recovery, always FP64.
__device__ inline Prim primitives(double r, double mx, double my, double mz, double E,
                                  const DevPhys& ph) {
  Prim P;
  const double ir = 1.0 / r;
  P.rho = r;
  P.u = mx * ir;
  P.v = my * ir;
  P.w = mz * ir;
  P.p = ph.gm1 * (E - 0.5 * r * (P.u * P.u + P.v * P.v + P.w * P.w));
  P.e = E * ir;
  return P;
}

__device__ inline void load_state(const double* U, long long stride, long long idx, double u[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = U[v * stride + idx];
}

// Kennedy-Gruber two-point flux along d of states a, b = (rho, u, v, w, p, e).
template <int d, typename R>
__device__ inline void kg_flux(const R a[6], const R b[6], R f[5]) {
  const R h = R(0.5);
  const R rho = h * (a[0] + b[0]);
  const R ud = h * (a[1 + d] + b[1 + d]);
  const R p = h * (a[4] + b[4]);
  const R e = h * (a[5] + b[5]);
  const R mass = rho * ud;
  f[0] = mass;
  f[1] = mass * (h * (a[1] + b[1]));
  f[2] = mass * (h * (a[2] + b[2]));
  f[3] = mass * (h * (a[3] + b[3]));
  f[1 + d] += p;
  f[4] = mass * e + p * ud;
}

// Euler flux along d of a = (rho, u, v, w, p, e).
template <typename R>
__device__ inline void euler_flux(int d, const R a[6], R f[5]) {
  const R ud = a[1 + d];
  const R mass = a[0] * ud;
  f[0] = mass;
  f[1] = mass * a[1];
  f[2] = mass * a[2];
  f[3] = mass * a[3];
  f[1 + d] += a[4];
  f[4] = (a[0] * a[5] + a[4]) * ud;
}

// Viscous flux along d: g[3 q + b] = d q / d x_b for q in (u, v, w, T);
// returns (tau_1d, tau_2d, tau_3d, u_a tau_ad + kappa dT/dx_d).
template <typename R>
__device__ inline void viscous_flux(int d, R u, R v, R w, const R g[12], R mu, R kappa, R f[4]) {
  const R div = g[0] + g[4] + g[8];
  R t0 = mu * (g[0 * 3 + d] + g[d * 3 + 0]);
  R t1 = mu * (g[1 * 3 + d] + g[d * 3 + 1]);
  R t2 = mu * (g[2 * 3 + d] + g[d * 3 + 2]);
  const R dd = R(2.0 / 3.0) * mu * div;
  if (d == 0) t0 -= dd;
  if (d == 1) t1 -= dd;
  if (d == 2) t2 -= dd;
  f[0] = t0;
  f[1] = t1;
  f[2] = t2;
  f[3] = u * t0 + v * t1 + w * t2 + kappa * g[9 + d];
}

// --------------------------------------------------------------------------
// k_lift
// --------------------------------------------------------------------------
template <int N, typename R>
__global__ __launch_bounds__(Cfg<N>::BS) void k_lift(const double* __restrict__ U,
                                                      R* __restrict__ grad, DevMesh mesh,
                                                      DevPhys ph, DevBasis basis) {
  using Gm = Geo<N>;
  constexpr int NP = Gm::NP, NF = Gm::NF, NN = Gm::NN, EB = Gm::EB;
  constexpr int EPB = Cfg<N>::EPB, BS = Cfg<N>::BS;
  __shared__ R sD[NP * NP];
  __shared__ R sq[EPB][4][EB];
  __shared__ R ssf[EPB][6][4][NF];

  const int tid = threadIdx.x;
  const long long nE = mesh.nE;
  const long long stride = nE * NN;
  const long long e0 = static_cast<long long>(xcd_remap(blockIdx.x, gridDim.x)) * EPB;
  for (int t = tid; t < NP * NP; t += BS) sD[t] = static_cast<R>(basis.D[t]);

  const int le = tid / NN;
  const int node = tid - le * NN;
  const long long e = e0 + le;
  const bool active = le < EPB && e < nE;
  const int i = node % NP, j = (node / NP) % NP, k = node / NF;

  if (active) {
    double s[5];
    load_state(U, stride, e * NN + node, s);
    const Prim P = primitives(s[0], s[1], s[2], s[3], s[4], ph);
    const int l = Gm::lds(i, j, k);
    sq[le][0][l] = static_cast<R>(P.u);
    sq[le][1][l] = static_cast<R>(P.v);
    sq[le][2][l] = static_cast<R>(P.w);
    sq[le][3][l] = static_cast<R>(P.p * ph.inv_R / P.rho);
  }
  __syncthreads();

  // face tasks: BR1 surface values q* = (q_own + q_nb)/2, or the wall value
  for (int t = tid; t < EPB * 6 * NF; t += BS) {
    const int tle = t / (6 * NF);
    const int rr = t - tle * 6 * NF;
    const int f = rr / NF;
    const int ab = rr - f * NF;
    const long long te = e0 + tle;
    if (te >= nE) continue;
    const int d = f >> 1;
    const bool up = (f & 1) != 0;
    int oi, oj, ok;
    face_node<N>(d, up, ab % NP, ab / NP, oi, oj, ok);
    int ex, ey, ez;
    elem_coords(te, mesh, ex, ey, ez);
    const long long nb = neighbour(mesh, ex, ey, ez, d, up);
    const int lo = Gm::lds(oi, oj, ok);
    R qo[4], qs[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) qo[c] = sq[tle][c][lo];
    if (nb < 0) {
      qs[0] = qs[1] = qs[2] = R(0);
      qs[3] = static_cast<R>(mesh.T_wall);
    } else {
      int ni = oi, nj = oj, nk = ok;
      const int opp = up ? 0 : N;
      if (d == 0) ni = opp;
      if (d == 1) nj = opp;
      if (d == 2) nk = opp;
      double s[5];
      load_state(U, stride, nb * NN + ni + NP * (nj + NP * nk), s);
      const Prim P = primitives(s[0], s[1], s[2], s[3], s[4], ph);
      const R qn[4] = {static_cast<R>(P.u), static_cast<R>(P.v), static_cast<R>(P.w),
                       static_cast<R>(P.p * ph.inv_R / P.rho)};
#pragma unroll
      for (int c = 0; c < 4; ++c) qs[c] = R(0.5) * (qo[c] + qn[c]);
    }
    const R sc = static_cast<R>(up ? basis.inv_w_end : -basis.inv_w_end);
#pragma unroll
    for (int c = 0; c < 4; ++c) ssf[tle][f][c][ab] = (qs[c] - qo[c]) * sc;
  }
  __syncthreads();

  if (active) {
    int ex, ey, ez;
    elem_coords(e, mesh, ex, ey, ez);
    const R sx = static_cast<R>(mesh.s[0][ex]);
    const R sy = static_cast<R>(mesh.s[1][ey]);
    const R sz = static_cast<R>(mesh.s[2][ez]);
    R* ge = grad + e * NN + node;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      R ax = R(0), ay = R(0), az = R(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        ax += sD[i * NP + m] * sq[le][c][Gm::lds(m, j, k)];
        ay += sD[j * NP + m] * sq[le][c][Gm::lds(i, m, k)];
        az += sD[k * NP + m] * sq[le][c][Gm::lds(i, j, m)];
      }
      if (i == 0) ax += ssf[le][0][c][j + NP * k];
      if (i == N) ax += ssf[le][1][c][j + NP * k];
      if (j == 0) ay += ssf[le][2][c][i + NP * k];
      if (j == N) ay += ssf[le][3][c][i + NP * k];
      if (k == 0) az += ssf[le][4][c][i + NP * j];
      if (k == N) az += ssf[le][5][c][i + NP * j];
      ge[(3 * c + 0) * stride] = sx * ax;
      ge[(3 * c + 1) * stride] = sy * ay;
      ge[(3 * c + 2) * stride] = sz * az;
    }
  }
}

// --------------------------------------------------------------------------
// k_rhs
// --------------------------------------------------------------------------
template <int N, typename R, int d>
__device__ inline void volume_sweep(const R (&own)[6], int i, int j, int k, const R* sD,
                                    const R (*sp)[Geo<N>::EB], const R (*sfv)[Geo<N>::EB],
                                    bool viscous, R ac[5], R av[4]) {
  using Gm = Geo<N>;
  constexpr int NP = Gm::NP;
  const int idx = d == 0 ? i : (d == 1 ? j : k);
#pragma unroll
  for (int v = 0; v < 5; ++v) ac[v] = R(0);
#pragma unroll
  for (int c = 0; c < 4; ++c) av[c] = R(0);
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int lm = d == 0 ? Gm::lds(m, j, k) : (d == 1 ? Gm::lds(i, m, k) : Gm::lds(i, j, m));
    const R Dim = sD[idx * NP + m];
    R b[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) b[q] = sp[q][lm];
    R f[5];
    kg_flux<d, R>(own, b, f);
#pragma unroll
    for (int v = 0; v < 5; ++v) ac[v] += Dim * f[v];
    if (viscous) {
#pragma unroll
      for (int c = 0; c < 4; ++c) av[c] += Dim * sfv[c][lm];
    }
  }
}

template <int N, typename R, bool RK>
__global__ __launch_bounds__(Cfg<N>::BS) void k_rhs(const double* __restrict__ U,
                                                     const R* __restrict__ grad,
                                                     double* __restrict__ out,
                                                     double* __restrict__ U_out, DevMesh mesh,
                                                     DevPhys ph, DevBasis basis, Stage st,
                                                     int* __restrict__ status) {
  using Gm = Geo<N>;
  constexpr int NP = Gm::NP, NF = Gm::NF, NN = Gm::NN, EB = Gm::EB;
  constexpr int EPB = Cfg<N>::EPB, BS = Cfg<N>::BS;
  __shared__ R sD[NP * NP];
  __shared__ R sp[EPB][6][EB];      // rho, u, v, w, p, e
  __shared__ R sfv[EPB][4][EB];     // viscous flux of the current direction
  __shared__ R ssf[EPB][6][5][NF];  // surface corrections per face node

  const int tid = threadIdx.x;
  const long long nE = mesh.nE;
  const long long stride = nE * NN;
  const long long e0 = static_cast<long long>(xcd_remap(blockIdx.x, gridDim.x)) * EPB;
  for (int t = tid; t < NP * NP; t += BS) sD[t] = static_cast<R>(basis.D[t]);
  const bool viscous = ph.viscous != 0;
  const R mu = static_cast<R>(ph.mu), kappa = static_cast<R>(ph.kappa);

  const int le = tid / NN;
  const int node = tid - le * NN;
  const long long e = e0 + le;
  const bool active = le < EPB && e < nE;
  const int i = node % NP, j = (node / NP) % NP, k = node / NF;
  const int l = Gm::lds(i, j, k);

  // phase 1: own node
  double u0[5] = {0, 0, 0, 0, 0};
  R own[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  R g[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) g[c] = R(0);
  if (active) {
    load_state(U, stride, e * NN + node, u0);
    const Prim P = primitives(u0[0], u0[1], u0[2], u0[3], u0[4], ph);
    if (!(P.rho > 0.0) || !(P.p > 0.0)) status[0] = 1;
    own[0] = static_cast<R>(P.rho);
    own[1] = static_cast<R>(P.u);
    own[2] = static_cast<R>(P.v);
    own[3] = static_cast<R>(P.w);
    own[4] = static_cast<R>(P.p);
    own[5] = static_cast<R>(P.e);
#pragma unroll
    for (int q = 0; q < 6; ++q) sp[le][q][l] = own[q];
    if (viscous) {
#pragma unroll
      for (int c = 0; c < 12; ++c) g[c] = grad[c * stride + e * NN + node];
    }
  }
  __syncthreads();

  // phase 2: face tasks
  for (int t = tid; t < EPB * 6 * NF; t += BS) {
    const int tle = t / (6 * NF);
    const int rr = t - tle * 6 * NF;
    const int f = rr / NF;
    const int ab = rr - f * NF;
    const long long te = e0 + tle;
    if (te >= nE) continue;
    const int d = f >> 1;
    const bool up = (f & 1) != 0;
    int oi, oj, ok;
    face_node<N>(d, up, ab % NP, ab / NP, oi, oj, ok);
    int ex, ey, ez;
    elem_coords(te, mesh, ex, ey, ez);
    const long long nb = neighbour(mesh, ex, ey, ez, d, up);
    const long long oidx = te * NN + oi + NP * (oj + NP * ok);

    double us[5];
    load_state(U, stride, oidx, us);
    const Prim Po = primitives(us[0], us[1], us[2], us[3], us[4], ph);
    const R a[6] = {static_cast<R>(Po.rho), static_cast<R>(Po.u), static_cast<R>(Po.v),
                    static_cast<R>(Po.w), static_cast<R>(Po.p), static_cast<R>(Po.e)};
    R go[12];
    R fvo[4] = {R(0), R(0), R(0), R(0)};
    if (viscous) {
#pragma unroll
      for (int c = 0; c < 12; ++c) go[c] = grad[c * stride + oidx];
      viscous_flux<R>(d, a[1], a[2], a[3], go, mu, kappa, fvo);
    }
    R fco[5];
    euler_flux<R>(d, a, fco);

    R Fs[5];  // F*_c - F*_v
    if (nb < 0) {
      // isothermal no-slip wall: pressure-only convective flux, viscous flux
      // with zero wall velocity and the interior gradients
      Fs[0] = R(0);
      Fs[1] = Fs[2] = Fs[3] = R(0);
      Fs[1 + d] = a[4];
      Fs[4] = R(0);
      if (viscous) {
        R fw[4];
        viscous_flux<R>(d, R(0), R(0), R(0), go, mu, kappa, fw);
#pragma unroll
        for (int c = 0; c < 4; ++c) Fs[1 + c] -= fw[c];
      }
    } else {
      int ni = oi, nj = oj, nk = ok;
      const int opp = up ? 0 : N;
      if (d == 0) ni = opp;
      if (d == 1) nj = opp;
      if (d == 2) nk = opp;
      const long long nidx = nb * NN + ni + NP * (nj + NP * nk);
      double un[5];
      load_state(U, stride, nidx, un);
      const Prim Pn = primitives(un[0], un[1], un[2], un[3], un[4], ph);
      const R b[6] = {static_cast<R>(Pn.rho), static_cast<R>(Pn.u), static_cast<R>(Pn.v),
                      static_cast<R>(Pn.w), static_cast<R>(Pn.p), static_cast<R>(Pn.e)};
      R fc[5];
      if (d == 0) kg_flux<0, R>(a, b, fc);
      if (d == 1) kg_flux<1, R>(a, b, fc);
      if (d == 2) kg_flux<2, R>(a, b, fc);
      if (!ph.central) {
        const double cu = fabs((d == 0) ? Po.u : (d == 1) ? Po.v : Po.w) +
                          sqrt(ph.gamma * Po.p / Po.rho);
        const double cn = fabs((d == 0) ? Pn.u : (d == 1) ? Pn.v : Pn.w) +
                          sqrt(ph.gamma * Pn.p / Pn.rho);
        const R lam = static_cast<R>(cu >= cn ? cu : cn);
        // -lambda/2 (U_R - U_L) with L the lower side of the face
        const R sgn = up ? R(-0.5) : R(0.5);
#pragma unroll
        for (int v = 0; v < 5; ++v) fc[v] += sgn * lam * static_cast<R>(un[v] - us[v]);
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) Fs[v] = fc[v];
      if (viscous) {
        R gn[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) gn[c] = grad[c * stride + nidx];
        R fvn[4];
        viscous_flux<R>(d, b[1], b[2], b[3], gn, mu, kappa, fvn);
#pragma unroll
        for (int c = 0; c < 4; ++c) Fs[1 + c] -= R(0.5) * (fvo[c] + fvn[c]);
      }
    }
    const R sc = static_cast<R>(up ? basis.inv_w_end : -basis.inv_w_end);
    ssf[tle][f][0][ab] = (Fs[0] - fco[0]) * sc;
#pragma unroll
    for (int c = 0; c < 4; ++c) ssf[tle][f][1 + c][ab] = (Fs[1 + c] - (fco[1 + c] - fvo[c])) * sc;
  }

  // phase 3: line sweeps, one direction at a time (the viscous flux of the
  // direction is staged in LDS, then differentiated along the lines)
  double ut[5] = {0, 0, 0, 0, 0};
  int ex = 0, ey = 0, ez = 0;
  if (active) elem_coords(e, mesh, ex, ey, ez);

#define DG_DIRECTION(D)                                                                   \
  {                                                                                       \
    if (active && viscous) {                                                              \
      R fv[4];                                                                            \
      viscous_flux<R>(D, own[1], own[2], own[3], g, mu, kappa, fv);                       \
      for (int c = 0; c < 4; ++c) sfv[le][c][l] = fv[c];                                  \
    }                                                                                     \
    __syncthreads();                                                                      \
    if (active) {                                                                         \
      R ac[5], av[4];                                                                     \
      volume_sweep<N, R, D>(own, i, j, k, sD, sp[le], sfv[le], viscous, ac, av);          \
      const int idx = D == 0 ? i : (D == 1 ? j : k);                                      \
      const int ab = D == 0 ? j + NP * k : (D == 1 ? i + NP * k : i + NP * j);            \
      R sf[5] = {R(0), R(0), R(0), R(0), R(0)};                                           \
      if (idx == 0)                                                                       \
        for (int v = 0; v < 5; ++v) sf[v] += ssf[le][2 * D][v][ab];                       \
      if (idx == N)                                                                       \
        for (int v = 0; v < 5; ++v) sf[v] += ssf[le][2 * D + 1][v][ab];                   \
      const double sd = mesh.s[D][D == 0 ? ex : (D == 1 ? ey : ez)];                       \
      ut[0] -= sd * static_cast<double>(R(2) * ac[0] + sf[0]);                            \
      for (int c = 0; c < 4; ++c)                                                         \
        ut[1 + c] -= sd * static_cast<double>(R(2) * ac[1 + c] - av[c] + sf[1 + c]);      \
    }                                                                                     \
    __syncthreads();                                                                      \
  }
  DG_DIRECTION(0)
  DG_DIRECTION(1)
  DG_DIRECTION(2)
#undef DG_DIRECTION

  // phase 4: write Ut or apply the low-storage RK stage
  if (active) {
    const long long idx = e * NN + node;
    if (RK) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double gv = (st.read_G ? st.A * out[v * stride + idx] : 0.0) + st.dt * ut[v];
        out[v * stride + idx] = gv;
        U_out[v * stride + idx] = u0[v] + st.B * gv;
      }
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) out[v * stride + idx] = ut[v];
    }
  }
}

template <int N>
int n_blocks(long long nE) {
  return static_cast<int>((nE + Cfg<N>::EPB - 1) / Cfg<N>::EPB);
}

template <int N, typename R>
hipError_t lift_n(const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                  void* grad, hipStream_t s) {
  hipLaunchKernelGGL((k_lift<N, R>), dim3(n_blocks<N>(m.nE)), dim3(Cfg<N>::BS), 0, s, U,
                     static_cast<R*>(grad), m, p, b);
  return hipGetLastError();
}

template <int N, typename R, bool RK>
hipError_t rhs_n(const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                 const void* grad, double* out, double* U_out, const Stage& st, int* status,
                 hipStream_t s) {
  hipLaunchKernelGGL((k_rhs<N, R, RK>), dim3(n_blocks<N>(m.nE)), dim3(Cfg<N>::BS), 0, s, U,
                     static_cast<const R*>(grad), out, U_out, m, p, b, st, status);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lift(int N, int precision, const DevMesh& m, const DevPhys& p,
                       const DevBasis& b, const double* U, void* grad, hipStream_t s) {
  if (m.nE <= 0) return hipSuccess;
  const bool f32 = precision == DG_MIXED;
  switch (N) {
    case 3: return f32 ? lift_n<3, float>(m, p, b, U, grad, s) : lift_n<3, double>(m, p, b, U, grad, s);
    case 5: return f32 ? lift_n<5, float>(m, p, b, U, grad, s) : lift_n<5, double>(m, p, b, U, grad, s);
    case 7: return f32 ? lift_n<7, float>(m, p, b, U, grad, s) : lift_n<7, double>(m, p, b, U, grad, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rhs(int N, int precision, const DevMesh& m, const DevPhys& p,
                      const DevBasis& b, const double* U, const void* grad, double* Ut,
                      int* status, hipStream_t s) {
  if (m.nE <= 0) return hipSuccess;
  const bool f32 = precision == DG_MIXED;
  const Stage st{0.0, 0.0, 0.0, 0};
  switch (N) {
    case 3: return f32 ? rhs_n<3, float, false>(m, p, b, U, grad, Ut, nullptr, st, status, s)
                       : rhs_n<3, double, false>(m, p, b, U, grad, Ut, nullptr, st, status, s);
    case 5: return f32 ? rhs_n<5, float, false>(m, p, b, U, grad, Ut, nullptr, st, status, s)
                       : rhs_n<5, double, false>(m, p, b, U, grad, Ut, nullptr, st, status, s);
    case 7: return f32 ? rhs_n<7, float, false>(m, p, b, U, grad, Ut, nullptr, st, status, s)
                       : rhs_n<7, double, false>(m, p, b, U, grad, Ut, nullptr, st, status, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rk_stage(int N, int precision, const DevMesh& m, const DevPhys& p,
                           const DevBasis& b, const double* U, const void* grad, double* G,
                           double* U_out, const Stage& st, int* status, hipStream_t s) {
  if (m.nE <= 0) return hipSuccess;
  const bool f32 = precision == DG_MIXED;
  switch (N) {
    case 3: return f32 ? rhs_n<3, float, true>(m, p, b, U, grad, G, U_out, st, status, s)
                       : rhs_n<3, double, true>(m, p, b, U, grad, G, U_out, st, status, s);
    case 5: return f32 ? rhs_n<5, float, true>(m, p, b, U, grad, G, U_out, st, status, s)
                       : rhs_n<5, double, true>(m, p, b, U, grad, G, U_out, st, status, s);
    case 7: return f32 ? rhs_n<7, float, true>(m, p, b, U, grad, G, U_out, st, status, s)
                       : rhs_n<7, double, true>(m, p, b, U, grad, G, U_out, st, status, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dg
