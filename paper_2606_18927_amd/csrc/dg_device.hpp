// Device helpers shared by the forward, lifting and adjoint kernels.
#pragma once

#include "dg_internal.hpp"

namespace dg {

// Workgroup shape per polynomial degree: EPB whole elements per workgroup,
// BS lanes, one lane per node and (in the face phases) one lane per face node:
// BS >= EPB (N+1)^3 and BS >= EPB 6 (N+1)^2.
template <int N>
struct Cfg;
template <>
struct Cfg<3> {
  // EPB elements per workgroup of BS lanes; FACE_WAVES: waves per SIMD the
  // face-flux kernel is register-bounded for
  static constexpr int EPB = 2, BS = 192, FACE_WAVES = 4;
};
template <>
struct Cfg<5> {
  static constexpr int EPB = 1, BS = 256, FACE_WAVES = 8;
};
template <>
struct Cfg<7> {
  static constexpr int EPB = 1, BS = 512, FACE_WAVES = 8;
};

// LDS block of one element and field: x-rows of RS entries (NP + PAD); with
// SWZ (NP a power of two, no padding) node i of row j sits at slot i ^ j of
// its row, so the NP rows that the lanes of a wave read at one x-position m
// (an x-line sweep) start in different banks, while a y- or z-line sweep
// still reads whole rows (a permutation of them).
template <int N, int PAD = 1, bool SWZ = false>
struct Geo {
  static constexpr int NP = N + 1, NF = NP * NP, NN = NF * NP;
  static constexpr int RS = NP + PAD;      // x-row stride of an LDS block
  static constexpr int EB = RS * NP * NP;  // LDS entries per element and field
  static constexpr int DS = NP + 1;        // padded row stride of D in LDS
  static_assert(!SWZ || (PAD == 0 && (NP & (NP - 1)) == 0), "the swizzle permutes unpadded rows of 2^n");
  __device__ static constexpr int lds(int i, int j, int k) {
    return (SWZ ? (i ^ (j & (NP - 1))) : i) + RS * (j + NP * k);
  }
};

template <int N>
__host__ __device__ constexpr int n_face_tasks() {
  return Cfg<N>::EPB * 6 * (N + 1) * (N + 1);
}

// Workgroup b of nb -> element block, so that XCD x = b % 8 (each XCD has its
// own L2) covers one contiguous range of element blocks.  Bijective for any nb.
__device__ inline int xcd_remap(int b, int nb) {
  constexpr int X = 8;
  const int q = nb / X, r = nb % X;
  const int x = b % X, l = b / X;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

// Element counts are below 2^31 (the host validates nE <= 2^28), so element
// indices and their (ex, ey, ez) decomposition use 32-bit unsigned arithmetic.
__device__ inline void elem_coords(long long e, const DevMesh& m, int& ex, int& ey, int& ez) {
  const unsigned ue = static_cast<unsigned>(e);
  const unsigned nx = static_cast<unsigned>(m.n[0]), ny = static_cast<unsigned>(m.n[1]);
  const unsigned t = ue / nx;
  ex = static_cast<int>(ue - t * nx);
  ez = static_cast<int>(t / ny);
  ey = static_cast<int>(t - static_cast<unsigned>(ez) * ny);
}

// Face neighbour of element (ex, ey, ez) across its lower (up = false) or
// upper face normal to d; -1 on a wall.
// a[d] for a per-lane d from three uniform values held in registers: a
// per-lane index into the by-value mesh argument (or a select between its
// fields, which the compiler folds into one) is a dependent memory load.
__device__ inline int pick3(int a0, int a1, int a2, int d) {
  a0 = __builtin_amdgcn_readfirstlane(a0);
  a1 = __builtin_amdgcn_readfirstlane(a1);
  a2 = __builtin_amdgcn_readfirstlane(a2);
  return d == 0 ? a0 : (d == 1 ? a1 : a2);
}

__device__ inline long long neighbour(const DevMesh& m, int ex, int ey, int ez, int d, bool up) {
  const int nd = pick3(m.n[0], m.n[1], m.n[2], d);
  const int bcd = pick3(m.bc[0], m.bc[1], m.bc[2], d);
  int v = (d == 0 ? ex : (d == 1 ? ey : ez)) + (up ? 1 : -1);
  if (v < 0 || v >= nd) {
    if (bcd != DG_BC_PERIODIC) return -1;
    v = v < 0 ? nd - 1 : 0;
  }
  const int x = d == 0 ? v : ex, y = d == 1 ? v : ey, z = d == 2 ? v : ez;
  return static_cast<long long>(x + m.n[0] * (y + m.n[1] * z));
}

// BR1 lifting value q* of q = (u, v, w, T) at a wall normal to d: the
// isothermal no-slip wall imposes (0, 0, 0, T_wall); the slip, adiabatic wall
// of the wall model keeps the own values qo with the normal velocity removed.
__device__ inline void wall_lifting_value(const DevMesh& m, int d, const double qo[4], double qs[4]) {
  if (pick3(m.bc[0], m.bc[1], m.bc[2], d) == DG_BC_WALL_MODEL) {
    qs[0] = d == 0 ? 0.0 : qo[0];
    qs[1] = d == 1 ? 0.0 : qo[1];
    qs[2] = d == 2 ? 0.0 : qo[2];
    qs[3] = qo[3];
  } else {
    qs[0] = qs[1] = qs[2] = 0.0;
    qs[3] = m.T_wall;
  }
}

// Index of the wall face of element (ex, ey, ez) on its lower (up = false) or
// upper wall normal to d, in the order of the wall-stress output: wall
// directions x, y, z; lower then upper wall; the wall elements with the first
// remaining element index fastest.
__device__ inline long long wall_face_index(const DevMesh& m, int ex, int ey, int ez, int d, bool up) {
  long long base = 0;
#pragma unroll
  for (int dd = 0; dd < 3; ++dd) {
    if (dd < d && m.bc[dd] != DG_BC_PERIODIC) {
      const long long na = dd == 0 ? m.n[1] : m.n[0], nb = dd == 2 ? m.n[1] : m.n[2];
      base += 2 * na * nb;
    }
  }
  const long long na = pick3(m.n[1], m.n[0], m.n[0], d), nb = pick3(m.n[2], m.n[2], m.n[1], d);
  const long long ea = d == 0 ? ey : ex, eb = d == 2 ? ey : ez;
  return base + (up ? na * nb : 0) + ea + na * eb;
}

// Node (i, j, k) of face f = 2 d + up with in-face coordinates (a, b):
// d = 0: (i, j, k) = (n, a, b); d = 1: (a, n, b); d = 2: (a, b, n), n = 0 or N.
template <int N>
__device__ inline void face_node(int d, bool up, int a, int b, int& i, int& j, int& k) {
  const int n = up ? N : 0;
  i = d == 0 ? n : a;
  j = d == 0 ? a : (d == 1 ? n : b);
  k = d == 2 ? n : b;
}

// Decoded face task t of a workgroup.
template <int N>
struct FaceTask {
  int le, f, d, ab, oi, oj, ok;
  bool up;
  __device__ FaceTask(int t) {
    constexpr int NF = (N + 1) * (N + 1);
    le = t / (6 * NF);
    const int rr = t - le * 6 * NF;
    f = rr / NF;
    ab = rr - f * NF;
    d = f >> 1;
    up = (f & 1) != 0;
    face_node<N>(d, up, ab % (N + 1), ab / (N + 1), oi, oj, ok);
  }
  // node of the neighbour element that coincides with the own face node
  __device__ int nb_node() const {
    const int opp = up ? 0 : N;
    const int ni = d == 0 ? opp : oi, nj = d == 1 ? opp : oj, nk = d == 2 ? opp : ok;
    return ni + (N + 1) * (nj + (N + 1) * nk);
  }
  __device__ int own_node() const { return oi + (N + 1) * (oj + (N + 1) * ok); }
};

// Face node number t (0 <= t < n_face_nodes) of an element -> (i, j, k): the
// two k planes first, then the boundary ring of each interior k plane.
template <int N>
__host__ __device__ inline void face_node_of(int t, int& i, int& j, int& k) {
  constexpr int NP = N + 1, NF = NP * NP, RING = 4 * N;
  if (t < 2 * NF) {
    k = t < NF ? 0 : N;
    const int ab = t < NF ? t : t - NF;
    i = ab % NP;
    j = ab / NP;
    return;
  }
  const int r = t - 2 * NF;
  k = 1 + r / RING;
  const int q = r % RING;
  if (q < NP) {
    i = q; j = 0;
  } else if (q < 2 * NP) {
    i = q - NP; j = N;
  } else if (q < 2 * NP + N - 1) {
    i = 0; j = q - 2 * NP + 1;
  } else {
    i = N; j = q - (2 * NP + N - 1) + 1;
  }
}

template <int N>
__host__ __device__ constexpr int n_face_nodes() {
  return 2 * (N + 1) * (N + 1) + (N - 1) * 4 * N;
}

// Inverse of face_node_of: the face node number of a node on the element's
// boundary.
template <int N>
__host__ __device__ constexpr int face_node_index(int i, int j, int k) {
  constexpr int NP = N + 1, NF = NP * NP, RING = 4 * N;
  if (k == 0 || k == N) return (k == 0 ? 0 : NF) + i + NP * j;
  const int q = j == 0 ? i : (j == N ? NP + i : (i == 0 ? 2 * NP + j - 1 : 2 * NP + N - 1 + j - 1));
  return 2 * NF + (k - 1) * RING + q;
}

struct Prim {
  double rho, u, v, w, p, e, T;
};

// Ideal-gas primitive recovery, always FP64.
__device__ inline Prim primitives(const double s[5], const DevPhys& ph) {
  Prim P;
  const double r = s[0];
  const double ir = 1.0 / r;
  P.rho = r;
  P.u = s[1] * ir;
  P.v = s[2] * ir;
  P.w = s[3] * ir;
  P.p = ph.gm1 * (s[4] - 0.5 * r * (P.u * P.u + P.v * P.v + P.w * P.w));
  P.e = s[4] * ir;
  P.T = P.p * ph.inv_R * ir;
  return P;
}

// mu(T) / mu (= kappa(T) / kappa): 1 for constant viscosity; Sutherland's law
// (T / T_ref)^(3/2) (T_ref + S) / (T + S) = c T sqrt(T) / (T + S).
__device__ inline double viscosity_ratio(const DevPhys& ph, double T) {
  return ph.suth ? ph.suth_c * T * sqrt(T) / (T + ph.suth_S) : 1.0;
}

__device__ inline double vel(const Prim& P, int d) { return d == 0 ? P.u : (d == 1 ? P.v : P.w); }

// Values a kernel reads or writes once (G, the neighbours' face viscous
// fluxes, the updated state): non-temporal accesses, so that they do not
// displace from L2 the states that neighbouring workgroups read.  Only for
// whole coalesced rows: the scattered face-flux stores of the face kernels
// were slower non-temporal (no write combining in L2).
template <typename T>
__device__ inline T load_once(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ inline void store_once(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

__device__ inline void load_state(const double* U, long long stride, long long idx, double u[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = U[v * stride + idx];
}

// ---- entropy-conserving flux and Roe flux helpers (FP64) ----

// 1 / x for x > 0 of moderate size: the hardware reciprocal estimate refined
// by two Newton-Raphson steps r <- r + r (1 - x r).
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Means of the entropy-conserving flux for one pair: rho_ln and 1 / beta_ln
// (logarithmic means) and p^ = {{rho}} / (2 {{beta}}).  The logarithmic mean of
// positive a, b is (a - b) / (ln a - ln b) = (a + b) / (2 F), F = atanh(f) / f,
// f = (a - b) / (a + b) (ln(a / b) = 2 atanh f).  For f^2 < 1e-4 F is its
// series 1 + f^2/3 + f^4/5 + f^6/7 and 1 / F the series
// 1 - f^2/3 - 4 f^4/45 - 44 f^6/945 (first dropped terms below 1.2e-17 and
// 3.1e-18), so the common case costs one reciprocal and no logarithm.
__device__ inline void ec_means(double ra, double rb, double ba, double bb, double& rho_ln,
                                double& inv_beta_ln, double& p_hat) {
  const double sr = ra + rb, sb = ba + bb;
  // both reciprocals from one: 1 / (sr sb) times the other sum
  const double x = rcp_nr(sr * sb);
  const double ir = sb * x, ib = sr * x;
  const double fr = (ra - rb) * ir, fb = (ba - bb) * ib;
  const double ur = fr * fr, ub = fb * fb;
  rho_ln = 0.5 * sr * (1.0 - ur * (1.0 / 3.0 + ur * (4.0 / 45.0 + ur * (44.0 / 945.0))));
  inv_beta_ln = 2.0 * ib * (1.0 + ub * (1.0 / 3.0 + ub * (0.2 + ub * (1.0 / 7.0))));
  if (ur >= 1e-4) rho_ln = 0.5 * sr * fr / atanh(fr);
  if (ub >= 1e-4) inv_beta_ln = 2.0 * ib * atanh(fb) / fb;
  p_hat = 0.5 * sr * ib;
}

// |lambda| with Harten's entropy correction in the Harten-Hyman form:
// (lambda^2 + delta^2) / (2 delta) where |lambda| < delta,
// delta = max(0, lambda - lambda_L, lambda_R - lambda).
__device__ inline double hh_abs(double lam, double lam_L, double lam_R) {
  double delta = fmax(lam - lam_L, lam_R - lam);
  delta = delta > 0.0 ? delta : 0.0;
  return fabs(lam) < delta ? (lam * lam + delta * delta) / (2.0 * delta) : fabs(lam);
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

// Viscous flux along d: g[3 q + b] = d q / d x_b for q in (u, v, w, T);
// returns (tau_1d, tau_2d, tau_3d, u_a tau_ad + kappa dT/dx_d).
template <int d, typename R>
__device__ inline void viscous_flux(R u, R v, R w, const R g[12], R mu, R kappa, R f[4]) {
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

template <int N>
inline int n_blocks(long long nE) {
  return static_cast<int>((nE + Cfg<N>::EPB - 1) / Cfg<N>::EPB);
}

}  // namespace dg
