// Forward kernels of the split-form DGSEM operator for gfx950.
//
// Per RK stage two kernels run (paper Sec. 2.2 split-form DG on LGL nodes,
// Sec. 4 viscous fluxes and low-storage RK):
//
//   k_face_flux : U -> the normal viscous flux f_v,d (4 components) on the six
//                 face planes of every element (BR1 lifting evaluated at the
//                 face nodes only);
//   k_rhs       : U, the neighbours' face viscous fluxes -> Ut, or the fused
//                 low-storage RK update G <- A G + dt Ut, U' <- U + B G.
//                 It recomputes its own element's lifted gradients from U.
//
// So the lifted gradients never travel through HBM: per DOF and stage the
// method moves U in twice, G in and out, U' out and three face-flux values
// (N = 7) out and in, instead of twelve gradient components out and in.
//
// One workgroup owns EPB whole elements, one lane per node.  Inside k_rhs:
//   P1  node lanes load U (SoA, coalesced), recover the primitives in FP64
//       and stage (rho, u, v, w, p, e) and T in LDS; face lanes (one per face
//       node) load the own and neighbour states at their face node and the
//       neighbour's face viscous flux, and form the BR1 lifting corrections;
//   P2  node lanes sweep the lines for the 12 lifted gradient components;
//   P3  per direction d: node lanes stage f_v,d in LDS, then sweep the
//       d-lines for 2 sum_m D_im f#_KG(U_i, U_m) - sum_m D_im f_v,d(U_m);
//   P4  face lanes form the surface corrections (LLF + BR1, or the wall flux);
//   P5  node lanes add them, scale by s_d = 2/width_d and write or update.
//
// Mixed precision (R = float): the LDS fields, gradients, viscous fluxes and
// line sums are FP32, and so are the Lax-Friedrichs surface fluxes (formed
// from FP64 differences of the two sides' states); U, G, the primitive
// recovery, the lifting corrections, the Roe surface flux of the
// entropy-conserving pair and the RK update stay FP64.  Pressure, specific energy and temperature are stored
// relative to the element's first node (p - p_ref, e - e_ref, T - T_ref, with
// the differences taken in FP64), and the exactly known contributions of the
// reference values are added back: sum_m D_im = 0 removes p_ref from the
// momentum flux differences and leaves 2 e_ref sum_m D_im (rho u_d)# +
// p_ref sum_m D_im u_d,m in the energy equation.  The entropy-conserving
// pair does the same with its own reference quantities (beta - beta_ref and
// rho (p - p_ref) / p per node, internal energy as e_ref).
//
// Workgroup ids are remapped so that each XCD (own L2) covers one contiguous
// range of elements, keeping face neighbours in the same L2.
#include "dg_device.hpp"

namespace dg {
namespace {

// Vector of two R values (one 64- or 128-bit LDS access).
template <typename R>
struct V2T;
template <>
struct V2T<double> {
  using type = double2;
};
template <>
struct V2T<float> {
  using type = float2;
};

// Line sums along direction d of (u, v, w, T) held as LDS pairs q[0] = (u, v),
// q[1] = (w, T) at node (i, j, k); D is read once per line position.
template <int N, typename R, int d, typename V2>
__device__ inline void line_sums_pairs(const R* sD, const V2 (*q)[Geo<N>::EB], int i, int j, int k,
                                       R a[4]) {
  using Gm = Geo<N>;
  constexpr int NP = Gm::NP;
  const int idx = d == 0 ? i : (d == 1 ? j : k);
  a[0] = a[1] = a[2] = a[3] = R(0);
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int lm = d == 0 ? Gm::lds(m, j, k) : (d == 1 ? Gm::lds(i, m, k) : Gm::lds(i, j, m));
    const R Dm = sD[idx * Gm::DS + m];
    const V2 uv = q[0][lm], wT = q[1][lm];
    a[0] += Dm * uv.x;
    a[1] += Dm * uv.y;
    a[2] += Dm * wT.x;
    a[3] += Dm * wT.y;
  }
}

// BR1 lifted gradients g[3 q + d] of (u, v, w, T) (LDS pairs) at node
// (i, j, k), with the lifting corrections ssq of the six faces.
template <int N, typename R, typename V2>
__device__ inline void lifted_gradients(const R* sD, const V2 (*q)[Geo<N>::EB],
                                        const R (*ssq)[4][Geo<N>::NF], int i, int j, int k, R sx,
                                        R sy, R sz, R g[12]) {
  constexpr int NP = N + 1;
  R a[4];
  line_sums_pairs<N, R, 0, V2>(sD, q, i, j, k, a);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (i == 0) a[c] += ssq[0][c][j + NP * k];
    if (i == N) a[c] += ssq[1][c][j + NP * k];
    g[3 * c + 0] = sx * a[c];
  }
  line_sums_pairs<N, R, 1, V2>(sD, q, i, j, k, a);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (j == 0) a[c] += ssq[2][c][i + NP * k];
    if (j == N) a[c] += ssq[3][c][i + NP * k];
    g[3 * c + 1] = sy * a[c];
  }
  line_sums_pairs<N, R, 2, V2>(sD, q, i, j, k, a);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (k == 0) a[c] += ssq[4][c][i + NP * j];
    if (k == N) a[c] += ssq[5][c][i + NP * j];
    g[3 * c + 2] = sz * a[c];
  }
}

// Viscous stress and heat flux of gradients g: tau = (t00, t11, t22, t01, t02, t12)
// = mu (grad u + grad u^T - 2/3 div u I), qT = kappa grad T.
template <typename R>
__device__ inline void stress(const R g[12], R mu, R kappa, R tau[6], R qT[3]) {
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

// f_v,d from the stress: (tau_0d, tau_1d, tau_2d, u_a tau_ad + kappa dT/dx_d).
template <int d, typename R>
__device__ inline void viscous_flux_tau(R u, R v, R w, const R tau[6], const R qT[3], R f[4]) {
  f[0] = d == 0 ? tau[0] : (d == 1 ? tau[3] : tau[4]);
  f[1] = d == 0 ? tau[3] : (d == 1 ? tau[1] : tau[5]);
  f[2] = d == 0 ? tau[4] : (d == 1 ? tau[5] : tau[2]);
  f[3] = u * f[0] + v * f[1] + w * f[2] + qT[d];
}

// Lifting corrections of one face task: (q* - q_own) (+-1/w_end), FP64.
__device__ inline void lifting_correction(const Prim& Po, const Prim& Pn, bool wall, const DevMesh& m,
                                          int d, bool up, double inv_w, double out[4]) {
  const double qo[4] = {Po.u, Po.v, Po.w, Po.T};
  double qs[4];
  wall_lifting_value(m, d, qo, qs);  // the wall's value (isothermal or wall-model wall)
  if (!wall) {
    const double qn[4] = {Pn.u, Pn.v, Pn.w, Pn.T};
#pragma unroll
    for (int c = 0; c < 4; ++c) qs[c] = 0.5 * (qo[c] + qn[c]);
  }
  const double sc = up ? inv_w : -inv_w;
#pragma unroll
  for (int c = 0; c < 4; ++c) out[c] = (qs[c] - qo[c]) * sc;
}

// Per-element reference (p, e, T) of the mixed-precision sweeps: the values at
// node 0 (state s0), or zero in FP64 and with the subtraction switched off.
template <typename R>
__device__ inline bool uses_ref(const DevPhys& ph) {
  return sizeof(R) == sizeof(float) && ph.mixed_ref;
}

template <typename R>
__device__ inline void element_ref(const double s0[5], const DevPhys& ph, double& p_ref,
                                   double& e_ref, double& T_ref) {
  if (!uses_ref<R>(ph)) {
    p_ref = e_ref = T_ref = 0.0;
    return;
  }
  const Prim P = primitives(s0, ph);
  p_ref = P.p;
  e_ref = P.e;
  T_ref = P.T;
}

// --------------------------------------------------------------------------
// k_face_flux: f_v,d on the face planes, layout ffv[e][face][c][ab]
// --------------------------------------------------------------------------
template <int N, typename R>
__global__ __launch_bounds__(Cfg<N>::BS) __attribute__((amdgpu_waves_per_eu(Cfg<N>::FACE_WAVES))) void k_face_flux(
    const double* __restrict__ U, R* __restrict__ ffv, DevMesh mesh, DevPhys ph, DevBasis basis) {
  using Gm = Geo<N>;
  constexpr int NP = Gm::NP, NF = Gm::NF, NN = Gm::NN, EB = Gm::EB;
  constexpr int EPB = Cfg<N>::EPB, BS = Cfg<N>::BS;
  constexpr int NFN = n_face_nodes<N>();
  static_assert(EPB * NFN <= BS, "one lane per face node");
  using V2 = typename V2T<R>::type;
  __shared__ R sD[NP * Gm::DS];
  __shared__ V2 sq[EPB][2][EB];  // (u, v), (w, T - T_ref)
  __shared__ R ssq[EPB][6][4][NF];
  constexpr bool MIXED = sizeof(R) == 4;
  // mixed precision: the FP64 (u, v, w, T) of every node, for the lifting terms
  __shared__ double sqd[MIXED ? EPB : 1][4][MIXED ? NN : 1];

  const int tid = threadIdx.x;
  const long long nE = mesh.nE;
  const long long stride = nE * NN;
  const long long e0 = static_cast<long long>(xcd_remap(blockIdx.x, gridDim.x)) * EPB;
  // D is fetched with the first loads and written to LDS before the first
  // barrier, so its latency is not paid on its own
  static_assert(NP * NP <= BS, "one lane per entry of D");
  double dval = 0.0;
  if (tid < NP * NP) dval = basis.D[tid];
  int ex0 = 0, ey0 = 0, ez0 = 0;
  elem_coords(e0 < nE ? e0 : 0, mesh, ex0, ey0, ez0);

  // P1: node lanes stage (u, v, w, T - T_ref) in LDS (and, in mixed
  // precision, an FP64 copy of (u, v, w, T)); face lanes fetch the
  // neighbour state and form the BR1 lifting corrections in FP64 after the
  // barrier, with the own values from LDS
  const bool face_lane = tid < n_face_tasks<N>();
  const bool face_ok = face_lane && (EPB == 1 ? e0 : e0 + FaceTask<N>(face_lane ? tid : 0).le) < nE;
  // the own state is fetched first, so that it and the neighbour's face node
  // are in flight together
  const int nle = EPB == 1 ? 0 : tid / NN;
  const int node = tid - nle * NN;
  const long long ne = EPB == 1 ? e0 : e0 + nle;
  const bool node_ok = (EPB == 1 ? tid < NN : nle < EPB) && ne < nE;
  double s[5] = {1.0, 0.0, 0.0, 0.0, 1.0}, s0[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
  if (node_ok) {
    load_state(U, stride, ne * NN + node, s);
    if (uses_ref<R>(ph)) load_state(U, stride, ne * NN, s0);
  }
  double sn[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
  bool fwall = true;
  if (face_ok) {
    const FaceTask<N> ft(tid);
    const long long te = EPB == 1 ? e0 : e0 + ft.le;
    int ex = ex0, ey = ey0, ez = ez0;
    if (EPB > 1) elem_coords(te, mesh, ex, ey, ez);
    const long long nb = neighbour(mesh, ex, ey, ez, ft.d, ft.up);
    fwall = nb < 0;
    if (!fwall) load_state(U, stride, nb * NN + ft.nb_node(), sn);
  }
  if (node_ok) {
    const int i = node % NP, j = (node / NP) % NP, k = node / NF;
    const Prim P = primitives(s, ph);
    double p_ref, e_ref, T_ref;
    element_ref<R>(s0, ph, p_ref, e_ref, T_ref);
    const int l = Gm::lds(i, j, k);
    sq[nle][0][l] = V2{static_cast<R>(P.u), static_cast<R>(P.v)};
    sq[nle][1][l] = V2{static_cast<R>(P.w), static_cast<R>(P.T - T_ref)};
    if (MIXED) {
      sqd[nle][0][node] = P.u;
      sqd[nle][1][node] = P.v;
      sqd[nle][2][node] = P.w;
      sqd[nle][3][node] = P.T;
    }
  }
  if (tid < NP * NP) sD[(tid / NP) * Gm::DS + tid % NP] = static_cast<R>(dval);
  __syncthreads();
  {
    if (face_ok) {
      const FaceTask<N> ft(tid);
      double qo[4];
      if (MIXED) {
        const int on = ft.own_node();
#pragma unroll
        for (int c = 0; c < 4; ++c) qo[c] = sqd[ft.le][c][on];
      } else {
        const int lo = Gm::lds(ft.oi, ft.oj, ft.ok);
        const V2 uv = sq[ft.le][0][lo], wT = sq[ft.le][1][lo];
        qo[0] = uv.x;
        qo[1] = uv.y;
        qo[2] = wT.x;
        qo[3] = wT.y;
      }
      double qs[4];
      wall_lifting_value(mesh, ft.d, qo, qs);
      if (!fwall) {
        const Prim Pn = primitives(sn, ph);
        qs[0] = 0.5 * (qo[0] + Pn.u);
        qs[1] = 0.5 * (qo[1] + Pn.v);
        qs[2] = 0.5 * (qo[2] + Pn.w);
        qs[3] = 0.5 * (qo[3] + Pn.T);
      }
      const double sc = ft.up ? basis.inv_w_end : -basis.inv_w_end;
#pragma unroll
      for (int c = 0; c < 4; ++c) ssq[ft.le][ft.f][c][ft.ab] = static_cast<R>((qs[c] - qo[c]) * sc);
    }
    __syncthreads();
  }

  // P2: one lane per face node: lifted gradients and f_v,d of each face the
  // node lies on
  const int le = EPB == 1 ? 0 : tid / NFN;
  const long long e = EPB == 1 ? e0 : e0 + le;
  if ((EPB == 1 ? tid < NFN : le < EPB) && e < nE) {
    int i, j, k;
    face_node_of<N>(tid - le * NFN, i, j, k);
    int ex = ex0, ey = ey0, ez = ez0;
    if (EPB > 1) elem_coords(e, mesh, ex, ey, ez);
    R g[12];
    lifted_gradients<N, R, V2>(sD, sq[le], ssq[le], i, j, k, static_cast<R>(mesh.s[0][ex]),
                               static_cast<R>(mesh.s[1][ey]), static_cast<R>(mesh.s[2][ez]), g);
    const int l = Gm::lds(i, j, k);
    const V2 uv = sq[le][0][l], wT = sq[le][1][l];
    const R u = uv.x, v = uv.y, w = wT.x;
    R mu = static_cast<R>(ph.mu), kappa = static_cast<R>(ph.kappa);
    if (ph.suth) {
      // mu(T) at the node's temperature: in FP64 the LDS holds T itself, in
      // mixed precision the FP64 copy holds it
      const double T = MIXED ? sqd[le][3][i + NP * (j + NP * k)] : static_cast<double>(wT.y);
      const R r = static_cast<R>(viscosity_ratio(ph, T));
      mu *= r;
      kappa *= r;
    }
    R* out = ffv + e * (6 * 4 * NF);
    R f[4];
    if (i == 0 || i == N) {
      viscous_flux<0, R>(u, v, w, g, mu, kappa, f);
      const int fi = i == 0 ? 0 : 1;
#pragma unroll
      for (int c = 0; c < 4; ++c) out[(fi * 4 + c) * NF + j + NP * k] = f[c];
    }
    if (j == 0 || j == N) {
      viscous_flux<1, R>(u, v, w, g, mu, kappa, f);
      const int fi = j == 0 ? 2 : 3;
#pragma unroll
      for (int c = 0; c < 4; ++c) out[(fi * 4 + c) * NF + i + NP * k] = f[c];
    }
    if (k == 0 || k == N) {
      viscous_flux<2, R>(u, v, w, g, mu, kappa, f);
      const int fi = k == 0 ? 4 : 5;
#pragma unroll
      for (int c = 0; c < 4; ++c) out[(fi * 4 + c) * NF + i + NP * j] = f[c];
    }
  }
}

// --------------------------------------------------------------------------
// k_rhs
// --------------------------------------------------------------------------

// LDS layout of k_rhs: unpadded x-rows, swizzled where N + 1 is a power of
// two.  In an x-line sweep the eight lanes of a row read one address and the
// wave reads NP rows at the same x-position: 128-bit reads of unswizzled rows
// then meet in the same banks (measured 9.0 instead of 4.9 CU cycles per wave
// read; padded rows fix that but slow the z-line reads to 9.2); the swizzle
// reads 5.0, 4.8 and 4.9 cycles in x, y and z.  k_face_flux keeps padded rows,
// which its ring lanes need.
template <int N>
using GeoR = Geo<N, 0, ((N + 1) & N) == 0>;

// Line sums along direction d of the half values of u, v, w (packed LDS
// fields) and of T at node (i, j, k); D is read once per line position.
template <int N, typename R, int d, typename V2>
__device__ inline void line_sums_half(const R* sD, const V2 (*sp)[GeoR<N>::EB], const R* sT, int i,
                                      int j, int k, R a[4]) {
  using Gm = GeoR<N>;
  constexpr int NP = Gm::NP;
  const int idx = d == 0 ? i : (d == 1 ? j : k);
  a[0] = a[1] = a[2] = a[3] = R(0);
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int lm = d == 0 ? Gm::lds(m, j, k) : (d == 1 ? Gm::lds(i, m, k) : Gm::lds(i, j, m));
    const R Dm = sD[idx * Gm::DS + m];
    const V2 ru = sp[0][lm], vw = sp[1][lm];
    a[0] += Dm * ru.y;
    a[1] += Dm * vw.x;
    a[2] += Dm * vw.y;
    a[3] += Dm * sT[lm];
  }
}

// BR1 lifted gradients g[3 q + d] at node (i, j, k) from the half values of
// u, v, w and from T, with the lifting corrections ssq of the six faces.
template <int N, typename R, typename V2, bool HALF = true>
__device__ inline void lifted_gradients_half(const R* sD, const V2 (*sp)[GeoR<N>::EB],
                                             const R* sT, const R (*ssq)[4][GeoR<N>::NF], int i,
                                             int j, int k, R sx, R sy, R sz, R g[12]) {
  constexpr int NP = N + 1;
  R a[4];
  // x
  line_sums_half<N, R, 0, V2>(sD, sp, sT, i, j, k, a);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    R t = c < 3 && HALF ? R(2) * a[c] : a[c];  // half values: twice the line sum (exact)
    if (i == 0) t += ssq[0][c][j + NP * k];
    if (i == N) t += ssq[1][c][j + NP * k];
    g[3 * c + 0] = sx * t;
  }
  // y
  line_sums_half<N, R, 1, V2>(sD, sp, sT, i, j, k, a);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    R t = c < 3 && HALF ? R(2) * a[c] : a[c];
    if (j == 0) t += ssq[2][c][i + NP * k];
    if (j == N) t += ssq[3][c][i + NP * k];
    g[3 * c + 1] = sy * t;
  }
  // z
  line_sums_half<N, R, 2, V2>(sD, sp, sT, i, j, k, a);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    R t = c < 3 && HALF ? R(2) * a[c] : a[c];
    if (k == 0) t += ssq[4][c][i + NP * j];
    if (k == N) t += ssq[5][c][i + NP * j];
    g[3 * c + 2] = sz * t;
  }
}

// One pass over the d-line through node (i, j, k) for both the lifted
// gradients and the convective flux differencing (Kennedy-Gruber pair, the
// line values read from LDS once for the two):
//   a[0..2] = sum_m D_im (u, v, w)_m / 2 and a[3] = sum_m D_im (T - T_ref)_m
//   (VISC only), ac = sum_m D_im f#_KG(own, m), and du = sum_m D_im u_d,m / 2
//   (the mixed-precision add-back; with VISC it is a[d]).
// Own and line values are halves: ((rho, u), (v, w), (p - p_ref, e - e_ref)) / 2,
// so that {{x}} = a.x + b.x exactly as (x_a + x_b) / 2.  The Kennedy-Gruber flux
//   f# = ({{rho}}{{u_d}}, {{rho}}{{u_d}}{{u}} + {{p}} delta_1d, ...,
//         {{u_d}} ({{rho}}{{e}} + {{p}}))
// enters the sums premultiplied by D_im: with s = D_im {{u_d}} and
// m = s {{rho}}, the five components take m, m {{u}}, m {{v}}, m {{w}}
// (+ D_im {{p}} in component 1 + d) and s ({{rho}}{{e}} + {{p}}).
template <int N, typename R, int d, bool VISC, bool MIXED, typename V2>
__device__ inline void fused_sweep(const V2 (&own)[3], int i, int j, int k, const R* sD,
                                   const V2 (*sp)[GeoR<N>::EB], const R* sT, R a[4], R ac[5],
                                   R& du) {
  using Gm = GeoR<N>;
  constexpr int NP = Gm::NP;
  const int idx = d == 0 ? i : (d == 1 ? j : k);
  for (int v = 0; v < 5; ++v) ac[v] = R(0);
  a[0] = a[1] = a[2] = a[3] = R(0);
  du = R(0);
  // partly unrolled (four positions at N = 7, two below): fully unrolled,
  // the hoisted line loads and the gradient and flux sums held together
  // spill registers
  constexpr int UF = NP >= 8 ? 4 : 2;
#pragma unroll UF
  for (int m = 0; m < NP; ++m) {
    const int lm = d == 0 ? Gm::lds(m, j, k) : (d == 1 ? Gm::lds(i, m, k) : Gm::lds(i, j, m));
    const R Dim = sD[idx * Gm::DS + m];
    const V2 b0 = sp[0][lm], b1 = sp[1][lm], b2 = sp[2][lm];
    if (VISC) {
      a[0] += Dim * b0.y;
      a[1] += Dim * b1.x;
      a[2] += Dim * b1.y;
      a[3] += Dim * sT[lm];
    } else if (MIXED) {
      du += Dim * (d == 0 ? b0.y : (d == 1 ? b1.x : b1.y));
    }
    const R rho = own[0].x + b0.x;
    const R u = own[0].y + b0.y, v = own[1].x + b1.x, w = own[1].y + b1.y;
    const R p = own[2].x + b2.x, e = own[2].y + b2.y;
    const R ud = d == 0 ? u : (d == 1 ? v : w);
    const R s = Dim * ud;
    const R mm = s * rho;
    ac[0] += mm;
    ac[1] += mm * u;
    ac[2] += mm * v;
    ac[3] += mm * w;
    ac[1 + d] += Dim * p;
    ac[4] += s * (rho * e + p);
  }
  if (VISC) du = a[d];
}

// Direction d of the fused pass: the three lifted gradient components along
// d (line sums, BR1 lifting corrections of the d-faces, scale s_d) and the
// convective part of the d-contribution to the right-hand side,
// ut -= s_d 2 sum_m D_im f#_KG (plus, in mixed precision, the reference
// state's exactly known part 2 s_d (e_ref sum D (rho u_d)# + p_ref sum D u_d)).
template <int N, typename R, int d, bool VISC, bool MIXED, typename V2>
__device__ inline void fused_direction(const V2 (&own)[3], int i, int j, int k, const R* sD,
                                       const V2 (*sp)[GeoR<N>::EB], const R* sT,
                                       const R (*ssq)[4][GeoR<N>::NF], double sd, double e_ref,
                                       double p_ref, R g[12], double ut[5]) {
  constexpr int NP = N + 1;
  R a[4], ac[5], du;
  fused_sweep<N, R, d, VISC, MIXED, V2>(own, i, j, k, sD, sp, sT, a, ac, du);
  if (VISC) {
    const int idx = d == 0 ? i : (d == 1 ? j : k);
    const int ab = d == 0 ? j + NP * k : (d == 1 ? i + NP * k : i + NP * j);
    const R s = static_cast<R>(sd);
    R t[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) t[c] = c < 3 ? R(2) * a[c] : a[c];  // half values: twice the line sum (exact)
    if (idx == 0 || idx == N) {  // one branch for the two line ends
      const int f = 2 * d + (idx == N ? 1 : 0);
#pragma unroll
      for (int c = 0; c < 4; ++c) t[c] += ssq[f][c][ab];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) g[3 * c + d] = s * t[c];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) ut[v] -= sd * static_cast<double>(R(2) * ac[v]);
  if (MIXED) ut[4] -= sd * 2.0 * (e_ref * static_cast<double>(ac[0]) + p_ref * static_cast<double>(du));
}

// av = sum_m D_im f_v,d(m) along the d-line through (i, j, k): the viscous
// flux of direction d staged in LDS as pairs (f0, f1), (f2, f3).
template <int N, typename R, int d, typename V2>
__device__ inline void viscous_sweep(int i, int j, int k, const R* sD,
                                     const V2 (*sfv)[GeoR<N>::EB], R av[4]) {
  using Gm = GeoR<N>;
  constexpr int NP = Gm::NP;
  const int idx = d == 0 ? i : (d == 1 ? j : k);
  av[0] = av[1] = av[2] = av[3] = R(0);
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int lm = d == 0 ? Gm::lds(m, j, k) : (d == 1 ? Gm::lds(i, m, k) : Gm::lds(i, j, m));
    const R Dim = sD[idx * Gm::DS + m];
    const V2 f01 = sfv[0][lm], f23 = sfv[1][lm];
    av[0] += Dim * f01.x;
    av[1] += Dim * f01.y;
    av[2] += Dim * f23.x;
    av[3] += Dim * f23.y;
  }
}

// Surface correction of one face task (FP64):
//   ((F*_c - F*_v) - (f_c - f_v)(own)) (+-1/w_end),
// accumulated term by term to keep few values live.  A = own (rho, u, v, w, p, e);
// so, sn: own and neighbour conservative states at the face node; fvo, fvn:
// their normal viscous fluxes.
template <int d>
__device__ inline void surface_correction(const double A[6], const double so[5], const double sn[5],
                                          bool wall, bool up, const double fvo[4],
                                          const double fvn[4], const DevPhys& ph, double inv_w,
                                          double corr[5]) {
  const double po = A[4];
  // minus the own physical flux (f_c - f_v)
  {
    const double ud = A[1 + d];
    const double mass = A[0] * ud;
    corr[0] = -mass;
    corr[1] = -mass * A[1] + fvo[0];
    corr[2] = -mass * A[2] + fvo[1];
    corr[3] = -mass * A[3] + fvo[2];
    corr[1 + d] -= po;
    corr[4] = -(so[4] + po) * ud + fvo[3];
  }
  if (wall) {
    // isothermal no-slip wall: pressure-only convective flux; viscous flux
    // with zero wall velocity and the interior gradients (drops u . tau)
    corr[1 + d] += po;
    corr[1] -= fvo[0];
    corr[2] -= fvo[1];
    corr[3] -= fvo[2];
    corr[4] -= fvo[3] - (A[1] * fvo[0] + A[2] * fvo[1] + A[3] * fvo[2]);
  } else {
    const double irn = 1.0 / sn[0];
    const double b1 = sn[1] * irn, b2 = sn[2] * irn, b3 = sn[3] * irn;
    const double pn = ph.gm1 * (sn[4] - 0.5 * sn[0] * (b1 * b1 + b2 * b2 + b3 * b3));
    const double B[6] = {sn[0], b1, b2, b3, pn, sn[4] * irn};
    double F[5];
    kg_flux<d, double>(A, B, F);
#pragma unroll
    for (int v = 0; v < 5; ++v) corr[v] += F[v];
    if (!ph.central) {
      const double cu = fabs(A[1 + d]) + sqrt(ph.gamma * po / A[0]);
      const double cn = fabs(B[1 + d]) + sqrt(ph.gamma * pn * irn);
      const double lam = cu >= cn ? cu : cn;
      // -lambda/2 (U_R - U_L), L = the lower side of the face
      const double sl = (up ? -0.5 : 0.5) * lam;
#pragma unroll
      for (int v = 0; v < 5; ++v) corr[v] += sl * (sn[v] - so[v]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) corr[1 + c] -= 0.5 * (fvo[c] + fvn[c]);
  }
  const double sc = up ? inv_w : -inv_w;
#pragma unroll
  for (int v = 0; v < 5; ++v) corr[v] *= sc;
}

// Surface correction of one face task in FP32 (mixed precision, Kennedy-Gruber
// / Lax-Friedrichs pair): the terms of surface_correction written in the
// differences dx = x_n - x_o of the neighbour's and the own primitives
// (formed in FP64 from the FP64 states, then rounded once), so that no FP32
// difference of large, nearly equal values is formed (p ~ 70, e ~ 180 at
// Ma = 0.1).  With m_o = rho_o u_d,o and dm = {{rho}}{{u_d}} - m_o
// = (drho/2) u_d,o + {{rho}} (du_d/2), exactly:
//   f#_d - f_d(own):  mass dm;  momentum a: dm {{u_a}} + m_o du_a/2 + e_ad dp/2;
//                     energy dm {{e}} + m_o de/2 + {{u_d}} dp/2 + p_o du_d/2;
// the dissipation -lambda/2 (U_R - U_L) from the FP64 differences of the
// conservative states; the BR1 viscous part (f_v,o - f_v,n)/2.  A wall face
// keeps the pressure-only convective flux and the zero-velocity viscous flux
// (own stresses; of the energy flux only the heat flux).
template <int d>
__device__ inline void surface_correction_f32(const Prim& Po, const double so[5], const double sn[5],
                                              bool wall, bool up, const double fvo[4], const double fvn[4],
                                              const DevPhys& ph, double inv_w, float corr[5]) {
  const float uo[3] = {static_cast<float>(Po.u), static_cast<float>(Po.v), static_cast<float>(Po.w)};
  const float ro = static_cast<float>(Po.rho);
  const float mo = ro * uo[d];
  if (wall) {
    corr[0] = -mo;
#pragma unroll
    for (int a = 0; a < 3; ++a) corr[1 + a] = -mo * uo[a];
    corr[4] = -static_cast<float>(so[4] + Po.p) * uo[d] +
              (uo[0] * static_cast<float>(fvo[0]) + uo[1] * static_cast<float>(fvo[1]) +
               uo[2] * static_cast<float>(fvo[2]));
  } else {
    const double irn = 1.0 / sn[0];
    const double un[3] = {sn[1] * irn, sn[2] * irn, sn[3] * irn};
    const double pn = ph.gm1 * (sn[4] - 0.5 * sn[0] * (un[0] * un[0] + un[1] * un[1] + un[2] * un[2]));
    const float h = 0.5f;
    const float hdr = h * static_cast<float>(sn[0] - Po.rho);
    const float hdu[3] = {h * static_cast<float>(un[0] - Po.u), h * static_cast<float>(un[1] - Po.v),
                          h * static_cast<float>(un[2] - Po.w)};
    const float hdp = h * static_cast<float>(pn - Po.p);
    const float hde = h * static_cast<float>(sn[4] * irn - Po.e);
    const float rm = ro + hdr;
    float um[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) um[a] = uo[a] + hdu[a];
    const float dm = hdr * uo[d] + rm * hdu[d];
    corr[0] = dm;
#pragma unroll
    for (int a = 0; a < 3; ++a) corr[1 + a] = dm * um[a] + mo * hdu[a];
    corr[1 + d] += hdp;
    corr[4] = dm * (static_cast<float>(Po.e) + hde) + mo * hde + um[d] * hdp + static_cast<float>(Po.p) * hdu[d];
    if (!ph.central) {
      const float gam = static_cast<float>(ph.gamma);
      const float cu = fabsf(uo[d]) + sqrtf(gam * static_cast<float>(Po.p) / ro);
      const float cn = fabsf(static_cast<float>(un[d])) + sqrtf(gam * static_cast<float>(pn * irn));
      const float lam = cu >= cn ? cu : cn;
      const float sl = (up ? -0.5f : 0.5f) * lam;
#pragma unroll
      for (int v = 0; v < 5; ++v) corr[v] += sl * static_cast<float>(sn[v] - so[v]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) corr[1 + c] += h * static_cast<float>(fvo[c] - fvn[c]);
  }
  const float sc = static_cast<float>(up ? inv_w : -inv_w);
#pragma unroll
  for (int v = 0; v < 5; ++v) corr[v] *= sc;
}

// ---------------------------------------------------------------------------
// Entropy-conserving volume flux and Roe surface flux (FP64)
// ---------------------------------------------------------------------------

// Chandrashekar's kinetic-energy-preserving, entropy-conserving two-point flux
// along d (paper Sec. 4 names it as the production volume flux).  a, b =
// (rho, u), (v, w), (beta, |u|^2) with beta = rho / (2 p); {{x}} arithmetic and
// x_ln logarithmic means:
//   f_rho = rho_ln {{u_d}},  f_m = f_rho {{u}} + p^ e_d,  p^ = {{rho}} / (2 {{beta}}),
//   f_E = f_rho (1 / (2 (gamma - 1) beta_ln) - {{|u|^2}} / 2) + {{u}} . f_m.
template <int d>
__device__ inline void ec_flux(const double2 a[3], const double2 b[3], double gm1, double f[5]) {
  double rho_ln, inv_beta_ln, p_hat;
  ec_means(a[0].x, b[0].x, a[2].x, b[2].x, rho_ln, inv_beta_ln, p_hat);
  const double u = 0.5 * (a[0].y + b[0].y), v = 0.5 * (a[1].x + b[1].x), w = 0.5 * (a[1].y + b[1].y);
  const double q2 = 0.5 * (a[2].y + b[2].y);
  const double ud = d == 0 ? u : (d == 1 ? v : w);
  const double F1 = rho_ln * ud;
  f[0] = F1;
  f[1] = F1 * u;
  f[2] = F1 * v;
  f[3] = F1 * w;
  f[1 + d] += p_hat;
  f[4] = F1 * (0.5 / gm1 * inv_beta_ln - 0.5 * q2) + f[1] * u + f[2] * v + f[3] * w;
}

// Line sums of direction d with the entropy-conserving flux: ac = sum_m D_im
// f#_EC(own, m), av = sum_m D_im f_v,d(m).
template <int N, int d, bool VISC>
__device__ inline void volume_sweep_ec(const double2 (&own)[3], int i, int j, int k, const double* sD,
                                       const double2 (*sp)[GeoR<N>::EB],
                                       const double2 (*sfv)[GeoR<N>::EB], double gm1, double ac[5],
                                       double av[4]) {
  using Gm = GeoR<N>;
  constexpr int NP = Gm::NP;
  const int idx = d == 0 ? i : (d == 1 ? j : k);
#pragma unroll
  for (int v = 0; v < 5; ++v) ac[v] = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) av[c] = 0.0;
  // not unrolled: the pair flux is long, and unrolled copies keep too many
  // values live
#pragma unroll 1
  for (int m = 0; m < NP; ++m) {
    const int lm = d == 0 ? Gm::lds(m, j, k) : (d == 1 ? Gm::lds(i, m, k) : Gm::lds(i, j, m));
    const double Dim = sD[idx * Gm::DS + m];
    const double2 b[3] = {sp[0][lm], sp[1][lm], sp[2][lm]};
    double f[5];
    ec_flux<d>(own, b, gm1, f);
#pragma unroll
    for (int v = 0; v < 5; ++v) ac[v] += Dim * f[v];
    if (VISC) {
      const double2 f01 = sfv[0][lm], f23 = sfv[1][lm];
      av[0] += Dim * f01.x;
      av[1] += Dim * f01.y;
      av[2] += Dim * f23.x;
      av[3] += Dim * f23.y;
    }
  }
}

// Line sums of direction d with the entropy-conserving flux in FP32 (mixed
// precision), relative to the element's reference state (p_ref, beta_ref):
// own, sp = (rho, u), (v, w), (beta - beta_ref, |u|^2), (pi, 0) with
// pi = rho (p - p_ref) / p = rho - 2 p_ref beta.  Then, with sb = beta_a + beta_b,
//   p^ - p_ref = (pi_a + pi_b) / (2 sb),
//   1 / beta_ln - 1 / beta_ref = (2 (F - 1) - (dbeta_a + dbeta_b) / beta_ref) / sb,
// F = atanh f / f of the beta pair (its series less the leading 1 below
// f^2 = 1e-2, where the dropped term is below 2e-10), so no FP32 difference
// of O(p_ref) terms is formed.  ac = sum_m D_im (f#_EC - (0, p_ref e_d,
// F1 e_ref + p_ref {{u_d}})), du = sum_m D_im {{u_d}}, e_ref = p_ref / ((gamma - 1) rho_ref)
// = kappa / beta_ref; the reference parts are added back in FP64 (the
// pressure part vanishes: the rows of D sum to zero).
template <int N, int d, bool VISC>
__device__ inline void volume_sweep_ec_mixed(const float2 (&own)[4], int i, int j, int k,
                                             const float* sD, const float2 (*sp)[GeoR<N>::EB],
                                             const float2 (*sfv)[GeoR<N>::EB], float kap,
                                             float beta_ref, float ibr, float ac[5], float av[4],
                                             float& du) {
  using Gm = GeoR<N>;
  constexpr int NP = Gm::NP;
  const int idx = d == 0 ? i : (d == 1 ? j : k);
#pragma unroll
  for (int v = 0; v < 5; ++v) ac[v] = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c) av[c] = 0.0f;
  du = 0.0f;
#pragma unroll 2
  for (int m = 0; m < NP; ++m) {
    const int lm = d == 0 ? Gm::lds(m, j, k) : (d == 1 ? Gm::lds(i, m, k) : Gm::lds(i, j, m));
    const float Dim = sD[idx * Gm::DS + m];
    const float2 b0 = sp[0][lm], b1 = sp[1][lm], b2 = sp[2][lm], b3 = sp[3][lm];
    const float sr = own[0].x + b0.x, sdb = own[2].x + b2.x;
    const float sb = 2.0f * beta_ref + sdb;
    const float x = __builtin_amdgcn_rcpf(sr * sb);
    const float ir = sb * x, ib = sr * x;
    const float fr = (own[0].x - b0.x) * ir, fb = (own[2].x - b2.x) * ib;
    const float ur = fr * fr, ub = fb * fb;
    float G = 1.0f - ur * (1.0f / 3.0f + ur * (4.0f / 45.0f + ur * (44.0f / 945.0f)));
    float Fs = ub * (1.0f / 3.0f + ub * (0.2f + ub * (1.0f / 7.0f)));
    if (ur >= 1e-2f) G = fr / atanhf(fr);
    if (ub >= 1e-2f) Fs = atanhf(fb) / fb - 1.0f;
    const float um = 0.5f * (own[0].y + b0.y), vm = 0.5f * (own[1].x + b1.x),
                wm = 0.5f * (own[1].y + b1.y);
    const float ud = d == 0 ? um : (d == 1 ? vm : wm);
    const float F1 = 0.5f * sr * G * ud;
    const float dp = 0.5f * (own[3].x + b3.x) * ib;
    const float dib = (2.0f * Fs - sdb * ibr) * ib;
    const float q2m = 0.5f * (own[2].y + b2.y);
    const float X = kap * dib - 0.5f * q2m + (um * um + vm * vm + wm * wm);
    const float s = Dim * F1;
    ac[0] += s;
    ac[1] += s * um;
    ac[2] += s * vm;
    ac[3] += s * wm;
    ac[1 + d] += Dim * dp;
    ac[4] += s * X + Dim * dp * ud;
    du += Dim * ud;
    if (VISC) {
      const float2 f01 = sfv[0][lm], f23 = sfv[1][lm];
      av[0] += Dim * f01.x;
      av[1] += Dim * f01.y;
      av[2] += Dim * f23.x;
      av[3] += Dim * f23.y;
    }
  }
}

// Roe's dissipation sum_k |lambda_k| alpha_k r_k across a face with normal e_d
// (L = lower side, R = upper side; primitives (rho, u, v, w, p) and total
// energies E), linearised at the Roe average: sqrt(rho)-weighted u and
// H = (E + p) / rho, rho~ = sqrt(rho_L rho_R), a~^2 = (gamma - 1)(H~ - |u~|^2 / 2).
// Waves: acoustic u~_d -+ a~, alpha = ([[p]] -+ rho~ a~ [[u_d]]) / (2 a~^2),
// r = (1, u~ -+ a~ e_d, H~ -+ u~_d a~) (eigenvalues with the correction above);
// entropy u~_d, alpha = [[rho]] - [[p]] / a~^2, r = (1, u~, |u~|^2 / 2); shear
// u~_d with rho~ (0, [[u_t]], u~ . [[u_t]]).
template <int d>
__device__ inline void roe_dissipation(const double L[5], double EL, const double R[5], double ER,
                                       double gamma, double D[5]) {
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
  const double un = ut[d];
  const double dp = R[4] - L[4];
  double du[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) du[c] = R[1 + c] - L[1 + c];
  const double al1 = (dp - rho * a * du[d]) / (2.0 * a2);
  const double al5 = (dp + rho * a * du[d]) / (2.0 * a2);
  const double al2 = (R[0] - L[0]) - dp / a2;
  const double cl = sqrt(gamma * L[4] / L[0]), cr = sqrt(gamma * R[4] / R[0]);
  const double l1 = hh_abs(un - a, L[1 + d] - cl, R[1 + d] - cr);
  const double l5 = hh_abs(un + a, L[1 + d] + cl, R[1 + d] + cr);
  const double l2 = fabs(un);
  const double t1 = l1 * al1, t5 = l5 * al5, t2 = l2 * al2, ts = l2 * rho;
  double udt = 0.0;
  D[0] = t1 + t2 + t5;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double sh = c == d ? 0.0 : du[c];
    udt += ut[c] * sh;
    D[1 + c] = t1 * ut[c] + t2 * ut[c] + t5 * ut[c] + ts * sh;
  }
  D[1 + d] += (t5 - t1) * a;
  D[4] = t1 * (H - un * a) + t2 * (0.5 * q2) + t5 * (H + un * a) + ts * udt;
}

// Surface correction of one face task with the entropy-conserving / Roe pair
// (FP64): ((F*_c - F*_v) - (f_c - f_v)(own)) (+-1/w_end),
// F*_c = f#_EC(U_L, U_R) - (1/2) Roe dissipation.  A = own (rho, u, v, w, p,
// beta), q2o = own |u|^2; so, sn: own and neighbour conservative states.
template <int d>
__device__ inline void surface_correction_ec(const double A[6], double q2o, const double so[5],
                                             const double sn[5], bool wall, bool up,
                                             const double fvo[4], const double fvn[4],
                                             const DevPhys& ph, double inv_w, double corr[5]) {
  const double po = A[4];
  {
    const double ud = A[1 + d];
    const double mass = A[0] * ud;
    corr[0] = -mass;
    corr[1] = -mass * A[1] + fvo[0];
    corr[2] = -mass * A[2] + fvo[1];
    corr[3] = -mass * A[3] + fvo[2];
    corr[1 + d] -= po;
    corr[4] = -(so[4] + po) * ud + fvo[3];
  }
  if (wall) {
    corr[1 + d] += po;
    corr[1] -= fvo[0];
    corr[2] -= fvo[1];
    corr[3] -= fvo[2];
    corr[4] -= fvo[3] - (A[1] * fvo[0] + A[2] * fvo[1] + A[3] * fvo[2]);
  } else {
    const double irn = 1.0 / sn[0];
    const double B[5] = {sn[0], sn[1] * irn, sn[2] * irn, sn[3] * irn, 0.0};
    const double q2n = B[1] * B[1] + B[2] * B[2] + B[3] * B[3];
    const double pn = ph.gm1 * (sn[4] - 0.5 * sn[0] * q2n);
    const double Bf[5] = {B[0], B[1], B[2], B[3], pn};
    const double2 a[3] = {double2{A[0], A[1]}, double2{A[2], A[3]}, double2{A[5], q2o}};
    const double2 b[3] = {double2{B[0], B[1]}, double2{B[2], B[3]}, double2{0.5 * sn[0] / pn, q2n}};
    double F[5];
    ec_flux<d>(a, b, ph.gm1, F);
#pragma unroll
    for (int v = 0; v < 5; ++v) corr[v] += F[v];
    if (!ph.central) {
      const double Ao[5] = {A[0], A[1], A[2], A[3], po};
      double Dr[5];
      if (up)
        roe_dissipation<d>(Ao, so[4], Bf, sn[4], ph.gamma, Dr);
      else
        roe_dissipation<d>(Bf, sn[4], Ao, so[4], ph.gamma, Dr);
#pragma unroll
      for (int v = 0; v < 5; ++v) corr[v] -= 0.5 * Dr[v];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) corr[1 + c] -= 0.5 * (fvo[c] + fvn[c]);
  }
  const double sc = up ? inv_w : -inv_w;
#pragma unroll
  for (int v = 0; v < 5; ++v) corr[v] *= sc;
}

template <int N, typename R, bool RK, bool VISC, bool EC>
__global__ __launch_bounds__(Cfg<N>::BS) __attribute__((amdgpu_waves_per_eu(4))) void k_rhs(const double* __restrict__ U,
                                                     const R* __restrict__ ffv,
                                                     double* __restrict__ out,
                                                     double* __restrict__ U_out, DevMesh mesh,
                                                     DevPhys ph, DevBasis basis, Stage st,
                                                     int* __restrict__ status) {
  using Gm = GeoR<N>;
  constexpr int NP = Gm::NP, NF = Gm::NF, NN = Gm::NN, EB = Gm::EB;
  constexpr int EPB = Cfg<N>::EPB, BS = Cfg<N>::BS;
  constexpr bool MIXED = sizeof(R) == 4;
  using V2 = typename V2T<R>::type;
  // entries of sp per node: 4 for the mixed-precision entropy-conserving pair
  constexpr int NSP = EC && MIXED ? 4 : 3;
  __shared__ R sD[NP * Gm::DS];
  // halves of (rho, u), (v, w), (p - p_ref, e - e_ref); with EC the full values
  // (rho, u), (v, w), (beta, |u|^2), in mixed precision (rho, u), (v, w),
  // (beta - beta_ref, |u|^2), (rho (p - p_ref) / p, 0)
  __shared__ V2 sp[EPB][NSP][EB];
  __shared__ V2 sfv[EPB][2][EB];    // f_v,d of the current direction; T - T_ref in P1-P2
  // sX: lifting corrections (P1-P2, as ssq), own f_v,d of the face nodes in
  // components 0..3 (P3-P4), surface corrections (P4-P5).  In P4 every face
  // lane reads and then overwrites only its own (face, node) entries.
  __shared__ R sX[EPB][6][5][NF];
  // neighbour conservative state at the face nodes (P1-P4); the own one too in
  // mixed precision, where the FP32 halves in sp cannot give it back in FP64
  __shared__ double sN[EPB][6][5][NF];
  __shared__ double sO[MIXED ? EPB : 1][6][5][MIXED ? NF : 1];
  R(*ssq)[6][4][NF] = reinterpret_cast<R(*)[6][4][NF]>(&sX[0][0][0][0]);

  const int tid = threadIdx.x;
  const long long nE = mesh.nE;
  const long long stride = nE * NN;
  const long long e0 = static_cast<long long>(xcd_remap(blockIdx.x, gridDim.x)) * EPB;
  // D is fetched with the first loads and written to LDS before the first
  // barrier, so its latency is not paid on its own
  static_assert(NP * NP <= BS, "one lane per entry of D");
  double dval = 0.0;
  if (tid < NP * NP) dval = basis.D[tid];
  const R mu = static_cast<R>(ph.mu), kappa = static_cast<R>(ph.kappa);

  // with one element per workgroup the element index is wave-uniform
  const int le = EPB == 1 ? 0 : tid / NN;
  const int node = tid - le * NN;
  const long long e = EPB == 1 ? e0 : e0 + le;
  const bool active = (EPB == 1 ? tid < NN : le < EPB) && e < nE;
  const int i = node % NP, j = (node / NP) % NP, k = node / NF;
  const int l = Gm::lds(i, j, k);
  int ex0 = 0, ey0 = 0, ez0 = 0;  // coordinates of element e0
  elem_coords(e0 < nE ? e0 : 0, mesh, ex0, ey0, ez0);

  // ---- P1: face lanes --------------------------------------------------
  // FP64: the face lanes only fetch the neighbour's state here and form the
  // lifting corrections after the barrier, with the own values from LDS.
  // Mixed precision: the corrections need FP64 own values, recovered from U.
  // The own state is fetched first, so that it and the neighbour's face node
  // are in flight together.  It stays in registers for the RK update:
  // re-reading it at the end of the workgroup's life would miss in L2.
  double u0[5] = {0, 0, 0, 0, 0}, s0[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
  if (active) {
    load_state(U, stride, e * NN + node, u0);
    if (uses_ref<R>(ph)) load_state(U, stride, e * NN, s0);
  }
  const bool face_lane = tid < n_face_tasks<N>();
  const bool face_ok = face_lane && e0 + FaceTask<N>(face_lane ? tid : 0).le < nE;
  double sn[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
  bool fwall = true;
  if (face_ok) {
    const FaceTask<N> ft(tid);
    const long long te = EPB == 1 ? e0 : e0 + ft.le;
    int fx = ex0, fy = ey0, fz = ez0;
    if (EPB > 1) elem_coords(te, mesh, fx, fy, fz);
    const long long nb = neighbour(mesh, fx, fy, fz, ft.d, ft.up);
    fwall = nb < 0;
    if (!fwall) load_state(U, stride, nb * NN + ft.nb_node(), sn);
    if (MIXED) {
      double so[5];
      load_state(U, stride, te * NN + ft.own_node(), so);
#pragma unroll
      for (int v = 0; v < 5; ++v) sO[ft.le][ft.f][v][ft.ab] = so[v];
      if (VISC) {
        double corr[4];
        lifting_correction(primitives(so, ph), primitives(sn, ph), fwall, mesh, ft.d, ft.up,
                           basis.inv_w_end, corr);
#pragma unroll
        for (int c = 0; c < 4; ++c) ssq[ft.le][ft.f][c][ft.ab] = static_cast<R>(corr[c]);
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sN[ft.le][ft.f][v][ft.ab] = sn[v];
  }

  // ---- P1: node lanes --------------------------------------------------
  V2 own[NSP];
#pragma unroll
  for (int q = 0; q < NSP; ++q) own[q].x = own[q].y = R(0);
  R uo = R(0), vo = R(0), wo = R(0);  // own velocity (full values)
  double p_ref = 0.0, e_ref = 0.0, beta_ref = 0.0, T_ref = 0.0;
  int ex = ex0, ey = ey0, ez = ez0;
  R* sT = reinterpret_cast<R*>(&sfv[le][0][0]);
  if (active) {
    if (EPB > 1) elem_coords(e, mesh, ex, ey, ez);
    const Prim P = primitives(u0, ph);
    if (!(P.rho > 0.0) || !(P.p > 0.0)) status[0] = 1;
    element_ref<R>(s0, ph, p_ref, e_ref, T_ref);
    uo = static_cast<R>(P.u);
    vo = static_cast<R>(P.v);
    wo = static_cast<R>(P.w);
    if (EC && MIXED) {
      // reference: beta_ref = rho_ref / (2 p_ref); e_ref becomes the internal
      // energy p_ref / ((gamma - 1) rho_ref) = kappa / beta_ref
      beta_ref = 0.5 * s0[0] / p_ref;
      e_ref = p_ref / (ph.gm1 * s0[0]);
      own[0].x = static_cast<R>(P.rho);
      own[0].y = static_cast<R>(P.u);
      own[1].x = static_cast<R>(P.v);
      own[1].y = static_cast<R>(P.w);
      own[2].x = static_cast<R>(0.5 * P.rho / P.p - beta_ref);
      own[2].y = static_cast<R>(P.u * P.u + P.v * P.v + P.w * P.w);
      own[NSP - 1].x = static_cast<R>(P.rho * (P.p - p_ref) / P.p);
    } else if (EC) {
      own[0].x = P.rho;
      own[0].y = P.u;
      own[1].x = P.v;
      own[1].y = P.w;
      own[2].x = 0.5 * P.rho / P.p;
      own[2].y = P.u * P.u + P.v * P.v + P.w * P.w;
    } else {
      own[0].x = static_cast<R>(0.5 * P.rho);
      own[0].y = static_cast<R>(0.5 * P.u);
      own[1].x = static_cast<R>(0.5 * P.v);
      own[1].y = static_cast<R>(0.5 * P.w);
      own[2].x = static_cast<R>(0.5 * (P.p - p_ref));
      own[2].y = static_cast<R>(0.5 * (P.e - e_ref));
    }
#pragma unroll
    for (int q = 0; q < NSP; ++q) sp[le][q][l] = own[q];
    if (VISC) sT[l] = static_cast<R>(P.T - T_ref);
  }
  if (tid < NP * NP) sD[(tid / NP) * Gm::DS + tid % NP] = static_cast<R>(dval);
  __syncthreads();

  if (VISC && !MIXED) {
    if (face_ok) {
      const FaceTask<N> ft(tid);
      const int lo = Gm::lds(ft.oi, ft.oj, ft.ok);
      const R* sTf = reinterpret_cast<const R*>(&sfv[ft.le][0][0]);
      const V2 ru = sp[ft.le][0][lo], vw = sp[ft.le][1][lo];
      constexpr double hv = EC ? 1.0 : 2.0;  // sp holds halves unless EC
      const double qo[4] = {hv * ru.y, hv * vw.x, hv * vw.y, sTf[lo]};
      double qs[4];
      wall_lifting_value(mesh, ft.d, qo, qs);
      if (!fwall) {
        const Prim Pn = primitives(sn, ph);
        qs[0] = 0.5 * (qo[0] + Pn.u);
        qs[1] = 0.5 * (qo[1] + Pn.v);
        qs[2] = 0.5 * (qo[2] + Pn.w);
        qs[3] = 0.5 * (qo[3] + Pn.T);
      }
      const double sc = ft.up ? basis.inv_w_end : -basis.inv_w_end;
#pragma unroll
      for (int c = 0; c < 4; ++c) ssq[ft.le][ft.f][c][ft.ab] = static_cast<R>((qs[c] - qo[c]) * sc);
    }
    __syncthreads();
  }

  // ---- P2: lifted gradients ------------------------------------------------
  // Kennedy-Gruber pair: one pass per line direction gives the lifted
  // gradients and the convective flux differencing together; P3 then sweeps
  // the viscous fluxes only.  Entropy-conserving pair: the lifted gradients
  // here, the whole flux differencing in P3.
  R tau[6], qT[3];
#pragma unroll
  for (int c = 0; c < 6; ++c) tau[c] = R(0);
  qT[0] = qT[1] = qT[2] = R(0);
  double ut[5];
  if constexpr (!EC) {
#pragma unroll
    for (int v = 0; v < 5; ++v) ut[v] = 0.0;
    if (active) {
      R g[12];
      fused_direction<N, R, 0, VISC, MIXED, V2>(own, i, j, k, sD, sp[le], sT, ssq[le], mesh.s[0][ex],
                                                e_ref, p_ref, g, ut);
      fused_direction<N, R, 1, VISC, MIXED, V2>(own, i, j, k, sD, sp[le], sT, ssq[le], mesh.s[1][ey],
                                                e_ref, p_ref, g, ut);
      fused_direction<N, R, 2, VISC, MIXED, V2>(own, i, j, k, sD, sp[le], sT, ssq[le], mesh.s[2][ez],
                                                e_ref, p_ref, g, ut);
      if (VISC) {
        if (ph.suth) {  // sT holds T - T_ref (T_ref = 0 in FP64)
          const R r = static_cast<R>(viscosity_ratio(ph, static_cast<double>(sT[l]) + T_ref));
          stress<R>(g, mu * r, kappa * r, tau, qT);
        } else {
          stress<R>(g, mu, kappa, tau, qT);
        }
      }
    }
    if (VISC) __syncthreads();
  } else if (VISC) {
    if (active) {
      R g[12];
      lifted_gradients_half<N, R, V2, false>(sD, sp[le], sT, ssq[le], i, j, k,
                                             static_cast<R>(mesh.s[0][ex]), static_cast<R>(mesh.s[1][ey]),
                                             static_cast<R>(mesh.s[2][ez]), g);
      if (ph.suth) {
        const R r = static_cast<R>(viscosity_ratio(ph, static_cast<double>(sT[l]) + T_ref));
        stress<R>(g, mu * r, kappa * r, tau, qT);
      } else {
        stress<R>(g, mu, kappa, tau, qT);
      }
    }
    __syncthreads();
  }
  if constexpr (EC) {
#pragma unroll
    for (int v = 0; v < 5; ++v) ut[v] = 0.0;
  }

  // ---- P3: line sweeps -------------------------------------------------
  // G of the RK update (node lanes) and the neighbour's face viscous flux
  // (face lanes) are fetched before the last sweep and first used in P4/P5,
  // so that their latency overlaps it.  The entropy-conserving instances,
  // whose sweeps hold more registers, and the two-element workgroups fetch
  // G after P3 and the face flux in P4.
  constexpr bool EARLY = !EC && EPB == 1;
  double gA[5] = {0, 0, 0, 0, 0};
  double fvn_pre[4] = {0, 0, 0, 0};
#define DG_DIRECTION(D)                                                                     \
  {                                                                                         \
    const int idx = D == 0 ? i : (D == 1 ? j : k);                                          \
    const int ab = D == 0 ? j + NP * k : (D == 1 ? i + NP * k : i + NP * j);                \
    if (VISC && active) {                                                                   \
      R fv[4];                                                                              \
      viscous_flux_tau<D, R>(uo, vo, wo, tau, qT, fv);                                      \
      sfv[le][0][l] = V2{fv[0], fv[1]};                                                     \
      sfv[le][1][l] = V2{fv[2], fv[3]};                                                     \
      if (idx == 0)                                                                         \
        _Pragma("unroll") for (int c = 0; c < 4; ++c) sX[le][2 * D][c][ab] = fv[c];         \
      if (idx == N)                                                                         \
        _Pragma("unroll") for (int c = 0; c < 4; ++c) sX[le][2 * D + 1][c][ab] = fv[c];     \
    }                                                                                       \
    if constexpr (D == 2 && EARLY) {                                                        \
      if (RK && active && st.read_G)                                                        \
        _Pragma("unroll") for (int v = 0; v < 5; ++v) gA[v] = load_once(&out[v * stride + e * NN + node]); \
      if (VISC && face_ok && !fwall) {                                                      \
        const FaceTask<N> ft(tid);                                                          \
        const long long nb = neighbour(mesh, ex0, ey0, ez0, ft.d, ft.up);                   \
        const R* src = ffv + nb * (6 * 4 * NF) + ((ft.f ^ 1) * 4) * NF + ft.ab;             \
        _Pragma("unroll") for (int c = 0; c < 4; ++c) fvn_pre[c] = static_cast<double>(load_once(&src[c * NF])); \
      }                                                                                     \
    }                                                                                       \
    __syncthreads();                                                                        \
    if (active) {                                                                           \
      const double sd = mesh.s[D][D == 0 ? ex : (D == 1 ? ey : ez)];                         \
      if constexpr (!EC) {                                                                  \
        R av[4];                                                                            \
        viscous_sweep<N, R, D, V2>(i, j, k, sD, sfv[le], av);                               \
        _Pragma("unroll") for (int c = 0; c < 4; ++c) ut[1 + c] += sd * static_cast<double>(av[c]); \
      } else {                                                                              \
        R ac[5], av[4], du = R(0);                                                          \
        if constexpr (MIXED)                                                                \
          volume_sweep_ec_mixed<N, D, VISC>(own, i, j, k, sD, sp[le], sfv[le],              \
                                            static_cast<float>(0.5 / ph.gm1),              \
                                            static_cast<float>(beta_ref),                  \
                                            static_cast<float>(1.0 / beta_ref), ac, av, du); \
        else                                                                                \
          volume_sweep_ec<N, D, VISC>(own, i, j, k, sD, sp[le], sfv[le], ph.gm1, ac, av);   \
        ut[0] -= sd * static_cast<double>(R(2) * ac[0]);                                    \
        _Pragma("unroll") for (int c = 0; c < 4; ++c)                                       \
            ut[1 + c] -= sd * static_cast<double>(R(2) * ac[1 + c] - av[c]);                \
        if (MIXED)                                                                          \
          ut[4] -= sd * 2.0 * (e_ref * static_cast<double>(ac[0]) +                         \
                               p_ref * static_cast<double>(du));                            \
      }                                                                                     \
    }                                                                                       \
    if constexpr (D < 2) __syncthreads();                                                   \
  }
  // No barrier after the last sweep: P4 reads the own face states (sp, sN,
  // sO) and the own face viscous fluxes stored before that sweep's barrier,
  // and overwrites only its own face entries of sX, which no sweep reads, so
  // each wave goes on to its surface terms as soon as its sweep is done.
  if (EC || VISC) {
    DG_DIRECTION(0)
    DG_DIRECTION(1)
    DG_DIRECTION(2)
  }
#undef DG_DIRECTION

  if (!EARLY || !VISC) {  // (Euler with the Kennedy-Gruber pair: no sweeps in P3)
    if (RK && active && st.read_G)
#pragma unroll
      for (int v = 0; v < 5; ++v) gA[v] = load_once(&out[v * stride + e * NN + node]);
  }

  // ---- P4: surface corrections (face lanes, FP64) -----------------------
  if (face_ok) {
    const FaceTask<N> ft(tid);
    const long long te = EPB == 1 ? e0 : e0 + ft.le;
    int fx = ex0, fy = ey0, fz = ez0;
    if (EPB > 1) elem_coords(te, mesh, fx, fy, fz);
    const long long nb = neighbour(mesh, fx, fy, fz, ft.d, ft.up);
    double fvo[4] = {0, 0, 0, 0}, fvn[4] = {fvn_pre[0], fvn_pre[1], fvn_pre[2], fvn_pre[3]};
    if (!EARLY && VISC && !fwall) {
      const R* src = ffv + nb * (6 * 4 * NF) + ((ft.f ^ 1) * 4) * NF + ft.ab;
#pragma unroll
      for (int c = 0; c < 4; ++c) fvn[c] = static_cast<double>(load_once(&src[c * NF]));
    }
    double A[6], so[5], sn[5], q2o = 0.0;
    if (MIXED) {
#pragma unroll
      for (int v = 0; v < 5; ++v) so[v] = sO[ft.le][ft.f][v][ft.ab];
      const Prim P = primitives(so, ph);
      A[0] = P.rho; A[1] = P.u; A[2] = P.v; A[3] = P.w; A[4] = P.p; A[5] = P.e;
      if (EC) {
        A[5] = 0.5 * P.rho / P.p;
        q2o = P.u * P.u + P.v * P.v + P.w * P.w;
      }
    } else if (EC) {
      // (rho, u, v, w, beta, |u|^2) from sp; p and E recovered from them
      const int lo = Gm::lds(ft.oi, ft.oj, ft.ok);
      const V2 a0 = sp[ft.le][0][lo], a1 = sp[ft.le][1][lo], a2 = sp[ft.le][2][lo];
      A[0] = a0.x; A[1] = a0.y; A[2] = a1.x; A[3] = a1.y;
      A[4] = 0.5 * a0.x / a2.x; A[5] = a2.x;
      q2o = a2.y;
      so[0] = A[0];
      so[1] = A[0] * A[1];
      so[2] = A[0] * A[2];
      so[3] = A[0] * A[3];
      so[4] = A[4] / ph.gm1 + 0.5 * A[0] * q2o;
    } else {
      // FP64: the halves in sp are exact, and p_ref = e_ref = 0
      const int lo = Gm::lds(ft.oi, ft.oj, ft.ok);
      const V2 a0 = sp[ft.le][0][lo], a1 = sp[ft.le][1][lo], a2 = sp[ft.le][2][lo];
      A[0] = 2.0 * a0.x; A[1] = 2.0 * a0.y; A[2] = 2.0 * a1.x; A[3] = 2.0 * a1.y;
      A[4] = 2.0 * a2.x; A[5] = 2.0 * a2.y;
      so[0] = A[0];
      so[1] = A[0] * A[1];
      so[2] = A[0] * A[2];
      so[3] = A[0] * A[3];
      so[4] = A[0] * A[5];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sn[v] = sN[ft.le][ft.f][v][ft.ab];
    if (VISC) {
#pragma unroll
      for (int c = 0; c < 4; ++c) fvo[c] = static_cast<double>(sX[ft.le][ft.f][c][ft.ab]);
    }
    // slip, adiabatic wall of the wall model: the viscous wall flux is the
    // modelled shear stress (negative on an upper wall), the own normal
    // stress and no energy flux
    bool wm = false;
    if (VISC && fwall && mesh.tauw != nullptr &&
        pick3(mesh.bc[0], mesh.bc[1], mesh.bc[2], ft.d) == DG_BC_WALL_MODEL) {
      wm = true;
      const long long w = wall_face_index(mesh, fx, fy, fz, ft.d, ft.up);
      const double* tw = mesh.tauw + w * 3 * NF + ft.ab;
      const double sg = ft.up ? -1.0 : 1.0;
      fvn[0] = ft.d == 0 ? fvo[0] : sg * tw[0];
      fvn[1] = ft.d == 1 ? fvo[1] : sg * tw[NF];
      fvn[2] = ft.d == 2 ? fvo[2] : sg * tw[2 * NF];
      fvn[3] = 0.0;
    }
    double corr[5];
    if constexpr (EC) {
      if (ft.d == 0) surface_correction_ec<0>(A, q2o, so, sn, fwall, ft.up, fvo, fvn, ph, basis.inv_w_end, corr);
      if (ft.d == 1) surface_correction_ec<1>(A, q2o, so, sn, fwall, ft.up, fvo, fvn, ph, basis.inv_w_end, corr);
      if (ft.d == 2) surface_correction_ec<2>(A, q2o, so, sn, fwall, ft.up, fvo, fvn, ph, basis.inv_w_end, corr);
    } else if constexpr (MIXED) {
      // mixed precision: the surface fluxes in FP32 from FP64 differences
      const Prim Po = primitives(so, ph);
      float c32[5];
      if (ft.d == 0) surface_correction_f32<0>(Po, so, sn, fwall, ft.up, fvo, fvn, ph, basis.inv_w_end, c32);
      if (ft.d == 1) surface_correction_f32<1>(Po, so, sn, fwall, ft.up, fvo, fvn, ph, basis.inv_w_end, c32);
      if (ft.d == 2) surface_correction_f32<2>(Po, so, sn, fwall, ft.up, fvo, fvn, ph, basis.inv_w_end, c32);
#pragma unroll
      for (int v = 0; v < 5; ++v) corr[v] = c32[v];
    } else {
      if (ft.d == 0) surface_correction<0>(A, so, sn, fwall, ft.up, fvo, fvn, ph, basis.inv_w_end, corr);
      if (ft.d == 1) surface_correction<1>(A, so, sn, fwall, ft.up, fvo, fvn, ph, basis.inv_w_end, corr);
      if (ft.d == 2) surface_correction<2>(A, so, sn, fwall, ft.up, fvo, fvn, ph, basis.inv_w_end, corr);
    }
    if (wm) {
      // the wall branch above subtracted the isothermal wall's viscous flux
      // (own stresses, heat flux only); swap in the wall-model flux fvn
      const double sc = ft.up ? basis.inv_w_end : -basis.inv_w_end;
      const double iso_e = fvo[3] - (A[1] * fvo[0] + A[2] * fvo[1] + A[3] * fvo[2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) corr[1 + c] += sc * (fvo[c] - fvn[c]);
      corr[4] += sc * (iso_e - fvn[3]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sX[ft.le][ft.f][v][ft.ab] = static_cast<R>(corr[v]);
  }
  __syncthreads();

  // ---- P5: surface terms, scaling, output -------------------------------
  if (active) {
    const double sx = mesh.s[0][ex], sy = mesh.s[1][ey], sz = mesh.s[2][ez];
    // a node lies on at most one face per direction: one branch each
    if (i == 0 || i == N) {
      const int f = i == 0 ? 0 : 1;
#pragma unroll
      for (int v = 0; v < 5; ++v) ut[v] -= sx * static_cast<double>(sX[le][f][v][j + NP * k]);
    }
    if (j == 0 || j == N) {
      const int f = j == 0 ? 2 : 3;
#pragma unroll
      for (int v = 0; v < 5; ++v) ut[v] -= sy * static_cast<double>(sX[le][f][v][i + NP * k]);
    }
    if (k == 0 || k == N) {
      const int f = k == 0 ? 4 : 5;
#pragma unroll
      for (int v = 0; v < 5; ++v) ut[v] -= sz * static_cast<double>(sX[le][f][v][i + NP * j]);
    }
    const long long idx = e * NN + node;
    if (RK) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double gv = st.A * gA[v] + st.dt * ut[v];
        store_once(&out[v * stride + idx], gv);
        // the entropy-conserving instance reads U again here: holding it
        // from the first phase spills its registers (6 % slower)
        store_once(&U_out[v * stride + idx], (EC ? U[v * stride + idx] : u0[v]) + st.B * gv);
      }
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) store_once(&out[v * stride + idx], ut[v]);
    }
  }
}

template <int N, typename R>
hipError_t face_flux_n(const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                       void* ffv, hipStream_t s) {
  hipLaunchKernelGGL((k_face_flux<N, R>), dim3(n_blocks<N>(m.nE)), dim3(Cfg<N>::BS), 0, s, U,
                     static_cast<R*>(ffv), m, p, b);
  return hipGetLastError();
}

template <int N, typename R, bool RK, bool VISC, bool EC>
void launch_k_rhs(const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                  const void* ffv, double* out, double* U_out, const Stage& st, int* status,
                  hipStream_t s) {
  hipLaunchKernelGGL((k_rhs<N, R, RK, VISC, EC>), dim3(n_blocks<N>(m.nE)), dim3(Cfg<N>::BS), 0, s,
                     U, static_cast<const R*>(ffv), out, U_out, m, p, b, st, status);
}

template <int N, typename R, bool RK>
hipError_t rhs_n(const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                 const void* ffv, double* out, double* U_out, const Stage& st, int* status,
                 hipStream_t s) {
  if constexpr (sizeof(R) == sizeof(double)) {
    if (p.ec) {
      if (p.viscous)
        launch_k_rhs<N, R, RK, true, true>(m, p, b, U, ffv, out, U_out, st, status, s);
      else
        launch_k_rhs<N, R, RK, false, true>(m, p, b, U, ffv, out, U_out, st, status, s);
      return hipGetLastError();
    }
  } else {
    if (p.ec) {
      if (!p.mixed_ref) return hipErrorInvalidValue;  // rejected at init: needs the reference state
      if (p.viscous)
        launch_k_rhs<N, R, RK, true, true>(m, p, b, U, ffv, out, U_out, st, status, s);
      else
        launch_k_rhs<N, R, RK, false, true>(m, p, b, U, ffv, out, U_out, st, status, s);
      return hipGetLastError();
    }
  }
  if (p.viscous)
    launch_k_rhs<N, R, RK, true, false>(m, p, b, U, ffv, out, U_out, st, status, s);
  else
    launch_k_rhs<N, R, RK, false, false>(m, p, b, U, ffv, out, U_out, st, status, s);
  return hipGetLastError();
}

template <typename R, bool RK>
hipError_t rhs_dispatch(int N, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                        const double* U, const void* ffv, double* out, double* U_out,
                        const Stage& st, int* status, hipStream_t s) {
  switch (N) {
    case 3: return rhs_n<3, R, RK>(m, p, b, U, ffv, out, U_out, st, status, s);
    case 5: return rhs_n<5, R, RK>(m, p, b, U, ffv, out, U_out, st, status, s);
    case 7: return rhs_n<7, R, RK>(m, p, b, U, ffv, out, U_out, st, status, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace


hipError_t launch_face_flux(int N, int precision, const DevMesh& m, const DevPhys& p,
                            const DevBasis& b, const double* U, void* ffv, hipStream_t s) {
  if (m.nE <= 0 || !p.viscous) return hipSuccess;
  const bool f32 = precision != DG_FP64;
  switch (N) {
    case 3: return f32 ? face_flux_n<3, float>(m, p, b, U, ffv, s) : face_flux_n<3, double>(m, p, b, U, ffv, s);
    case 5: return f32 ? face_flux_n<5, float>(m, p, b, U, ffv, s) : face_flux_n<5, double>(m, p, b, U, ffv, s);
    case 7: return f32 ? face_flux_n<7, float>(m, p, b, U, ffv, s) : face_flux_n<7, double>(m, p, b, U, ffv, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rhs(int N, int precision, const DevMesh& m, const DevPhys& p,
                      const DevBasis& b, const double* U, const void* ffv, double* Ut,
                      int* status, hipStream_t s) {
  if (m.nE <= 0) return hipSuccess;
  const Stage st{0.0, 0.0, 0.0, 0};
  return precision != DG_FP64
             ? rhs_dispatch<float, false>(N, m, p, b, U, ffv, Ut, nullptr, st, status, s)
             : rhs_dispatch<double, false>(N, m, p, b, U, ffv, Ut, nullptr, st, status, s);
}

hipError_t launch_rk_stage(int N, int precision, const DevMesh& m, const DevPhys& p,
                           const DevBasis& b, const double* U, const void* ffv, double* G,
                           double* U_out, const Stage& st, int* status, hipStream_t s) {
  if (m.nE <= 0) return hipSuccess;
  return precision != DG_FP64
             ? rhs_dispatch<float, true>(N, m, p, b, U, ffv, G, U_out, st, status, s)
             : rhs_dispatch<double, true>(N, m, p, b, U, ffv, G, U_out, st, status, s);
}

}  // namespace dg
