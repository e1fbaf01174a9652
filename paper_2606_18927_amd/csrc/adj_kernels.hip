// Vector-Jacobian product (adjoint) of the DGSEM right-hand side, FP64.
//
// Ubar = (dL/dU)^T lam is evaluated as a gather: every element computes the
// cotangent of its own nodal state and pulls what its neighbours' equations
// contribute through shared face nodes, so no atomics are needed and the
// result is deterministic.  Two kernels:
//
//   k_vjp_a : lam (+ neighbour lam at face nodes), U ->
//             the forward BR1 gradients of U (recomputed in LDS, as in the
//             forward right-hand side), then
//             gbar = cotangent of the lifted gradients (12 per node) and the
//             part of Ubar that does not pass through the lifting:
//               * volume split form: for each line pair (i, m),
//                 Pbar_i += -2 s_d J1(P_i, P_m)^T (D_im lam_i + D_mi lam_m),
//                 J1 = d f#(a, b) / d a of the symmetric two-point flux
//                 (Kennedy-Gruber, or Chandrashekar's with its logarithmic
//                 means differentiated on the branch the forward takes);
//               * viscous volume term: Fvbar_d(m) = s_d sum_i D_im lam_i, then
//                 the transpose of f_v,d(u, grad) -> (ubar, gbar);
//               * each face node's numerical flux, which enters both sides'
//                 equations, with the combined cotangent
//                 phi = -(sc_o s_o lam_o + sc_n s_n lam_n)  (sc = +-1/w_end);
//                 the own physical flux with -sc_o s_o lam_o;
//               * the primitive map P(U) transposed.
//   k_vjp_b : gbar (+ neighbour gbar at face nodes) -> qbar of q = (u, v, w, T)
//             through the transposed BR1 lifting, then Ubar += (dq/dU)^T qbar.
//
// The Roe dissipation's derivative is written out in reverse mode.  Non-smooth
// points: |u_d| and the max of the Lax-Friedrichs speed, and |lambda| and the
// entropy correction's branch of the Roe flux, take the derivative of the
// branch that is active (ties to the lower side L), as the CPU oracle's
// reverse mode does.
#include "dg_device.hpp"

namespace dg {
namespace {

// abar += (d f#_d(a, b) / d a)^T mu, a and b primitive (rho, u, v, w, p, e).
template <int d>
__device__ inline void kg_vjp(const double a[6], const double b[6], const double mu[5],
                              double abar[6]) {
  const double rho = 0.5 * (a[0] + b[0]);
  const double u0 = 0.5 * (a[1] + b[1]), u1 = 0.5 * (a[2] + b[2]), u2 = 0.5 * (a[3] + b[3]);
  const double p = 0.5 * (a[4] + b[4]);
  const double e = 0.5 * (a[5] + b[5]);
  const double ud = d == 0 ? u0 : (d == 1 ? u1 : u2);
  const double mass = rho * ud;
  const double S = mu[0] + u0 * mu[1] + u1 * mu[2] + u2 * mu[3] + e * mu[4];
  abar[0] += 0.5 * ud * S;
  abar[1] += 0.5 * mass * mu[1];
  abar[2] += 0.5 * mass * mu[2];
  abar[3] += 0.5 * mass * mu[3];
  abar[1 + d] += 0.5 * (rho * S + p * mu[4]);
  abar[4] += 0.5 * (mu[1 + d] + ud * mu[4]);
  abar[5] += 0.5 * mass * mu[4];
}

// abar += (d f_d(a) / d a)^T mu for the Euler flux
// f = (rho u_d, rho u u_d + p e_d, (rho e + p) u_d).
template <int d>
__device__ inline void euler_vjp(const double a[6], const double mu[5], double abar[6]) {
  const double rho = a[0], ud = a[1 + d], p = a[4], e = a[5];
  const double Sk = a[1] * mu[1] + a[2] * mu[2] + a[3] * mu[3];
  abar[0] += ud * (mu[0] + Sk + e * mu[4]);
  abar[1] += rho * ud * mu[1];
  abar[2] += rho * ud * mu[2];
  abar[3] += rho * ud * mu[3];
  abar[1 + d] += rho * (mu[0] + Sk) + (rho * e + p) * mu[4];
  abar[4] += mu[1 + d] + ud * mu[4];
  abar[5] += rho * ud * mu[4];
}

// Ubar += (dP/dU)^T Pbar + (dT/dU)^T Tbar, P = (rho, u, v, w, p, e), T = p/(rho R).
__device__ inline void prim_vjp(const double s[5], const double Pb[6], double Tb,
                                const DevPhys& ph, double Ub[5]) {
  const double ir = 1.0 / s[0];
  const double u = s[1] * ir, v = s[2] * ir, w = s[3] * ir;
  const double q2 = u * u + v * v + w * w;
  const double p = ph.gm1 * (s[4] - 0.5 * s[0] * q2);
  const double e = s[4] * ir;
  const double T = p * ph.inv_R * ir;
  const double pb = Pb[4] + Tb * ir * ph.inv_R;
  const double rb = Pb[0] - Tb * T * ir;
  Ub[0] += rb - ir * (u * Pb[1] + v * Pb[2] + w * Pb[3]) + 0.5 * ph.gm1 * q2 * pb - e * ir * Pb[5];
  Ub[1] += ir * Pb[1] - ph.gm1 * u * pb;
  Ub[2] += ir * Pb[2] - ph.gm1 * v * pb;
  Ub[3] += ir * Pb[3] - ph.gm1 * w * pb;
  Ub[4] += ph.gm1 * pb + ir * Pb[5];
}

// abar += lb d(|u_d| + c)/dP, c = sqrt(gamma p / rho).
template <int d>
__device__ inline void speed_vjp(const double a[6], double lb, const DevPhys& ph, double abar[6]) {
  const double c = sqrt(ph.gamma * a[4] / a[0]);
  const double ud = a[1 + d];
  abar[1 + d] += lb * (ud > 0.0 ? 1.0 : (ud < 0.0 ? -1.0 : 0.0));
  abar[4] += lb * 0.5 * c / a[4];
  abar[0] -= lb * 0.5 * c / a[0];
}

__device__ inline void to_prim(const double s[5], const DevPhys& ph, double a[6]) {
  const Prim P = primitives(s, ph);
  a[0] = P.rho;
  a[1] = P.u;
  a[2] = P.v;
  a[3] = P.w;
  a[4] = P.p;
  a[5] = P.e;
}

// ---- entropy-conserving / Roe pair ----

// Logarithmic-mean factors of f = (x_a - x_b) / (x_a + x_b) (the forward
// pair's switch: series for f^2 < 1e-4, atanh otherwise):
//   G = f / atanh f (x_ln = (x_a + x_b) G / 2),  F = atanh f / f (1 / x_ln = 2 F / (x_a + x_b)),
// with dG = dG/df and dF = dF/df.
__device__ inline void ln_mean_factors(double f, double& G, double& dG, double& F, double& dF,
                                       bool want_G) {
  const double u = f * f;
  if (u < 1e-4) {
    G = 1.0 - u * (1.0 / 3.0 + u * (4.0 / 45.0 + u * (44.0 / 945.0)));
    dG = -2.0 * f * (1.0 / 3.0 + u * (8.0 / 45.0 + u * (132.0 / 945.0)));
    F = 1.0 + u * (1.0 / 3.0 + u * (0.2 + u * (1.0 / 7.0)));
    dF = 2.0 * f * (1.0 / 3.0 + u * (0.4 + u * (3.0 / 7.0)));
  } else {
    const double t = atanh(f), r = f / (1.0 - u);
    if (want_G) {
      G = f / t;
      dG = (t - r) / (t * t);
    } else {
      F = t / f;
      dF = (r - t) / u;
    }
  }
}

// abar += (d f#_EC(a, b) / d a)^T mu for Chandrashekar's flux along d, a and b
// = (rho, u, v, w, p, beta), beta = rho / (2 p); abar[5] is the cotangent of
// beta (p enters the flux only through beta).  With um = {{u}},
// q2m = {{|u|^2}}, F1 = rho_ln um_d, p^ = {{rho}} / (2 {{beta}}) and
// kappa = 1 / (2 (gamma - 1)), mu . f# = F1 A + p^ Bp where
//   A = mu_0 + mu_m . um + mu_4 (kappa / beta_ln - q2m / 2 + |um|^2),  Bp = mu_{1+d} + mu_4 um_d.
template <int d>
__device__ inline void ec_vjp(const double a[6], const double b[6], const double mu[5],
                              double gm1, double abar[6]) {
  const double sr = a[0] + b[0], sb = a[5] + b[5];
  const double ir = 1.0 / sr, ib = 1.0 / sb;
  double G, dG, F, dF, unused0, unused1;
  ln_mean_factors((a[0] - b[0]) * ir, G, dG, unused0, unused1, true);
  ln_mean_factors((a[5] - b[5]) * ib, unused0, unused1, F, dF, false);
  const double rho_ln = 0.5 * sr * G;
  const double ibl = 2.0 * ib * F;
  const double p_hat = 0.5 * sr * ib;
  const double um[3] = {0.5 * (a[1] + b[1]), 0.5 * (a[2] + b[2]), 0.5 * (a[3] + b[3])};
  const double q2m = 0.5 * (a[1] * a[1] + a[2] * a[2] + a[3] * a[3] + b[1] * b[1] + b[2] * b[2] + b[3] * b[3]);
  const double um2 = um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
  const double F1 = rho_ln * um[d];
  const double kap = 0.5 / gm1;
  const double A = mu[0] + mu[1] * um[0] + mu[2] * um[1] + mu[3] * um[2] +
                   mu[4] * (kap * ibl - 0.5 * q2m + um2);
  const double Bp = mu[1 + d] + mu[4] * um[d];
  // d rho_ln / d rho_a = G / 2 + rho_b G' / sr;  d (1 / beta_ln) / d beta_a = -2 ib^2 F + 4 beta_b ib^3 F'
  const double drl = 0.5 * G + b[0] * dG * ir;
  const double dibl = ib * ib * (-2.0 * F + 4.0 * b[5] * ib * dF);
  abar[0] += A * um[d] * drl + 0.5 * ib * Bp;
  abar[5] += F1 * mu[4] * kap * dibl - 0.5 * sr * ib * ib * Bp;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double sk = F1 * (mu[1 + k] + 2.0 * mu[4] * um[k]);
    if (k == d) sk += mu[4] * p_hat + A * rho_ln;
    abar[1 + k] += 0.5 * sk - 0.5 * F1 * mu[4] * a[1 + k];
  }
}

// Pb += the (rho, u, v, w, p) cotangent of Pbe, whose slot 5 is the cotangent
// of beta = rho / (2 p) at the primitives a.
__device__ inline void fold_beta(const double a[6], const double Pbe[6], double Pb[6]) {
  const double ip = 1.0 / a[4];
#pragma unroll
  for (int q = 0; q < 5; ++q) Pb[q] += Pbe[q];
  Pb[0] += 0.5 * ip * Pbe[5];
  Pb[4] -= a[5] * ip * Pbe[5];
}

// lam_bar, lamL_bar, lamR_bar += gb d hh(lam, lamL, lamR): Harten-Hyman |lambda|
// (the branch and the max that the values select, ties to the first argument).
__device__ inline void hh_vjp(double lam, double lamL, double lamR, double gb, double& lb,
                              double& lLb, double& lRb) {
  const double d1 = lam - lamL, d2 = lamR - lam;
  const bool first = d1 >= d2;
  const double delta = first ? d1 : d2;
  if (delta > 0.0 && fabs(lam) < delta) {
    const double bd = gb * (delta * delta - lam * lam) / (2.0 * delta * delta);
    lb += gb * lam / delta + (first ? bd : -bd);
    if (first)
      lLb -= bd;
    else
      lRb += bd;
  } else {
    lb += lam > 0.0 ? gb : (lam < 0.0 ? -gb : 0.0);
  }
}

// Pb += -(1/2) (d Roe(U_L, U_R) / d P_own)^T phi in the own primitives
// (rho, u, v, w, p, e): reverse mode of the Roe dissipation (the forward
// quantities of that function, then their cotangents in reverse order), own =
// L when own_L; E = rho e carries the total-energy cotangent into rho and e.
template <int d>
__device__ inline void roe_vjp(const double so[5], const double sn[5], bool own_L,
                               const double phi[5], const DevPhys& ph, double Pb[6]) {
  const double* sL = own_L ? so : sn;
  const double* sR = own_L ? sn : so;
  double L[5], R[5];
  {
    const double il = 1.0 / sL[0], ir = 1.0 / sR[0];
    L[0] = sL[0];
    R[0] = sR[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      L[1 + c] = sL[1 + c] * il;
      R[1 + c] = sR[1 + c] * ir;
    }
    L[4] = ph.gm1 * (sL[4] - 0.5 * sL[0] * (L[1] * L[1] + L[2] * L[2] + L[3] * L[3]));
    R[4] = ph.gm1 * (sR[4] - 0.5 * sR[0] * (R[1] * R[1] + R[2] * R[2] + R[3] * R[3]));
  }
  const double EL = sL[4], ER = sR[4];
  // forward
  const double sl = sqrt(L[0]), sr = sqrt(R[0]);
  const double isum = 1.0 / (sl + sr);
  const double wl = sl * isum, wr = sr * isum;
  double ut[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) ut[c] = wl * L[1 + c] + wr * R[1 + c];
  const double hL = (EL + L[4]) / L[0], hR = (ER + R[4]) / R[0];
  const double H = wl * hL + wr * hR;
  const double q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  const double a2 = ph.gm1 * (H - 0.5 * q2);
  const double a = sqrt(a2);
  const double rho = sl * sr;
  const double un = ut[d];
  const double dp = R[4] - L[4];
  const double dud = R[1 + d] - L[1 + d];
  const double i2a2 = 0.5 / a2;
  const double al1 = (dp - rho * a * dud) * i2a2, al5 = (dp + rho * a * dud) * i2a2;
  const double al2 = (R[0] - L[0]) - dp / a2;
  const double cl = sqrt(ph.gamma * L[4] / L[0]), cr = sqrt(ph.gamma * R[4] / R[0]);
  const double l1 = hh_abs(un - a, L[1 + d] - cl, R[1 + d] - cr);
  const double l5 = hh_abs(un + a, L[1 + d] + cl, R[1 + d] + cr);
  const double l2 = fabs(un);
  const double t1 = l1 * al1, t5 = l5 * al5, t2 = l2 * al2, ts = l2 * rho;
  const double T = t1 + t2 + t5;
  // reverse, with the cotangent -phi/2 of the dissipation
  double g[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) g[v] = -0.5 * phi[v];
  double Lb[5] = {0, 0, 0, 0, 0}, Rb[5] = {0, 0, 0, 0, 0};
  double Tb = g[0], tsb = 0.0, udtb = g[4] * ts, utb[3], udt = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double sh = c == d ? 0.0 : R[1 + c] - L[1 + c];
    udt += ut[c] * sh;
    Tb += g[1 + c] * ut[c];
    utb[c] = g[1 + c] * T + udtb * sh;
    tsb += g[1 + c] * sh;
    // the shear jump (c != d): ts d(D_{1+c})/d du_c + ut_c d(D_4)/d du_c
    const double dub = c == d ? 0.0 : g[1 + c] * ts + udtb * ut[c];
    Rb[1 + c] += dub;
    Lb[1 + c] -= dub;
  }
  double t5b = g[1 + d] * a + g[4] * (H + un * a) + Tb;
  double t1b = -g[1 + d] * a + g[4] * (H - un * a) + Tb;
  const double t2b = g[4] * 0.5 * q2 + Tb;
  tsb += g[4] * udt;
  double ab = (g[1 + d] + g[4] * un) * (t5 - t1);
  double Hb = g[4] * (t1 + t5);
  double unb = g[4] * a * (t5 - t1);
  double q2b = g[4] * 0.5 * t2;
  const double l2b = tsb * rho + t2b * al2;
  double rhob = tsb * l2;
  const double al2b = t2b * l2, al5b = t5b * l5, al1b = t1b * l1;
  unb += un > 0.0 ? l2b : (un < 0.0 ? -l2b : 0.0);
  double b5 = 0.0, bL5 = 0.0, bR5 = 0.0, b1 = 0.0, bL1 = 0.0, bR1 = 0.0;
  hh_vjp(un + a, L[1 + d] + cl, R[1 + d] + cr, t5b * al5, b5, bL5, bR5);
  hh_vjp(un - a, L[1 + d] - cl, R[1 + d] - cr, t1b * al1, b1, bL1, bR1);
  unb += b5 + b1;
  ab += b5 - b1;
  Lb[1 + d] += bL5 + bL1;
  Rb[1 + d] += bR5 + bR1;
  const double clb = bL5 - bL1, crb = bR5 - bR1;
  Lb[4] += clb * cl / (2.0 * L[4]);
  Lb[0] -= clb * cl / (2.0 * L[0]);
  Rb[4] += crb * cr / (2.0 * R[4]);
  Rb[0] -= crb * cr / (2.0 * R[0]);
  Rb[0] += al2b;
  Lb[0] -= al2b;
  const double dpb = -al2b / a2 + (al1b + al5b) * i2a2;
  double a2b = al2b * dp / (a2 * a2) - (al1b * al1 + al5b * al5) / a2;
  const double dal = (al5b - al1b) * i2a2;
  rhob += dal * a * dud;
  ab += dal * rho * dud;
  const double dudb = dal * rho * a;
  Rb[1 + d] += dudb;
  Lb[1 + d] -= dudb;
  Rb[4] += dpb;
  Lb[4] -= dpb;
  utb[d] += unb;
  double slb = rhob * sr, srb = rhob * sl;
  a2b += ab / (2.0 * a);
  Hb += a2b * ph.gm1;
  q2b -= 0.5 * a2b * ph.gm1;
  double wlb = Hb * hL, wrb = Hb * hR;
  const double hLb = Hb * wl, hRb = Hb * wr;
  const double ELb = hLb / L[0], ERb = hRb / R[0];
  Lb[4] += ELb;
  Lb[0] -= ELb * hL;
  Rb[4] += ERb;
  Rb[0] -= ERb * hR;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double u_b = utb[c] + 2.0 * q2b * ut[c];
    wlb += u_b * L[1 + c];
    wrb += u_b * R[1 + c];
    Lb[1 + c] += u_b * wl;
    Rb[1 + c] += u_b * wr;
  }
  slb += (wlb - wrb) * sr * isum * isum;
  srb += (wrb - wlb) * sl * isum * isum;
  Lb[0] += slb / (2.0 * sl);
  Rb[0] += srb / (2.0 * sr);
  // the own side: (rho, u, v, w, p) and E = rho e
  const double* Xb = own_L ? Lb : Rb;
  const double Eb = own_L ? ELb : ERb;
#pragma unroll
  for (int q = 0; q < 5; ++q) Pb[q] += Xb[q];
  Pb[0] += Eb * so[4] / so[0];
  Pb[5] += Eb * so[0];
}

// Cotangents of one face node of the own element (o) in k_vjp_a: the state
// cotangent Ud (the primitive map already applied), the cotangent Fvb of the
// own normal viscous flux f_v,d, and om, the cotangent of the u . tau_d term
// that a wall removes from the viscous flux.
template <int d, bool EC>
__device__ inline void face_vjp(const double so[5], const double lo[5], const double sn[5],
                                const double ln[5], bool wall, bool up, double s_o, double s_n,
                                const DevPhys& ph, double inv_w, double Ud[5], double Fvb[4],
                                double& om) {
  double Po[6];
  to_prim(so, ph, Po);
  const double sc_o = up ? inv_w : -inv_w;
  double psi[5], phi[5], Pb[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int v = 0; v < 5; ++v) psi[v] = -sc_o * s_o * lo[v];
#pragma unroll
  for (int v = 0; v < 5; ++v) Ud[v] = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) Fvb[c] = 0.0;
  om = 0.0;
  if (wall) {
    // F*_c = (0, p_o e_d, 0); F*_v = f_v,o - (0, 0, 0, 0, u . tau_d)
    Pb[4] += psi[1 + d];
#pragma unroll
    for (int c = 0; c < 4; ++c) Fvb[c] -= psi[1 + c];
    om += psi[4];
  } else {
    double Pn[6];
    to_prim(sn, ph, Pn);
    const double sc_n = -sc_o;
#pragma unroll
    for (int v = 0; v < 5; ++v) phi[v] = psi[v] - sc_n * s_n * ln[v];
    if constexpr (EC) {
      // F*_c = f#_EC(U_L, U_R) - (1/2) Roe(U_L, U_R), the own element is L when up
      const double Ae[6] = {Po[0], Po[1], Po[2], Po[3], Po[4], 0.5 * Po[0] / Po[4]};
      const double Be[6] = {Pn[0], Pn[1], Pn[2], Pn[3], Pn[4], 0.5 * Pn[0] / Pn[4]};
      double Pbe[6] = {0, 0, 0, 0, 0, 0};
      ec_vjp<d>(Ae, Be, phi, ph.gm1, Pbe);
      fold_beta(Ae, Pbe, Pb);
      if (!ph.central) roe_vjp<d>(so, sn, up, phi, ph, Pb);
    } else {
      kg_vjp<d>(Po, Pn, phi, Pb);
      if (!ph.central) {
        const double co = fabs(Po[1 + d]) + sqrt(ph.gamma * Po[4] / Po[0]);
        const double cn = fabs(Pn[1 + d]) + sqrt(ph.gamma * Pn[4] / Pn[0]);
        // the own element is the lower side L of the face when the face is its upper one
        const bool own_L = up;
        const double lam = own_L ? (co >= cn ? co : cn) : (cn >= co ? cn : co);
        const bool own_active = own_L ? (co >= cn) : (co > cn);
        // F*_c contains -lam/2 (U_R - U_L)
        const double dU = own_L ? 0.5 * lam : -0.5 * lam;
        double lb = 0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          Ud[v] += dU * phi[v];
          const double jump = own_L ? sn[v] - so[v] : so[v] - sn[v];
          lb -= 0.5 * phi[v] * jump;
        }
        if (own_active) speed_vjp<d>(Po, lb, ph, Pb);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) Fvb[c] -= 0.5 * phi[1 + c];
  }
  // the own physical flux -(f_c - f_v)(o) of the own equation
  double mpsi[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) mpsi[v] = -psi[v];
  euler_vjp<d>(Po, mpsi, Pb);
#pragma unroll
  for (int c = 0; c < 4; ++c) Fvb[c] += psi[1 + c];
  prim_vjp(so, Pb, 0.0, ph, Ud);
}

// Scale s_d of the neighbour across face (d, up) of element (ex, ey, ez).
__device__ inline double nb_scale(const DevMesh& m, int ex, int ey, int ez, int d, bool up) {
  const int c = d == 0 ? ex : (d == 1 ? ey : ez);
  int v = c + (up ? 1 : -1);
  if (v < 0) v = m.n[d] - 1;
  if (v >= m.n[d]) v = 0;
  return m.s[d][v];
}

// --------------------------------------------------------------------------
// k_vjp_a
// --------------------------------------------------------------------------
// The line loops of the volume cotangents stay rolled and the kernel is
// bounded for four waves per SIMD: unrolled, each iteration's LDS operands
// are hoisted and the kernel needs all 256 registers (two waves per SIMD,
// 15 % slower at degree 5).
template <int N, bool EC>
__global__ __launch_bounds__(Cfg<N>::BS) __attribute__((amdgpu_waves_per_eu(4))) void k_vjp_a(const double* __restrict__ U,
                                                       const double* __restrict__ lam,
                                                       double* __restrict__ gbar,
                                                       double* __restrict__ ubar, DevMesh mesh,
                                                       DevPhys ph, DevBasis basis) {
  using Gm = Geo<N>;
  constexpr int NP = Gm::NP, NF = Gm::NF, NN = Gm::NN, EB = Gm::EB, DS = Gm::DS;
  constexpr int EPB = Cfg<N>::EPB, BS = Cfg<N>::BS;
  __shared__ double sD[NP * DS];
  __shared__ double sP[EPB][6][EB];
  __shared__ double sL[EPB][5][EB];
  __shared__ double sFU[EPB][6][5][NF];
  __shared__ double sFV[EPB][6][5][NF];
  __shared__ double sT[EPB][EB];          // T, for the forward lifting
  __shared__ double ssq[EPB][6][4][NF];   // BR1 lifting corrections of the faces

  const int tid = threadIdx.x;
  const long long nE = mesh.nE;
  const long long stride = nE * NN;
  const long long e0 = static_cast<long long>(xcd_remap(blockIdx.x, gridDim.x)) * EPB;
  for (int t = tid; t < NP * NP; t += BS) sD[(t / NP) * DS + t % NP] = basis.D[t];
  int ex0 = 0, ey0 = 0, ez0 = 0;
  elem_coords(e0 < nE ? e0 : 0, mesh, ex0, ey0, ez0);

  const int le = EPB == 1 ? 0 : tid / NN;
  const int node = tid - le * NN;
  const long long e = EPB == 1 ? e0 : e0 + le;
  const bool active = (EPB == 1 ? tid < NN : le < EPB) && e < nE;
  const int i = node % NP, j = (node / NP) % NP, k = node / NF;
  const int l = Gm::lds(i, j, k);

  // P1: node lanes stage primitives and lam; face lanes form the face cotangents
  double own[6] = {0, 0, 0, 0, 0, 0}, lo[5] = {0, 0, 0, 0, 0};
  int ex = ex0, ey = ey0, ez = ez0;
  if (active) {
    if (EPB > 1) elem_coords(e, mesh, ex, ey, ez);
    double s[5];
    load_state(U, stride, e * NN + node, s);
    to_prim(s, ph, own);
    if (EC) own[5] = 0.5 * own[0] / own[4];  // beta in place of e
    load_state(lam, stride, e * NN + node, lo);
#pragma unroll
    for (int q = 0; q < 6; ++q) sP[le][q][l] = own[q];
#pragma unroll
    for (int v = 0; v < 5; ++v) sL[le][v][l] = lo[v];
    sT[le][l] = own[4] * ph.inv_R / own[0];
  }
  if (tid < n_face_tasks<N>()) {
    const FaceTask<N> ft(tid);
    const long long te = EPB == 1 ? e0 : e0 + ft.le;
    if (te < nE) {
      int fx = ex0, fy = ey0, fz = ez0;
      if (EPB > 1) elem_coords(te, mesh, fx, fy, fz);
      const long long nb = neighbour(mesh, fx, fy, fz, ft.d, ft.up);
      const bool wall = nb < 0;
      const long long oidx = te * NN + ft.own_node();
      double so[5], fl[5], sn[5] = {1, 0, 0, 0, 1}, ln[5] = {0, 0, 0, 0, 0};
      load_state(U, stride, oidx, so);
      load_state(lam, stride, oidx, fl);
      double s_n = 0.0;
      if (!wall) {
        const long long nidx = nb * NN + ft.nb_node();
        load_state(U, stride, nidx, sn);
        load_state(lam, stride, nidx, ln);
        s_n = nb_scale(mesh, fx, fy, fz, ft.d, ft.up);
      }
      const double s_o = mesh.s[ft.d][ft.d == 0 ? fx : (ft.d == 1 ? fy : fz)];
      if (ph.viscous) {
        // forward lifting correction (q* - q_own) (+-1/w_end) of this face node
        const Prim Po = primitives(so, ph);
        const double qo[4] = {Po.u, Po.v, Po.w, Po.T};
        double qs[4];
        wall_lifting_value(mesh, ft.d, qo, qs);
        if (!wall) {
          const Prim Pn = primitives(sn, ph);
          qs[0] = 0.5 * (qo[0] + Pn.u);
          qs[1] = 0.5 * (qo[1] + Pn.v);
          qs[2] = 0.5 * (qo[2] + Pn.w);
          qs[3] = 0.5 * (qo[3] + Pn.T);
        }
        const double sc = ft.up ? basis.inv_w_end : -basis.inv_w_end;
#pragma unroll
        for (int c = 0; c < 4; ++c) ssq[ft.le][ft.f][c][ft.ab] = (qs[c] - qo[c]) * sc;
      }
      double Ud[5], Fvb[4], om;
      if (ft.d == 0)
        face_vjp<0, EC>(so, fl, sn, ln, wall, ft.up, s_o, s_n, ph, basis.inv_w_end, Ud, Fvb, om);
      else if (ft.d == 1)
        face_vjp<1, EC>(so, fl, sn, ln, wall, ft.up, s_o, s_n, ph, basis.inv_w_end, Ud, Fvb, om);
      else
        face_vjp<2, EC>(so, fl, sn, ln, wall, ft.up, s_o, s_n, ph, basis.inv_w_end, Ud, Fvb, om);
#pragma unroll
      for (int v = 0; v < 5; ++v) sFU[ft.le][ft.f][v][ft.ab] = Ud[v];
#pragma unroll
      for (int c = 0; c < 4; ++c) sFV[ft.le][ft.f][c][ft.ab] = Fvb[c];
      sFV[ft.le][ft.f][4][ft.ab] = om;
    }
  }
  __syncthreads();
  if (!active) return;

  // P2: node lanes
  const bool visc = ph.viscous != 0;
  // viscosity and conductivity at this node's temperature (Sutherland's law,
  // or constant: r = 1)
  const double Tn = sT[le][l];
  const double rT = viscosity_ratio(ph, Tn);
  const double mu = ph.mu * rT, kappa = ph.kappa * rT;
  // forward BR1 gradients g[3 q + d] of q = (u, v, w, T) at this node
  double g[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) g[c] = 0.0;
  if (visc) {
    const double sx = mesh.s[0][ex], sy = mesh.s[1][ey], sz = mesh.s[2][ez];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double* q = c < 3 ? sP[le][1 + c] : sT[le];
      double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        ax += sD[i * DS + m] * q[Gm::lds(m, j, k)];
        ay += sD[j * DS + m] * q[Gm::lds(i, m, k)];
        az += sD[k * DS + m] * q[Gm::lds(i, j, m)];
      }
      if (i == 0) ax += ssq[le][0][c][j + NP * k];
      if (i == N) ax += ssq[le][1][c][j + NP * k];
      if (j == 0) ay += ssq[le][2][c][i + NP * k];
      if (j == N) ay += ssq[le][3][c][i + NP * k];
      if (k == 0) az += ssq[le][4][c][i + NP * j];
      if (k == N) az += ssq[le][5][c][i + NP * j];
      g[3 * c + 0] = sx * ax;
      g[3 * c + 1] = sy * ay;
      g[3 * c + 2] = sz * az;
    }
  }
  // stress tau_ab (a, b in 0..2), symmetric
  const double dv = (2.0 / 3.0) * (g[0] + g[4] + g[8]);
  double tau[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) tau[3 * a + b] = mu * (g[3 * a + b] + g[3 * b + a] - (a == b ? dv : 0.0));

  double Pb[6] = {0, 0, 0, 0, 0, 0};
  double tb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double gT[3] = {0, 0, 0};
  double Ub[5] = {0, 0, 0, 0, 0};

#define DG_ADJ_DIRECTION(D)                                                                    \
  {                                                                                            \
    const int idx = D == 0 ? i : (D == 1 ? j : k);                                             \
    const int ab = D == 0 ? j + NP * k : (D == 1 ? i + NP * k : i + NP * j);                   \
    const double sd = mesh.s[D][D == 0 ? ex : (D == 1 ? ey : ez)];                              \
    double Fv[4] = {0, 0, 0, 0};                                                               \
    _Pragma("unroll 1") for (int m = 0; m < NP; ++m) {                                         \
      const int lm = D == 0 ? Gm::lds(m, j, k) : (D == 1 ? Gm::lds(i, m, k) : Gm::lds(i, j, m)); \
      const double Dim = sD[idx * DS + m], Dmi = sD[m * DS + idx];                              \
      double b[6], lmv[5], mu5[5];                                                             \
      _Pragma("unroll") for (int q = 0; q < 6; ++q) b[q] = sP[le][q][lm];                      \
      _Pragma("unroll") for (int v = 0; v < 5; ++v) lmv[v] = sL[le][v][lm];                    \
      _Pragma("unroll") for (int v = 0; v < 5; ++v) mu5[v] = -2.0 * sd * (Dim * lo[v] + Dmi * lmv[v]); \
      if constexpr (EC)                                                                        \
        ec_vjp<D>(own, b, mu5, ph.gm1, Pb);                                                    \
      else                                                                                     \
        kg_vjp<D>(own, b, mu5, Pb);                                                            \
      _Pragma("unroll") for (int c = 0; c < 4; ++c) Fv[c] += sd * Dmi * lmv[1 + c];             \
    }                                                                                          \
    double omd = 0.0;                                                                          \
    if (idx == 0) {                                                                            \
      _Pragma("unroll") for (int c = 0; c < 4; ++c) Fv[c] += sFV[le][2 * D][c][ab];            \
      omd += sFV[le][2 * D][4][ab];                                                            \
      _Pragma("unroll") for (int v = 0; v < 5; ++v) Ub[v] += sFU[le][2 * D][v][ab];            \
    }                                                                                          \
    if (idx == N) {                                                                            \
      _Pragma("unroll") for (int c = 0; c < 4; ++c) Fv[c] += sFV[le][2 * D + 1][c][ab];        \
      omd += sFV[le][2 * D + 1][4][ab];                                                        \
      _Pragma("unroll") for (int v = 0; v < 5; ++v) Ub[v] += sFU[le][2 * D + 1][v][ab];        \
    }                                                                                          \
    if (visc) {                                                                                \
      const double eb = Fv[3] + omd;                                                           \
      _Pragma("unroll") for (int a = 0; a < 3; ++a) {                                          \
        tb[3 * a + D] += Fv[a] + eb * own[1 + a];                                              \
        Pb[1 + a] += eb * tau[3 * a + D];                                                      \
      }                                                                                        \
      gT[D] += kappa * Fv[3];                                                                  \
    }                                                                                          \
  }
  DG_ADJ_DIRECTION(0)
  DG_ADJ_DIRECTION(1)
  DG_ADJ_DIRECTION(2)
#undef DG_ADJ_DIRECTION

  const long long idx = e * NN + node;
  if (visc) {
    const double tr = tb[0] + tb[4] + tb[8];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int y = 0; y < 3; ++y)
        store_once(&gbar[(3 * x + y) * stride + idx],
                   mu * (tb[3 * x + y] + tb[3 * y + x]) - (x == y ? (2.0 / 3.0) * mu * tr : 0.0));
#pragma unroll
    for (int d = 0; d < 3; ++d) store_once(&gbar[(9 + d) * stride + idx], gT[d]);
  }
  // Sutherland's law: tau and q scale with r(T), so T gets
  // (d ln r / dT) (tbar : tau + sum_d Fv_d,E q_d), d ln r / dT = 3 / (2 T) - 1 / (T + S)
  double Tb = 0.0;
  if (visc && ph.suth) {
    double st = 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) st += tb[c] * tau[c];
#pragma unroll
    for (int d = 0; d < 3; ++d) st += gT[d] * g[9 + d];
    Tb = (1.5 / Tn - 1.0 / (Tn + ph.suth_S)) * st;
  }
  if (EC) {
    // slot 5 holds the cotangent of beta = rho / (2 p)
    const double Pbe[6] = {0, 0, 0, 0, 0, Pb[5]};
    Pb[5] = 0.0;
    fold_beta(own, Pbe, Pb);
  }
  double s[5];
  load_state(U, stride, idx, s);
  prim_vjp(s, Pb, Tb, ph, Ub);
#pragma unroll
  for (int v = 0; v < 5; ++v) store_once(&ubar[v * stride + idx], Ub[v]);
}

// --------------------------------------------------------------------------
// k_vjp_b: transposed lifting
// --------------------------------------------------------------------------
template <int N, bool ACC>
__global__ __launch_bounds__(Cfg<N>::BS) void k_vjp_b(const double* __restrict__ U,
                                                       const double* __restrict__ gbar,
                                                       const double* __restrict__ ubar,
                                                       double* __restrict__ out, double scale,
                                                       double* __restrict__ cot, double cot_a,
                                                       double cot_b, DevMesh mesh, DevPhys ph,
                                                       DevBasis basis) {
  using Gm = Geo<N>;
  constexpr int NP = Gm::NP, NF = Gm::NF, NN = Gm::NN, EB = Gm::EB, DS = Gm::DS;
  constexpr int EPB = Cfg<N>::EPB, BS = Cfg<N>::BS;
  __shared__ double sD[NP * DS];
  __shared__ double sG[EPB][12][EB];
  __shared__ double sQ[EPB][6][4][NF];

  const int tid = threadIdx.x;
  const long long nE = mesh.nE;
  const long long stride = nE * NN;
  const long long e0 = static_cast<long long>(xcd_remap(blockIdx.x, gridDim.x)) * EPB;
  for (int t = tid; t < NP * NP; t += BS) sD[(t / NP) * DS + t % NP] = basis.D[t];
  int ex0 = 0, ey0 = 0, ez0 = 0;
  elem_coords(e0 < nE ? e0 : 0, mesh, ex0, ey0, ez0);

  const int le = EPB == 1 ? 0 : tid / NN;
  const int node = tid - le * NN;
  const long long e = EPB == 1 ? e0 : e0 + le;
  const bool active = (EPB == 1 ? tid < NN : le < EPB) && e < nE;
  const int i = node % NP, j = (node / NP) % NP, k = node / NF;
  const int l = Gm::lds(i, j, k);
  const bool visc = ph.viscous != 0;

  if (active && visc) {
#pragma unroll
    for (int c = 0; c < 12; ++c) sG[le][c][l] = gbar[c * stride + e * NN + node];
  }
  __syncthreads();
  if (visc && tid < n_face_tasks<N>()) {
    const FaceTask<N> ft(tid);
    const long long te = EPB == 1 ? e0 : e0 + ft.le;
    if (te < nE) {
      int fx = ex0, fy = ey0, fz = ez0;
      if (EPB > 1) elem_coords(te, mesh, fx, fy, fz);
      const long long nb = neighbour(mesh, fx, fy, fz, ft.d, ft.up);
      const double s_o = mesh.s[ft.d][ft.d == 0 ? fx : (ft.d == 1 ? fy : fz)];
      const double sgn = (ft.up ? -1.0 : 1.0) * basis.inv_w_end;
      const int lo = Gm::lds(ft.oi, ft.oj, ft.ok);
      if (nb < 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sQ[ft.le][ft.f][c][ft.ab] = sgn * s_o * sG[ft.le][3 * c + ft.d][lo];
      } else {
        const double s_n = nb_scale(mesh, fx, fy, fz, ft.d, ft.up);
        const long long nidx = nb * NN + ft.nb_node();
#pragma unroll
        for (int c = 0; c < 4; ++c)
          sQ[ft.le][ft.f][c][ft.ab] =
              0.5 * sgn * (s_o * sG[ft.le][3 * c + ft.d][lo] + s_n * gbar[(3 * c + ft.d) * stride + nidx]);
      }
    }
  }
  __syncthreads();
  if (!active) return;

  int ex = ex0, ey = ey0, ez = ez0;
  if (EPB > 1) elem_coords(e, mesh, ex, ey, ez);
  const long long idx = e * NN + node;
  double Ub[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) Ub[v] = load_once(&ubar[v * stride + idx]);
  if (visc) {
    const double sx = mesh.s[0][ex], sy = mesh.s[1][ey], sz = mesh.s[2][ez];
    double qb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        ax += sD[m * DS + i] * sG[le][3 * c + 0][Gm::lds(m, j, k)];
        ay += sD[m * DS + j] * sG[le][3 * c + 1][Gm::lds(i, m, k)];
        az += sD[m * DS + k] * sG[le][3 * c + 2][Gm::lds(i, j, m)];
      }
      qb[c] = sx * ax + sy * ay + sz * az;
      if (i == 0) qb[c] += sQ[le][0][c][j + NP * k];
      if (i == N) qb[c] += sQ[le][1][c][j + NP * k];
      if (j == 0) qb[c] += sQ[le][2][c][i + NP * k];
      if (j == N) qb[c] += sQ[le][3][c][i + NP * k];
      if (k == 0) qb[c] += sQ[le][4][c][i + NP * j];
      if (k == N) qb[c] += sQ[le][5][c][i + NP * j];
    }
    double s[5];
    load_state(U, stride, idx, s);
    const double Pb[6] = {0.0, qb[0], qb[1], qb[2], 0.0, 0.0};
    prim_vjp(s, Pb, qb[3], ph, Ub);
  }
  if (ACC) {
    // out += scale Ubar; with cot, also the next RK stage cotangent
    // cot <- cot_a cot + cot_b out at this node (no workgroup reads cot here)
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double nv = load_once(&out[v * stride + idx]) + scale * Ub[v];
      store_once(&out[v * stride + idx], nv);
      if (cot) store_once(&cot[v * stride + idx], cot_a * load_once(&cot[v * stride + idx]) + cot_b * nv);
    }
  } else {
#pragma unroll
    for (int v = 0; v < 5; ++v) store_once(&out[v * stride + idx], Ub[v]);
  }
}

// y = a y + b x; with a = 0 the old y is not read (a cleared or never written
// buffer may hold anything), with x null y = a y.
__global__ void k_axpby(double* __restrict__ y, const double* __restrict__ x, double a, double b,
                        long long n) {
  for (long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += static_cast<long long>(gridDim.x) * blockDim.x) {
    const double ay = a == 0.0 ? 0.0 : a * load_once(&y[t]);
    store_once(&y[t], x ? ay + b * load_once(&x[t]) : ay);
  }
}

template <int N>
hipError_t vjp_n(const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                 const double* lam, double* gbar, double* ubar, double* out,
                 bool acc, double scale, double* cot, double cot_a, double cot_b, hipStream_t s) {
  if (p.ec)
    hipLaunchKernelGGL((k_vjp_a<N, true>), dim3(n_blocks<N>(m.nE)), dim3(Cfg<N>::BS), 0, s, U,
                       lam, gbar, ubar, m, p, b);
  else
    hipLaunchKernelGGL((k_vjp_a<N, false>), dim3(n_blocks<N>(m.nE)), dim3(Cfg<N>::BS), 0, s, U,
                       lam, gbar, ubar, m, p, b);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if (acc)
    hipLaunchKernelGGL((k_vjp_b<N, true>), dim3(n_blocks<N>(m.nE)), dim3(Cfg<N>::BS), 0, s, U,
                       gbar, ubar, out, scale, cot, cot_a, cot_b, m, p, b);
  else
    hipLaunchKernelGGL((k_vjp_b<N, false>), dim3(n_blocks<N>(m.nE)), dim3(Cfg<N>::BS), 0, s, U,
                       gbar, ubar, out, scale, static_cast<double*>(nullptr), 0.0, 0.0, m, p, b);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rhs_vjp(int N, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                          const double* U, const double* lam, double* gbar, double* ubar,
                          double* out, bool accumulate, double scale, hipStream_t s, double* cot,
                          double cot_a, double cot_b) {
  if (m.nE <= 0) return hipSuccess;
  if (cot && !accumulate) return hipErrorInvalidValue;
  switch (N) {
    case 3: return vjp_n<3>(m, p, b, U, lam, gbar, ubar, out, accumulate, scale, cot, cot_a, cot_b, s);
    case 5: return vjp_n<5>(m, p, b, U, lam, gbar, ubar, out, accumulate, scale, cot, cot_a, cot_b, s);
    case 7: return vjp_n<7>(m, p, b, U, lam, gbar, ubar, out, accumulate, scale, cot, cot_a, cot_b, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_axpby(double* y, const double* x, double a, double b, long long n, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_axpby, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, y, x, a, b, n);
  return hipGetLastError();
}

}  // namespace dg
