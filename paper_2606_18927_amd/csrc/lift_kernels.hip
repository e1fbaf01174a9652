// BR1 lifting of the primitive gradients as a stand-alone kernel (FP64):
// grad(u, v, w, T) at every node, written as grad[3 q + d][e][node].  Used by
// dg_eval_lift and by the adjoint, whose reverse sweep needs the forward
// gradients of a stage.  The forward RK path computes the same gradients
// inside the fused right-hand-side kernel instead (fwd_kernels.hip).
//
// g_d[i] = s_d ( sum_m D_im q_m + delta_iN (q*_R - q_N)/w_N - delta_i0 (q*_L - q_0)/w_0 ),
// q* = (q_own + q_nb)/2 on shared faces; on walls (0, 0, 0, T_wall)
// (isothermal) or the own values without the normal velocity (wall model).
#include "dg_device.hpp"

namespace dg {
namespace {

template <int N>
__global__ __launch_bounds__(Cfg<N>::BS) void k_lift(const double* __restrict__ U,
                                                      double* __restrict__ grad, DevMesh mesh,
                                                      DevPhys ph, DevBasis basis) {
  using Gm = Geo<N>;
  constexpr int NP = Gm::NP, NF = Gm::NF, NN = Gm::NN, EB = Gm::EB;
  constexpr int EPB = Cfg<N>::EPB, BS = Cfg<N>::BS;
  __shared__ double sD[NP * Gm::DS];
  __shared__ double sq[EPB][4][EB];
  __shared__ double ssq[EPB][6][4][NF];

  const int tid = threadIdx.x;
  const long long nE = mesh.nE;
  const long long stride = nE * NN;
  const long long e0 = static_cast<long long>(xcd_remap(blockIdx.x, gridDim.x)) * EPB;
  for (int t = tid; t < NP * NP; t += BS) sD[(t / NP) * Gm::DS + t % NP] = basis.D[t];

  const int le = tid / NN;
  const int node = tid - le * NN;
  const long long e = e0 + le;
  const bool active = le < EPB && e < nE;
  const int i = node % NP, j = (node / NP) % NP, k = node / NF;

  if (tid < n_face_tasks<N>()) {
    const FaceTask<N> ft(tid);
    const long long te = e0 + ft.le;
    if (te < nE) {
      int ex, ey, ez;
      elem_coords(te, mesh, ex, ey, ez);
      const long long nb = neighbour(mesh, ex, ey, ez, ft.d, ft.up);
      double so[5];
      load_state(U, stride, te * NN + ft.own_node(), so);
      const Prim Po = primitives(so, ph);
      const double qo[4] = {Po.u, Po.v, Po.w, Po.T};
      double qs[4];
      wall_lifting_value(mesh, ft.d, qo, qs);
      if (nb >= 0) {
        double sn[5];
        load_state(U, stride, nb * NN + ft.nb_node(), sn);
        const Prim Pn = primitives(sn, ph);
        const double qn[4] = {Pn.u, Pn.v, Pn.w, Pn.T};
#pragma unroll
        for (int c = 0; c < 4; ++c) qs[c] = 0.5 * (qo[c] + qn[c]);
      }
      const double sc = ft.up ? basis.inv_w_end : -basis.inv_w_end;
#pragma unroll
      for (int c = 0; c < 4; ++c) ssq[ft.le][ft.f][c][ft.ab] = (qs[c] - qo[c]) * sc;
    }
  }
  if (active) {
    double s[5];
    load_state(U, stride, e * NN + node, s);
    const Prim P = primitives(s, ph);
    const int l = Gm::lds(i, j, k);
    sq[le][0][l] = P.u;
    sq[le][1][l] = P.v;
    sq[le][2][l] = P.w;
    sq[le][3][l] = P.T;
  }
  __syncthreads();

  if (active) {
    int ex, ey, ez;
    elem_coords(e, mesh, ex, ey, ez);
    const double sx = mesh.s[0][ex], sy = mesh.s[1][ey], sz = mesh.s[2][ez];
    double* ge = grad + e * NN + node;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        ax += sD[i * Gm::DS + m] * sq[le][c][Gm::lds(m, j, k)];
        ay += sD[j * Gm::DS + m] * sq[le][c][Gm::lds(i, m, k)];
        az += sD[k * Gm::DS + m] * sq[le][c][Gm::lds(i, j, m)];
      }
      if (i == 0) ax += ssq[le][0][c][j + NP * k];
      if (i == N) ax += ssq[le][1][c][j + NP * k];
      if (j == 0) ay += ssq[le][2][c][i + NP * k];
      if (j == N) ay += ssq[le][3][c][i + NP * k];
      if (k == 0) az += ssq[le][4][c][i + NP * j];
      if (k == N) az += ssq[le][5][c][i + NP * j];
      ge[(3 * c + 0) * stride] = sx * ax;
      ge[(3 * c + 1) * stride] = sy * ay;
      ge[(3 * c + 2) * stride] = sz * az;
    }
  }
}

template <int N>
hipError_t lift_n(const DevMesh& m, const DevPhys& p, const DevBasis& b, const double* U,
                  double* grad, hipStream_t s) {
  hipLaunchKernelGGL((k_lift<N>), dim3(n_blocks<N>(m.nE)), dim3(Cfg<N>::BS), 0, s, U, grad, m, p,
                     b);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lift(int N, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                       const double* U, double* grad, hipStream_t s) {
  if (m.nE <= 0) return hipSuccess;
  switch (N) {
    case 3: return lift_n<3>(m, p, b, U, grad, s);
    case 5: return lift_n<5>(m, p, b, U, grad, s);
    case 7: return lift_n<7>(m, p, b, U, grad, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dg
