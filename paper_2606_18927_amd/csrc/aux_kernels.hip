// Kinetic-energy functional and its gradient (the scalar flow functional
// whose initial-state gradient the adjoint computes), plus the STREAM triad
// used as the measured HBM ceiling.
//
// J(U) = sum_nodes w_i w_j w_k J_e |m|^2 / (2 rho) / |Omega|, with J_e = 1/(s_x s_y s_z)
// the affine Jacobian (s_d = 2 / width_d) and |Omega| = sum_e 8 J_e.
// The reduction is deterministic: a fixed grid of partial sums in a fixed
// order, then one workgroup adds the partials in index order.
#include "dg_internal.hpp"

namespace dg {
namespace {

constexpr int kBS = 256;

__device__ inline double node_weight(int N, long long g, long long nn, const DevMesh& m,
                                     const double* w, double& invJ) {
  const long long e = g / nn;
  const int node = static_cast<int>(g - e * nn);
  const int NP = N + 1;
  const int i = node % NP, j = (node / NP) % NP, k = node / (NP * NP);
  const int ex = static_cast<int>(e % m.n[0]);
  const long long t = e / m.n[0];
  const int ey = static_cast<int>(t % m.n[1]);
  const int ez = static_cast<int>(t / m.n[1]);
  invJ = m.s[0][ex] * m.s[1][ey] * m.s[2][ez];
  return w[i] * w[j] * w[k];
}

__global__ __launch_bounds__(kBS) void k_ke_partial(int N, DevMesh m, const double* __restrict__ w,
                                                    const double* __restrict__ U,
                                                    double* __restrict__ partial) {
  __shared__ double red[kBS];
  const long long nn = static_cast<long long>(N + 1) * (N + 1) * (N + 1);
  const long long n = m.nE * nn;
  double acc = 0.0;
  for (long long g = static_cast<long long>(blockIdx.x) * kBS + threadIdx.x; g < n;
       g += static_cast<long long>(gridDim.x) * kBS) {
    double invJ;
    const double wq = node_weight(N, g, nn, m, w, invJ);
    const double r = U[g], mx = U[n + g], my = U[2 * n + g], mz = U[3 * n + g];
    acc += wq / invJ * (0.5 * (mx * mx + my * my + mz * mz) / r);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBS) void k_ke_final(const double* __restrict__ partial, int np,
                                                  double inv_vol, double* __restrict__ J) {
  __shared__ double red[kBS];
  double acc = 0.0;
  for (int b = threadIdx.x; b < np; b += kBS) acc += partial[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBS / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) J[0] = red[0] * inv_vol;
}

__global__ __launch_bounds__(kBS) void k_ke_grad(int N, DevMesh m, const double* __restrict__ w,
                                                 const double* __restrict__ U, double inv_vol,
                                                 double* __restrict__ lam) {
  const long long nn = static_cast<long long>(N + 1) * (N + 1) * (N + 1);
  const long long n = m.nE * nn;
  for (long long g = static_cast<long long>(blockIdx.x) * kBS + threadIdx.x; g < n;
       g += static_cast<long long>(gridDim.x) * kBS) {
    double invJ;
    const double sc = node_weight(N, g, nn, m, w, invJ) / invJ * inv_vol;
    const double r = U[g];
    const double u = U[n + g] / r, v = U[2 * n + g] / r, ww = U[3 * n + g] / r;
    lam[g] = -0.5 * sc * (u * u + v * v + ww * ww);
    lam[n + g] = sc * u;
    lam[2 * n + g] = sc * v;
    lam[3 * n + g] = sc * ww;
    lam[4 * n + g] = 0.0;
  }
}

// a[i] = b[i] + s c[i]: reads 16 B and writes 8 B per element.  The fast
// form moves 16-byte pairs, one pair per lane and no grid-stride loop, with
// non-temporal loads and stores (7 % faster than cached ones: the ceiling the
// operator's HBM rate is compared with); the 8-byte form serves pointers
// that are not 16-byte aligned.
__global__ __launch_bounds__(kBS) void k_triad2(const double2* __restrict__ b,
                                                const double2* __restrict__ c, double s,
                                                double2* __restrict__ a, long long n2) {
  const long long g = static_cast<long long>(blockIdx.x) * kBS + threadIdx.x;
  if (g < n2) {
    const double* bp = reinterpret_cast<const double*>(b) + 2 * g;
    const double* cp = reinterpret_cast<const double*>(c) + 2 * g;
    const double2 x{__builtin_nontemporal_load(bp), __builtin_nontemporal_load(bp + 1)};
    const double2 y{__builtin_nontemporal_load(cp), __builtin_nontemporal_load(cp + 1)};
    double* ap = reinterpret_cast<double*>(a) + 2 * g;
    __builtin_nontemporal_store(x.x + s * y.x, ap);
    __builtin_nontemporal_store(x.y + s * y.y, ap + 1);
  }
}

__global__ __launch_bounds__(kBS) void k_triad(const double* __restrict__ b,
                                               const double* __restrict__ c, double s,
                                               double* __restrict__ a, long long n) {
  for (long long g = static_cast<long long>(blockIdx.x) * kBS + threadIdx.x; g < n;
       g += static_cast<long long>(gridDim.x) * kBS)
    a[g] = b[g] + s * c[g];
}

}  // namespace

hipError_t launch_triad(const double* b, const double* c, double s, double* a, long long n,
                        hipStream_t st) {
  const auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
  const long long n2 = n / 2;
  if (al16(a) && al16(b) && al16(c) && n2 > 0 && (n2 + kBS - 1) / kBS < (1LL << 31)) {
    const long long blocks = (n2 + kBS - 1) / kBS;
    hipLaunchKernelGGL(k_triad2, dim3(static_cast<unsigned>(blocks)), dim3(kBS), 0, st,
                       reinterpret_cast<const double2*>(b), reinterpret_cast<const double2*>(c), s,
                       reinterpret_cast<double2*>(a), n2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n % 2 == 0) return e;
    // the odd last element
    hipLaunchKernelGGL(k_triad, dim3(1), dim3(kBS), 0, st, b + 2 * n2, c + 2 * n2, s, a + 2 * n2, 1LL);
    return hipGetLastError();
  }
  long long blocks = (n + kBS - 1) / kBS;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_triad, dim3(static_cast<unsigned>(blocks)), dim3(kBS), 0, st, b, c, s, a, n);
  return hipGetLastError();
}

hipError_t launch_kinetic_energy(int N, const DevMesh& m, const double* w, const double* U,
                                 double* partial, int n_partial, double inv_vol, double* J,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_ke_partial, dim3(n_partial), dim3(kBS), 0, s, N, m, w, U, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_ke_final, dim3(1), dim3(kBS), 0, s, partial, n_partial, inv_vol, J);
  return hipGetLastError();
}

hipError_t launch_kinetic_energy_grad(int N, const DevMesh& m, const double* w, const double* U,
                                      double inv_vol, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_ke_grad, dim3(1024), dim3(kBS), 0, s, N, m, w, U, inv_vol, lam);
  return hipGetLastError();
}

}  // namespace dg
