// Internal declarations shared by the host API and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

#include "../../include/dgsem.h"

struct dg_ctx;

namespace dg {

constexpr int kMaxN = 7;
constexpr int kMaxNP = kMaxN + 1;

// Mesh data a kernel needs.  Every element is an axis-aligned box; its
// metric scale along direction d is s_d = 2 / width_d (one table per direction).
struct DevMesh {
  int n[3];           // elements per direction (x, y, z)
  int bc[3];          // DG_BC_PERIODIC or DG_BC_ISOTHERMAL_WALL
  double T_wall;
  const double* s[3]; // device tables of s_d per element index along d
  long long nE;       // number of elements
  const double* tauw; // wall-model stress per wall-face node (DG_BC_WALL_MODEL), or null
  const double* geo;  // curvilinear metrics geo[c][e][node] (c = 3 i + n: J a^i_n; 9: 1/J), or null
  const double* geoF; // the same ten fields at the element's boundary nodes only,
                      // geoF[c][e][t] (t: face node number), or null
};

// Gas constants and switches (FP64; kernels cast where they compute in FP32).
struct DevPhys {
  double gamma, gm1, R, inv_R, mu, kappa, cv;
  int viscous, central;
  int mixed_ref;      // mixed precision: subtract the element reference state
  int ec;             // Chandrashekar volume flux and Roe surface flux
  int suth;           // Sutherland's law: mu(T) = mu suth_c T^(3/2) / (T + suth_S)
  double suth_S, suth_c;
};

// LGL tables of one N, held in device memory inside the workspace.
struct DevBasis {
  const double* D;    // D[i * NP + m] = l_m'(xi_i)
  double inv_w_end;   // 1 / w_0 (= 1 / w_N)
};

// RK stage coefficients of one launch.
struct Stage {
  double A, B, dt;
  int read_G;         // 0 on the first stage (A_1 = 0): G is not read
};

// Kernel launchers.  ffv (face viscous fluxes, face_flux_values_per_element
// values per element) is double* for DG_FP64 and float* for DG_MIXED.
inline size_t face_flux_values_per_element(int N) { return static_cast<size_t>(6 * 4 * (N + 1) * (N + 1)); }
// nodes on an element's boundary: the two k planes and the ring of each interior one
inline size_t face_nodes_per_element(int N) { return static_cast<size_t>(2 * (N + 1) * (N + 1) + (N - 1) * 4 * N); }
hipError_t launch_face_flux(int N, int precision, const DevMesh& m, const DevPhys& p,
                            const DevBasis& b, const double* U, void* ffv, hipStream_t s);
hipError_t launch_rhs(int N, int precision, const DevMesh& m, const DevPhys& p,
                      const DevBasis& b, const double* U, const void* ffv, double* Ut,
                      int* status, hipStream_t s);
hipError_t launch_rk_stage(int N, int precision, const DevMesh& m, const DevPhys& p,
                           const DevBasis& b, const double* U, const void* ffv, double* G,
                           double* U_out, const Stage& st, int* status, hipStream_t s);
// Stand-alone FP64 lifting, grad[3 q + d][e][node] (lift_kernels.hip).
hipError_t launch_lift(int N, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                       const double* U, double* grad, hipStream_t s);

// Adjoint (adj_kernels.hip): Ubar = (dL/dU)^T lam at U, given the forward
// gradients grad of U; gbar and ubar are scratch (12 and 5 values per DOF).
// accumulate: out += scale * Ubar, else out = Ubar.
// With accumulate, cot (optional) receives the next RK stage cotangent
// cot_a cot + cot_b out after out is updated (node by node, fused in the
// second kernel).
hipError_t launch_rhs_vjp(int N, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                          const double* U, const double* lam, double* gbar, double* ubar,
                          double* out, bool accumulate, double scale, hipStream_t s,
                          double* cot = nullptr, double cot_a = 0.0, double cot_b = 0.0);
// y = a y + b x over n doubles; a = 0 does not read y and x = null drops the
// b x term, so (y, null, 0, 0) clears y (a kernel, not a memset node, for
// callers that capture the stream into a graph).
hipError_t launch_axpby(double* y, const double* x, double a, double b, long long n, hipStream_t s);

// Curvilinear hexahedra (curv_kernels.hip): metric terms from the node
// coordinates X[n][e][node] (status[0] = 1 where J <= 0; with_f32: also
// their FP32 copy after the ten FP64 fields, for mixed precision; geoF: the
// FP64 fields of the boundary nodes, contiguous per element), and the operator
// (face viscous fluxes double*, or float* unless precision is DG_FP64; one RK
// stage or the right-hand side alone).
hipError_t launch_metrics(int N, const double* X, double* geo, double* geoF, bool with_f32, const DevBasis& b,
                          long long nE, int* status, hipStream_t s);
hipError_t launch_face_flux_curv(int N, int precision, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                                 const double* U, void* ffv, hipStream_t s);
hipError_t launch_rhs_curv(int N, int precision, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                           const double* U, const void* ffv, double* Ut, int* status, hipStream_t s);
hipError_t launch_rk_stage_curv(int N, int precision, const DevMesh& m, const DevPhys& p, const DevBasis& b,
                                const double* U, const void* ffv, double* G, double* U_out,
                                const Stage& st, int* status, hipStream_t s);

// Gas constants and switches of a context as the kernels take them (api.cpp).
DevPhys device_physics(const dg_ctx* c);

// Wall-stress model: number of wall faces of the mesh, and the kernel (one
// lane per wall-face node).
long long wall_faces(const DevMesh& m);
hipError_t launch_wall_stress(int N, const DevMesh& m, const DevPhys& p, const double* U, int n_wm,
                              double xi_wm1, double recovery, double* tau, hipStream_t s);

// Reductions and elementwise kernels (aux_kernels.hip).
hipError_t launch_kinetic_energy(int N, const DevMesh& m, const double* w, const double* U,
                                 double* partial, int n_partial, double inv_vol, double* J,
                                 hipStream_t s);
hipError_t launch_kinetic_energy_grad(int N, const DevMesh& m, const double* w, const double* U,
                                      double inv_vol, double* lam, hipStream_t s);
hipError_t launch_triad(const double* b, const double* c, double s, double* a, long long n,
                        hipStream_t st);

// Host LGL construction (lgl.cpp): Newton on (1 - x^2) P_N'(x), barycentric D.
void lgl_nodes_weights(int N, std::vector<double>& xi, std::vector<double>& w);
void lgl_diff_matrix(const std::vector<double>& xi, std::vector<double>& D);

}  // namespace dg

struct dg_ctx {
  int N = 0;
  int nelem[3] = {0, 0, 0};
  std::vector<double> faces[3];
  int bc[3] = {0, 0, 0};
  double T_wall = 1.0;
  int wm_node = 1;            // interface node of the wall model
  bool wall_model = false;    // some direction has DG_BC_WALL_MODEL ends
  double* tauw = nullptr;     // wall stress of the current stage (workspace)
  bool curvilinear = false;   // node coordinates given: curved elements
  std::vector<double> nodes;  // their host copy [n][e][node]
  double* geo = nullptr;      // metric terms (workspace)
  double* geoF = nullptr;     // their boundary-node copy (workspace)
  long long n_wall_faces = 0;
  dg_physics phys{};
  hipStream_t stream = nullptr;
  long long nE = 0, nn = 0, n_dof = 0;

  std::vector<double> xi, w, D, s[3];

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  bool adjoint_bound = false;
  double* dD = nullptr;
  double* dw = nullptr;
  double* ds[3] = {nullptr, nullptr, nullptr};
  int* dstatus = nullptr;
  double* dpartial = nullptr;
  int n_partial = 0;
  double* U[2] = {nullptr, nullptr};
  int cur = 0;
  double* G = nullptr;
  void* ffv = nullptr;        // face viscous fluxes of the current stage
  // adjoint buffers
  double* stages = nullptr;   // 5 stage input states of one step
  double* lamG = nullptr;
  double* lamU = nullptr;
  double* ubar = nullptr;     // per-node partial cotangent of the state
  double* gbar = nullptr;     // cotangent of the lifted gradients
  double* tmp = nullptr;      // one state of scratch

  // measurement: one event after each timed launch (kernel class 0 = lift, 1 = rhs)
  std::vector<hipEvent_t> events;
  std::vector<int> event_class;
  hipEvent_t event_start = nullptr;
  bool timing = false;

  // RK steps captured into a HIP graph (dg_rk_graph_build): the instantiated
  // graph, its step count and the state buffer it reads and leaves the result in
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0;
  int graph_cur = 0;

  std::string err;
};
