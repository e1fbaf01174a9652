// C ABI of the DGSEM operator (declared in include/dgsem.h): argument
// validation, host tables, workspace partitioning and kernel dispatch.
// No call allocates device memory; every device operation is enqueued on the
// context's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dg_internal.hpp"

namespace dg {

// Wall faces of the mesh: 2 nb nc per direction with wall ends (host only).
long long wall_faces(const DevMesh& m) {
  long long n = 0;
  for (int d = 0; d < 3; ++d) {
    if (m.bc[d] == DG_BC_PERIODIC) continue;
    const int na = d == 0 ? m.n[1] : m.n[0];
    const int nb = d == 2 ? m.n[1] : m.n[2];
    n += 2LL * na * nb;
  }
  return n;
}

}  // namespace dg

namespace {

// Carpenter-Kennedy five-stage fourth-order 2N-storage coefficients
// (the fourth-order low-storage RK of paper Sec. 4).
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0,
                        -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0,
                        -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

constexpr int kPartials = 1024;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

dg_status fail(dg_ctx* c, dg_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

dg_status hip_check(dg_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return DG_OK;
  return fail(c, DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Layout {
  size_t D, w, s[3], status, partial, U0, U1, G, ffv, tauw, geo, geoF;
  size_t stages, lamG, lamU, ubar, gbar, tmp;
  size_t fwd_end, adj_end;
};

Layout layout(const dg_ctx* c) {
  Layout L{};
  const size_t NP = c->N + 1;
  const size_t dof = static_cast<size_t>(c->n_dof);
  const size_t state = 5 * dof * sizeof(double);
  const size_t rsize = c->phys.precision == DG_FP64 ? sizeof(double) : sizeof(float);
  const size_t fbytes = static_cast<size_t>(c->nE) * dg::face_flux_values_per_element(c->N) * rsize;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.D = take(NP * NP * sizeof(double));
  L.w = take(NP * sizeof(double));
  for (int d = 0; d < 3; ++d) L.s[d] = take(c->nelem[d] * sizeof(double));
  L.status = take(sizeof(int));
  L.partial = take(kPartials * sizeof(double));
  L.U0 = take(state);
  L.U1 = take(state);
  L.G = take(state);
  L.ffv = c->phys.viscous ? take(fbytes) : off;
  L.tauw = c->wall_model ? take(static_cast<size_t>(c->n_wall_faces) * 3 * NP * NP * sizeof(double)) : off;
  // FP64 metric terms, and their FP32 copy for the mixed-precision sweeps
  L.geo = c->curvilinear
              ? take(10 * dof * (sizeof(double) + (c->phys.precision == DG_FP64 ? 0 : sizeof(float))))
              : off;
  // the ten FP64 fields once more at the boundary nodes, contiguous per element
  // for the face-flux kernel and the surface terms
  L.geoF = c->curvilinear
               ? take(10 * static_cast<size_t>(c->nE) * dg::face_nodes_per_element(c->N) * sizeof(double))
               : off;
  L.fwd_end = off;
  L.stages = take(5 * state);
  L.lamG = take(state);
  L.lamU = take(state);
  L.ubar = take(state);
  L.gbar = take(12 * dof * sizeof(double));
  L.tmp = take(state);
  L.adj_end = off;
  return L;
}

dg::DevMesh dev_mesh(const dg_ctx* c) {
  dg::DevMesh m{};
  for (int d = 0; d < 3; ++d) {
    m.n[d] = c->nelem[d];
    m.bc[d] = c->bc[d];
    m.s[d] = c->ds[d];
  }
  m.T_wall = c->T_wall;
  m.nE = c->nE;
  m.tauw = c->wall_model ? c->tauw : nullptr;
  m.geo = c->curvilinear ? c->geo : nullptr;
  m.geoF = c->curvilinear ? c->geoF : nullptr;
  return m;
}

dg::DevPhys dev_phys(const dg_ctx* c) { return dg::device_physics(c); }

}  // namespace

dg::DevPhys dg::device_physics(const dg_ctx* c) {
  dg::DevPhys p{};
  p.gamma = c->phys.gamma;
  p.gm1 = c->phys.gamma - 1.0;
  p.R = c->phys.R;
  p.inv_R = 1.0 / c->phys.R;
  p.mu = c->phys.mu;
  p.kappa = c->phys.mu * c->phys.gamma * c->phys.R / ((c->phys.gamma - 1.0) * c->phys.Pr);
  p.cv = c->phys.R / (c->phys.gamma - 1.0);
  p.viscous = c->phys.viscous;
  p.central = c->phys.central_only;
  p.mixed_ref = c->phys.precision == DG_MIXED ? 1 : 0;
  p.ec = c->phys.flux == DG_FLUX_EC_ROE ? 1 : 0;
  p.suth = c->phys.viscosity == DG_VISC_SUTHERLAND ? 1 : 0;
  p.suth_S = p.suth ? c->phys.S : 0.0;
  p.suth_c = p.suth ? (c->phys.T_ref + c->phys.S) / (c->phys.T_ref * std::sqrt(c->phys.T_ref)) : 1.0;
  return p;
}

namespace {

dg::DevBasis dev_basis(const dg_ctx* c) {
  dg::DevBasis b{};
  b.D = c->dD;
  b.inv_w_end = 1.0 / c->w[0];
  return b;
}

double inv_volume(const dg_ctx* c) {
  double v = 1.0;
  for (int d = 0; d < 3; ++d) v *= c->faces[d].back() - c->faces[d].front();
  return 1.0 / v;
}

// Record the end of a timed launch of kernel class `cls`.
void mark(dg_ctx* c, int cls) {
  if (!c->timing) return;
  const size_t k = c->event_class.size();
  if (k >= c->events.size()) return;
  if (hipEventRecord(c->events[k], c->stream) == hipSuccess) c->event_class.push_back(cls);
}

// Release the captured RK graph (its kernel arguments point into the bound
// workspace, so a new binding drops it too), after its launches on the
// context's stream have finished.
void drop_graph(dg_ctx* c) {
  if (c->graph) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipGraphExecDestroy(c->graph);
  }
  c->graph = nullptr;
  c->graph_steps = 0;
}

dg_status need_bound(dg_ctx* c) {
  if (!c) return DG_EINVAL;
  if (!c->bound) return fail(c, DG_ESTATE, "no workspace bound (dg_bind_workspace)");
  return DG_OK;
}

// The wall model's stress of state U at DG_BC_WALL_MODEL walls, for the
// right-hand side of U (no-op without such walls or viscosity).
dg_status wall_model_stress(dg_ctx* c, const double* U) {
  if (!c->wall_model || !c->phys.viscous) return DG_OK;
  return hip_check(c, dg::launch_wall_stress(c->N, dev_mesh(c), dev_phys(c), U, c->wm_node,
                                             c->xi[c->wm_node] + 1.0, std::cbrt(c->phys.Pr), c->tauw,
                                             c->stream),
                   "wall stress kernel");
}

// Kernels of one stage for the context's element kind.
hipError_t face_flux_any(const dg_ctx* c, const dg::DevMesh& m, const dg::DevPhys& p, const dg::DevBasis& b,
                         const double* U) {
  if (c->curvilinear) return dg::launch_face_flux_curv(c->N, c->phys.precision, m, p, b, U, c->ffv, c->stream);
  return dg::launch_face_flux(c->N, c->phys.precision, m, p, b, U, c->ffv, c->stream);
}

hipError_t rhs_any(const dg_ctx* c, const dg::DevMesh& m, const dg::DevPhys& p, const dg::DevBasis& b,
                   const double* U, double* Ut) {
  if (c->curvilinear)
    return dg::launch_rhs_curv(c->N, c->phys.precision, m, p, b, U, c->ffv, Ut, c->dstatus, c->stream);
  return dg::launch_rhs(c->N, c->phys.precision, m, p, b, U, c->ffv, Ut, c->dstatus, c->stream);
}

hipError_t rk_stage_any(const dg_ctx* c, const dg::DevMesh& m, const dg::DevPhys& p, const dg::DevBasis& b,
                        const double* U, double* U_out, const dg::Stage& st) {
  if (c->curvilinear)
    return dg::launch_rk_stage_curv(c->N, c->phys.precision, m, p, b, U, c->ffv, c->G, U_out, st,
                                    c->dstatus, c->stream);
  return dg::launch_rk_stage(c->N, c->phys.precision, m, p, b, U, c->ffv, c->G, U_out, st, c->dstatus,
                             c->stream);
}

// Lifting (if viscous) then the right-hand side of U into Ut.
dg_status eval_rhs_into(dg_ctx* c, const double* U, double* Ut) {
  const dg::DevMesh m = dev_mesh(c);
  const dg::DevPhys p = dev_phys(c);
  const dg::DevBasis b = dev_basis(c);
  if (c->phys.viscous) {
    dg_status st = hip_check(c, face_flux_any(c, m, p, b, U), "face flux kernel");
    if (st != DG_OK) return st;
    mark(c, 0);
  }
  if (dg_status st = wall_model_stress(c, U); st != DG_OK) return st;
  dg_status st = hip_check(c, rhs_any(c, m, p, b, U, Ut), "rhs kernel");
  if (st == DG_OK) mark(c, 1);
  return st;
}

// The five stage inputs of one RK step from `in` (stage 0): stage s + 1 is
// written to stage_out(s) for s < 4 and the step's result to stage_out(4).
template <typename Out>
dg_status forward_stages(dg_ctx* c, const double* in, double dt, Out stage_out) {
  const dg::DevMesh m = dev_mesh(c);
  const dg::DevPhys p = dev_phys(c);
  const dg::DevBasis b = dev_basis(c);
  dg_status st = DG_OK;
  const double* cur = in;
  for (int s = 0; s < 5; ++s) {
    if (c->phys.viscous &&
        (st = hip_check(c, face_flux_any(c, m, p, b, cur), "face flux kernel")) != DG_OK)
      return st;
    if ((st = wall_model_stress(c, cur)) != DG_OK) return st;
    const dg::Stage stage{kRkA[s], kRkB[s], dt, s == 0 ? 0 : 1};
    double* out = stage_out(s);
    if ((st = hip_check(c, rk_stage_any(c, m, p, b, cur, out, stage), "rk stage kernel")) != DG_OK)
      return st;
    cur = out;
  }
  return DG_OK;
}

// Reverse sweep of one RK step over its five stage inputs stage_in(s):
// cot_s = A_{s+1} cot_{s+1} + B_s lamU;  lamU += dt (dL/dU(U_s))^T cot_s.
template <typename In>
dg_status reverse_stages(dg_ctx* c, In stage_in, double dt, const double* lam_np1, double* lam_n) {
  const dg::DevMesh m = dev_mesh(c);
  const dg::DevPhys p = dev_phys(c);
  const dg::DevBasis b = dev_basis(c);
  const size_t bytes = static_cast<size_t>(5 * c->n_dof) * sizeof(double);
  dg_status st = DG_OK;
  if ((st = hip_check(c, hipMemcpyAsync(c->lamU, lam_np1, bytes, hipMemcpyDeviceToDevice, c->stream),
                      "lam copy")) != DG_OK)
    return st;
  // cot_4 = B_4 lamU (A_5 = 0; a = 0 does not read the old lamG); each later
  // cot_{s-1} = A_s cot_s + B_{s-1} lamU is formed by the VJP kernel of stage s
  // right after it updates lamU
  if ((st = hip_check(c, dg::launch_axpby(c->lamG, c->lamU, 0.0, kRkB[4], 5 * c->n_dof, c->stream),
                      "axpby kernel")) != DG_OK)
    return st;
  for (int s = 4; s >= 0; --s) {
    if ((st = hip_check(c, dg::launch_rhs_vjp(c->N, m, p, b, stage_in(s), c->lamG, c->gbar,
                                              c->ubar, c->lamU, true, dt, c->stream,
                                              s > 0 ? c->lamG : nullptr, kRkA[s],
                                              s > 0 ? kRkB[s - 1] : 0.0),
                        "vjp kernels")) != DG_OK)
      return st;
  }
  return hip_check(c, hipMemcpyAsync(lam_n, c->lamU, bytes, hipMemcpyDeviceToDevice, c->stream),
                   "lam copy");
}

dg_status need_adjoint(dg_ctx* c) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (!c->adjoint_bound) return fail(c, DG_ESTATE, "workspace bound without the adjoint buffers");
  if (c->wall_model) return fail(c, DG_EUNSUPPORTED, "the adjoint does not cover the wall model");
  if (c->curvilinear) return fail(c, DG_EUNSUPPORTED, "the adjoint is built for axis-aligned elements");
  return DG_OK;
}

}  // namespace

extern "C" {

const char* dg_version(void) { return "dgsem-gfx950 0.1"; }

dg_status dg_lgl(int N, double* xi, double* w) {
  if (N < 1 || N > 16 || !xi || !w) return DG_EINVAL;
  std::vector<double> x, ww;
  dg::lgl_nodes_weights(N, x, ww);
  std::memcpy(xi, x.data(), (N + 1) * sizeof(double));
  std::memcpy(w, ww.data(), (N + 1) * sizeof(double));
  return DG_OK;
}

dg_status dg_init_mesh(const dg_mesh_desc* mesh, const dg_physics* phys, void* hip_stream,
                       dg_ctx** out) {
  if (!mesh || !phys || !out) return DG_EINVAL;
  *out = nullptr;
  if (mesh->N != 3 && mesh->N != 5 && mesh->N != 7) return DG_EUNSUPPORTED;
  const bool curved = mesh->nodes != nullptr;
  long long nE = 1;
  for (int d = 0; d < 3; ++d) {
    if (mesh->nelem[d] <= 0 || (!curved && !mesh->faces[d])) return DG_EINVAL;
    if (mesh->bc[d] != DG_BC_PERIODIC && mesh->bc[d] != DG_BC_ISOTHERMAL_WALL &&
        mesh->bc[d] != DG_BC_WALL_MODEL)
      return DG_EINVAL;
    if (mesh->faces[d]) {
      for (int i = 0; i < mesh->nelem[d]; ++i) {
        const double a = mesh->faces[d][i], b = mesh->faces[d][i + 1];
        if (!(b > a) || !std::isfinite(a) || !std::isfinite(b)) return DG_EINVAL;
      }
    }
    nE *= mesh->nelem[d];
  }
  const long long nn = static_cast<long long>(mesh->N + 1) * (mesh->N + 1) * (mesh->N + 1);
  if (nE > (1LL << 31) / 8 || nE * nn * 12 > (1LL << 40)) return DG_EINVAL;
  if (!(phys->gamma > 1.0) || !(phys->R > 0.0) || !(phys->mu >= 0.0) || !(phys->Pr > 0.0))
    return DG_EINVAL;
  if (phys->precision != DG_FP64 && phys->precision != DG_MIXED &&
      phys->precision != DG_MIXED_NOREF)
    return DG_EINVAL;
  if (phys->flux != DG_FLUX_KG_LLF && phys->flux != DG_FLUX_EC_ROE) return DG_EINVAL;
  if (phys->flux == DG_FLUX_EC_ROE && phys->precision == DG_MIXED_NOREF) return DG_EUNSUPPORTED;
  if (phys->viscosity != DG_VISC_CONSTANT && phys->viscosity != DG_VISC_SUTHERLAND) return DG_EINVAL;
  if (phys->viscosity == DG_VISC_SUTHERLAND) {
    if (!(phys->T_ref > 0.0) || !(phys->S >= 0.0) || !std::isfinite(phys->T_ref) || !std::isfinite(phys->S))
      return DG_EINVAL;
  }
  const bool wall_model = mesh->bc[0] == DG_BC_WALL_MODEL || mesh->bc[1] == DG_BC_WALL_MODEL ||
                          mesh->bc[2] == DG_BC_WALL_MODEL;
  if (wall_model && (mesh->wm_node < 1 || mesh->wm_node > mesh->N)) return DG_EINVAL;
  if (mesh->bc[0] == DG_BC_ISOTHERMAL_WALL || mesh->bc[1] == DG_BC_ISOTHERMAL_WALL ||
      mesh->bc[2] == DG_BC_ISOTHERMAL_WALL) {
    if (!(mesh->T_wall > 0.0)) return DG_EINVAL;
  }
  if (curved) {
    if (wall_model) return DG_EUNSUPPORTED;
    const long long n3 = 3 * nE * nn;
    for (long long q = 0; q < n3; ++q)
      if (!std::isfinite(mesh->nodes[q])) return DG_EINVAL;
  }

  dg_ctx* c = new (std::nothrow) dg_ctx();
  if (!c) return DG_EINVAL;
  c->N = mesh->N;
  for (int d = 0; d < 3; ++d) {
    c->nelem[d] = mesh->nelem[d];
    if (mesh->faces[d]) {
      c->faces[d].assign(mesh->faces[d], mesh->faces[d] + mesh->nelem[d] + 1);
    } else {  // curved mesh without faces: unit-width placeholders (the scales are unused)
      c->faces[d].resize(mesh->nelem[d] + 1);
      for (int i = 0; i <= mesh->nelem[d]; ++i) c->faces[d][i] = i;
    }
    c->bc[d] = mesh->bc[d];
    c->s[d].resize(mesh->nelem[d]);
    for (int i = 0; i < mesh->nelem[d]; ++i)
      c->s[d][i] = 2.0 / (c->faces[d][i + 1] - c->faces[d][i]);
  }
  c->T_wall = mesh->T_wall;
  c->wall_model = wall_model;
  c->wm_node = mesh->wm_node;
  c->curvilinear = curved;
  if (curved) c->nodes.assign(mesh->nodes, mesh->nodes + 3 * nE * nn);
  c->phys = *phys;
  c->phys.viscous = phys->viscous ? 1 : 0;
  c->phys.central_only = phys->central_only ? 1 : 0;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->nE = nE;
  c->nn = nn;
  c->n_dof = nE * nn;
  c->n_wall_faces = dg::wall_faces(dev_mesh(c));
  dg::lgl_nodes_weights(c->N, c->xi, c->w);
  dg::lgl_diff_matrix(c->xi, c->D);
  *out = c;
  return DG_OK;
}

dg_status dg_workspace_bytes(const dg_ctx* ctx, int with_adjoint, size_t* bytes) {
  if (!ctx || !bytes) return DG_EINVAL;
  const Layout L = layout(ctx);
  *bytes = with_adjoint ? L.adj_end : L.fwd_end;
  return DG_OK;
}

dg_status dg_n_dof(const dg_ctx* ctx, long long* n_dof) {
  if (!ctx || !n_dof) return DG_EINVAL;
  *n_dof = ctx->n_dof;
  return DG_OK;
}

dg_status dg_bind_workspace(dg_ctx* c, void* dev_ptr, size_t bytes, int with_adjoint) {
  if (!c || !dev_ptr) return DG_EINVAL;
  if (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign != 0)
    return fail(c, DG_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = layout(c);
  const size_t need = with_adjoint ? L.adj_end : L.fwd_end;
  if (bytes < need) return fail(c, DG_EINVAL, "workspace too small");
  drop_graph(c);
  char* ws = static_cast<char*>(dev_ptr);
  c->ws = ws;
  c->ws_bytes = bytes;
  c->dD = reinterpret_cast<double*>(ws + L.D);
  c->dw = reinterpret_cast<double*>(ws + L.w);
  for (int d = 0; d < 3; ++d) c->ds[d] = reinterpret_cast<double*>(ws + L.s[d]);
  c->dstatus = reinterpret_cast<int*>(ws + L.status);
  c->dpartial = reinterpret_cast<double*>(ws + L.partial);
  c->n_partial = kPartials;
  c->U[0] = reinterpret_cast<double*>(ws + L.U0);
  c->U[1] = reinterpret_cast<double*>(ws + L.U1);
  c->cur = 0;
  c->G = reinterpret_cast<double*>(ws + L.G);
  c->ffv = c->phys.viscous ? static_cast<void*>(ws + L.ffv) : nullptr;
  c->tauw = c->wall_model ? reinterpret_cast<double*>(ws + L.tauw) : nullptr;
  c->geo = c->curvilinear ? reinterpret_cast<double*>(ws + L.geo) : nullptr;
  c->geoF = c->curvilinear ? reinterpret_cast<double*>(ws + L.geoF) : nullptr;
  if (with_adjoint) {
    c->stages = reinterpret_cast<double*>(ws + L.stages);
    c->lamG = reinterpret_cast<double*>(ws + L.lamG);
    c->lamU = reinterpret_cast<double*>(ws + L.lamU);
    c->ubar = reinterpret_cast<double*>(ws + L.ubar);
    c->gbar = reinterpret_cast<double*>(ws + L.gbar);
    c->tmp = reinterpret_cast<double*>(ws + L.tmp);
  } else {
    c->stages = c->lamG = c->lamU = c->ubar = c->tmp = c->gbar = nullptr;
  }
  c->adjoint_bound = with_adjoint != 0;
  const size_t NP = c->N + 1;
  dg_status st;
  if ((st = hip_check(c, hipMemcpyAsync(c->dD, c->D.data(), NP * NP * sizeof(double),
                                        hipMemcpyHostToDevice, c->stream), "upload D")) != DG_OK)
    return st;
  if ((st = hip_check(c, hipMemcpyAsync(c->dw, c->w.data(), NP * sizeof(double),
                                        hipMemcpyHostToDevice, c->stream), "upload w")) != DG_OK)
    return st;
  for (int d = 0; d < 3; ++d)
    if ((st = hip_check(c, hipMemcpyAsync(c->ds[d], c->s[d].data(), c->nelem[d] * sizeof(double),
                                          hipMemcpyHostToDevice, c->stream), "upload s")) != DG_OK)
      return st;
  if ((st = hip_check(c, hipMemsetAsync(c->dstatus, 0, sizeof(int), c->stream), "clear status")) != DG_OK)
    return st;
  if ((st = hip_check(c, hipMemsetAsync(c->G, 0, 5 * c->n_dof * sizeof(double), c->stream),
                      "clear G")) != DG_OK)
    return st;
  if (c->curvilinear) {
    // metric terms from the node coordinates, staged through G (5 values per DOF)
    const size_t xbytes = 3 * static_cast<size_t>(c->n_dof) * sizeof(double);
    if ((st = hip_check(c, hipMemcpyAsync(c->G, c->nodes.data(), xbytes, hipMemcpyHostToDevice, c->stream),
                        "upload nodes")) != DG_OK)
      return st;
    if ((st = hip_check(c, dg::launch_metrics(c->N, c->G, c->geo, c->geoF, c->phys.precision != DG_FP64,
                                             dev_basis(c), c->nE, c->dstatus, c->stream),
                        "metrics kernel")) != DG_OK)
      return st;
    int bad = 0;
    if ((st = hip_check(c, hipMemcpyAsync(&bad, c->dstatus, sizeof(int), hipMemcpyDeviceToHost, c->stream),
                        "metrics status")) != DG_OK)
      return st;
    if ((st = hip_check(c, hipStreamSynchronize(c->stream), "metrics sync")) != DG_OK) return st;
    if (bad) return fail(c, DG_EINVAL, "non-positive Jacobian at some node of the curved mesh");
    if ((st = hip_check(c, hipMemsetAsync(c->G, 0, 5 * c->n_dof * sizeof(double), c->stream), "clear G")) != DG_OK)
      return st;
  }
  // the host tables above live in the context, so the asynchronous copies may
  // still be in flight after return; they complete before any later kernel.
  c->bound = true;
  return DG_OK;
}

dg_status dg_set_state(dg_ctx* c, const double* U) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (!U) return fail(c, DG_EINVAL, "null state");
  c->cur = 0;
  const size_t bytes = 5 * c->n_dof * sizeof(double);
  if ((st = hip_check(c, hipMemcpyAsync(c->U[0], U, bytes, hipMemcpyDeviceToDevice, c->stream),
                      "set_state copy")) != DG_OK)
    return st;
  // cleared by a kernel: a caller may capture this call into a graph
  return hip_check(c, dg::launch_axpby(c->G, nullptr, 0.0, 0.0, 5 * c->n_dof, c->stream), "clear G");
}

dg_status dg_get_state(const dg_ctx* cc, double* U) {
  dg_ctx* c = const_cast<dg_ctx*>(cc);
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (!U) return fail(c, DG_EINVAL, "null state");
  return hip_check(c, hipMemcpyAsync(U, c->U[c->cur], 5 * c->n_dof * sizeof(double),
                                     hipMemcpyDeviceToDevice, c->stream),
                   "get_state copy");
}

dg_status dg_eval_rhs(dg_ctx* c, const double* U, double* Ut, double /*t*/) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (!U || !Ut || U == Ut) return fail(c, DG_EINVAL, "bad U/Ut pointers");
  return eval_rhs_into(c, U, Ut);
}

dg_status dg_eval_lift(dg_ctx* c, const double* U, double* grad) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (!U || !grad) return fail(c, DG_EINVAL, "bad pointers");
  if (c->phys.precision != DG_FP64) return fail(c, DG_EUNSUPPORTED, "eval_lift: FP64 contexts only");
  if (c->curvilinear) return fail(c, DG_EUNSUPPORTED, "eval_lift: axis-aligned elements only");
  return hip_check(c, dg::launch_lift(c->N, dev_mesh(c), dev_phys(c), dev_basis(c), U, grad, c->stream),
                   "lift kernel");
}

dg_status dg_rk_step(dg_ctx* c, double /*t*/, double dt, int nsteps) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (nsteps < 0 || !std::isfinite(dt)) return fail(c, DG_EINVAL, "bad dt/nsteps");
  const dg::DevMesh m = dev_mesh(c);
  const dg::DevPhys p = dev_phys(c);
  const dg::DevBasis b = dev_basis(c);
  for (int n = 0; n < nsteps; ++n) {
    for (int s = 0; s < 5; ++s) {
      const double* Uin = c->U[c->cur];
      double* Uout = c->U[c->cur ^ 1];
      if (c->phys.viscous) {
        if ((st = hip_check(c, face_flux_any(c, m, p, b, Uin), "face flux kernel")) != DG_OK)
          return st;
        mark(c, 0);
      }
      if ((st = wall_model_stress(c, Uin)) != DG_OK) return st;
      const dg::Stage stage{kRkA[s], kRkB[s], dt, s == 0 ? 0 : 1};
      if ((st = hip_check(c, rk_stage_any(c, m, p, b, Uin, Uout, stage), "rk stage kernel")) != DG_OK)
        return st;
      mark(c, 1);
      c->cur ^= 1;
    }
  }
  return DG_OK;
}

dg_status dg_eval_rhs_vjp(dg_ctx* c, const double* U, const double* lam, double* Ubar, double /*t*/) {
  dg_status st = need_adjoint(c);
  if (st != DG_OK) return st;
  if (!U || !lam || !Ubar || Ubar == U || Ubar == lam) return fail(c, DG_EINVAL, "bad pointers");
  const dg::DevMesh m = dev_mesh(c);
  const dg::DevPhys p = dev_phys(c);
  const dg::DevBasis b = dev_basis(c);
  return hip_check(c, dg::launch_rhs_vjp(c->N, m, p, b, U, lam, c->gbar, c->ubar, Ubar, false, 1.0,
                                         c->stream),
                   "vjp kernels");
}

dg_status dg_rk_step_vjp(dg_ctx* c, const double* U_n, double /*t*/, double dt, const double* lam_np1,
                         double* lam_n) {
  dg_status st = need_adjoint(c);
  if (st != DG_OK) return st;
  if (!U_n || !lam_np1 || !lam_n || !std::isfinite(dt)) return fail(c, DG_EINVAL, "bad arguments");
  const long long n5 = 5 * c->n_dof;
  const size_t bytes = n5 * sizeof(double);
  auto stage_state = [&](int s) { return c->stages + static_cast<size_t>(s) * n5; };
  // forward recompute of the five stage inputs with the context's own forward
  if ((st = hip_check(c, hipMemcpyAsync(stage_state(0), U_n, bytes, hipMemcpyDeviceToDevice, c->stream),
                      "stage copy")) != DG_OK)
    return st;
  if ((st = forward_stages(c, stage_state(0), dt,
                           [&](int s) { return s < 4 ? stage_state(s + 1) : c->tmp; })) != DG_OK)
    return st;
  return reverse_stages(c, [&](int s) -> const double* { return stage_state(s); }, dt, lam_np1, lam_n);
}

dg_status dg_rk_record_stages(dg_ctx* c, const double* U0, double /*t*/, double dt, int nsteps,
                              double* stages) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (!U0 || !stages || nsteps < 1 || !std::isfinite(dt)) return fail(c, DG_EINVAL, "bad arguments");
  const size_t n5 = static_cast<size_t>(5 * c->n_dof);
  if (U0 >= stages && U0 < stages + static_cast<size_t>(nsteps) * 5 * n5)
    return fail(c, DG_EINVAL, "U0 inside the stage buffer");
  auto slot = [&](long long q) { return stages + static_cast<size_t>(q) * n5; };
  if ((st = hip_check(c, hipMemcpyAsync(slot(0), U0, n5 * sizeof(double), hipMemcpyDeviceToDevice,
                                        c->stream),
                      "stage copy")) != DG_OK)
    return st;
  for (int n = 0; n < nsteps; ++n) {
    // the last stage of step n writes stage 0 of step n + 1, or the context's
    // state after the last step
    double* next = n + 1 < nsteps ? slot(5LL * (n + 1)) : c->U[c->cur ^ 1];
    if ((st = forward_stages(c, slot(5LL * n), dt,
                             [&](int s) { return s < 4 ? slot(5LL * n + s + 1) : next; })) != DG_OK)
      return st;
  }
  c->cur ^= 1;
  return DG_OK;
}

dg_status dg_rk_step_vjp_stages(dg_ctx* c, const double* stages, double /*t*/, double dt,
                                const double* lam_np1, double* lam_n) {
  dg_status st = need_adjoint(c);
  if (st != DG_OK) return st;
  if (!stages || !lam_np1 || !lam_n || !std::isfinite(dt)) return fail(c, DG_EINVAL, "bad arguments");
  const size_t n5 = static_cast<size_t>(5 * c->n_dof);
  return reverse_stages(c, [&](int s) { return stages + static_cast<size_t>(s) * n5; }, dt, lam_np1, lam_n);
}

dg_status dg_wall_faces(const dg_ctx* c, long long* n) {
  if (!c || !n) return DG_EINVAL;
  *n = dg::wall_faces(dev_mesh(c));
  return DG_OK;
}

dg_status dg_wall_stress(dg_ctx* c, const double* U, int n_wm, double* tau) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (n_wm < 1 || n_wm > c->N) return fail(c, DG_EINVAL, "interface node index outside 1..N");
  if (dg::wall_faces(dev_mesh(c)) == 0) return DG_OK;  // no walls: nothing to write
  if (!U || !tau) return fail(c, DG_EINVAL, "bad pointers");
  const double recovery = std::cbrt(c->phys.Pr);
  return hip_check(c, dg::launch_wall_stress(c->N, dev_mesh(c), dev_phys(c), U, n_wm, c->xi[n_wm] + 1.0,
                                             recovery, tau, c->stream),
                   "wall stress kernel");
}

dg_status dg_kinetic_energy(dg_ctx* c, const double* U, double* J) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (!U || !J) return fail(c, DG_EINVAL, "bad pointers");
  if (c->curvilinear) return fail(c, DG_EUNSUPPORTED, "kinetic energy: axis-aligned elements only");
  return hip_check(c, dg::launch_kinetic_energy(c->N, dev_mesh(c), c->dw, U, c->dpartial, c->n_partial,
                                                inv_volume(c), J, c->stream),
                   "kinetic energy kernels");
}

dg_status dg_kinetic_energy_grad(dg_ctx* c, const double* U, double* lam) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (!U || !lam) return fail(c, DG_EINVAL, "bad pointers");
  if (c->curvilinear) return fail(c, DG_EUNSUPPORTED, "kinetic energy: axis-aligned elements only");
  return hip_check(c, dg::launch_kinetic_energy_grad(c->N, dev_mesh(c), c->dw, U, inv_volume(c), lam,
                                                     c->stream),
                   "kinetic energy gradient kernel");
}

dg_status dg_stream_triad(const double* b, const double* cc, double s, double* a, long long n,
                          void* hip_stream) {
  if (!b || !cc || !a || n < 0) return DG_EINVAL;
  return dg::launch_triad(b, cc, s, a, n, static_cast<hipStream_t>(hip_stream)) == hipSuccess
             ? DG_OK
             : DG_EHIP;
}

dg_status dg_timing_begin(dg_ctx* c, int max_launches) {
  if (!c || max_launches <= 0) return DG_EINVAL;
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  c->events.clear();
  c->event_class.clear();
  if (c->event_start) (void)hipEventDestroy(c->event_start);
  c->event_start = nullptr;
  dg_status st = hip_check(c, hipEventCreate(&c->event_start), "event create");
  if (st != DG_OK) return st;
  c->events.resize(max_launches, nullptr);
  for (auto& e : c->events)
    if ((st = hip_check(c, hipEventCreate(&e), "event create")) != DG_OK) return st;
  if ((st = hip_check(c, hipEventRecord(c->event_start, c->stream), "event record")) != DG_OK) return st;
  c->timing = true;
  return DG_OK;
}

dg_status dg_timing_end(dg_ctx* c, double ms[2], int count[2]) {
  if (!c || !ms || !count) return DG_EINVAL;
  if (!c->timing) return fail(c, DG_ESTATE, "dg_timing_end without dg_timing_begin");
  c->timing = false;
  dg_status st = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
  if (st != DG_OK) return st;
  ms[0] = ms[1] = 0.0;
  count[0] = count[1] = 0;
  hipEvent_t prev = c->event_start;
  for (size_t k = 0; k < c->event_class.size(); ++k) {
    float t = 0.0f;
    if ((st = hip_check(c, hipEventElapsedTime(&t, prev, c->events[k]), "event elapsed")) != DG_OK) return st;
    ms[c->event_class[k]] += t;
    count[c->event_class[k]] += 1;
    prev = c->events[k];
  }
  return DG_OK;
}

dg_status dg_sync(dg_ctx* c) {
  if (!c) return DG_EINVAL;
  dg_status st = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
  if (st != DG_OK || !c->bound) return st;
  int flag = 0;
  if ((st = hip_check(c, hipMemcpyAsync(&flag, c->dstatus, sizeof(int), hipMemcpyDeviceToHost, c->stream),
                      "read status")) != DG_OK)
    return st;
  if ((st = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize")) != DG_OK) return st;
  if (flag) {
    if ((st = hip_check(c, hipMemsetAsync(c->dstatus, 0, sizeof(int), c->stream), "clear status")) != DG_OK)
      return st;
    return fail(c, DG_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or NaN) seen by a kernel");
  }
  return DG_OK;
}

const char* dg_last_error(const dg_ctx* c) { return c ? c->err.c_str() : "null context"; }

dg_status dg_rk_graph_build(dg_ctx* c, double dt, int nsteps) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (nsteps < 2 || nsteps % 2 != 0 || !std::isfinite(dt))
    return fail(c, DG_EINVAL, "rk graph: nsteps must be even and >= 2, dt finite");
  if (c->timing) return fail(c, DG_ESTATE, "rk graph: not while dg_timing is active");
  drop_graph(c);
  // The stages are captured on a private stream (the context's may be the
  // null stream, which cannot be captured); launches later go to the
  // context's stream.  5 nsteps stages, an even number, leave the state in
  // the buffer the graph reads, so the graph can be replayed back to back.
  hipStream_t cap = nullptr;
  if ((st = hip_check(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "rk graph stream")) != DG_OK)
    return st;
  const hipStream_t saved = c->stream;
  const int cur0 = c->cur;
  hipGraph_t g = nullptr;
  st = hip_check(c, hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "rk graph capture");
  if (st == DG_OK) {
    c->stream = cap;
    const dg_status run = dg_rk_step(c, 0.0, dt, nsteps);
    c->stream = saved;
    const dg_status end = hip_check(c, hipStreamEndCapture(cap, &g), "rk graph capture end");
    st = run != DG_OK ? run : end;
  }
  c->cur = cur0;
  if (st == DG_OK)
    st = hip_check(c, hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0), "rk graph instantiate");
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  if (st != DG_OK) {
    c->graph = nullptr;
    return st;
  }
  c->graph_steps = nsteps;
  c->graph_cur = cur0;
  return DG_OK;
}

dg_status dg_rk_graph_launch(dg_ctx* c, int repeats) {
  dg_status st = need_bound(c);
  if (st != DG_OK) return st;
  if (!c->graph) return fail(c, DG_ESTATE, "no rk graph (dg_rk_graph_build)");
  if (repeats < 0) return fail(c, DG_EINVAL, "repeats < 0");
  if (repeats == 0) return DG_OK;
  if (c->cur != c->graph_cur) {
    // the state sits in the other buffer (dg_set_state, an odd dg_rk_step):
    // move it to the one the graph reads
    const size_t bytes = 5 * static_cast<size_t>(c->n_dof) * sizeof(double);
    if ((st = hip_check(c, hipMemcpyAsync(c->U[c->graph_cur], c->U[c->cur], bytes, hipMemcpyDeviceToDevice,
                                          c->stream),
                        "rk graph state copy")) != DG_OK)
      return st;
    c->cur = c->graph_cur;
  }
  for (int r = 0; r < repeats; ++r)
    if ((st = hip_check(c, hipGraphLaunch(c->graph, c->stream), "rk graph launch")) != DG_OK) return st;
  return DG_OK;
}

dg_status dg_free(dg_ctx* c) {
  if (c) {
    for (hipEvent_t e : c->events)
      if (e) (void)hipEventDestroy(e);
    if (c->event_start) (void)hipEventDestroy(c->event_start);
    drop_graph(c);
  }
  delete c;
  return DG_OK;
}

}  // extern "C"
