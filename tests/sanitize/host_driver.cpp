// Host paths of the C ABI under AddressSanitizer and UBSan (CPU only): the
// LGL tables, mesh and physics validation (including the host copies of the
// face and node arrays), workspace sizing, wall-face counts and the
// state errors of every call made before a workspace is bound.  Exit status 0
// when every expectation holds.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/dgsem.h"

static int failures = 0;
#define EXPECT(cond)                                                     \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

struct Mesh {
  std::vector<double> f[3];
  dg_mesh_desc d{};
  Mesh(int N, int nx, int ny, int nz, int bc0 = 0, int bc1 = 0, int bc2 = 0) {
    const int n[3] = {nx, ny, nz}, bc[3] = {bc0, bc1, bc2};
    d.N = N;
    for (int k = 0; k < 3; ++k) {
      f[k].resize(n[k] + 1);
      for (int i = 0; i <= n[k]; ++i) f[k][i] = 0.1 * i * i + i;  // strictly increasing, non-uniform
      d.nelem[k] = n[k];
      d.faces[k] = f[k].data();
      d.bc[k] = bc[k];
    }
    d.T_wall = 1.0;
    d.wm_node = 1;
  }
};

static dg_physics gas(int precision = DG_FP64, int flux = DG_FLUX_KG_LLF) {
  dg_physics p{};
  p.gamma = 1.4;
  p.R = 1.0;
  p.mu = 0.01;
  p.Pr = 0.72;
  p.viscous = 1;
  p.precision = precision;
  p.flux = flux;
  return p;
}

int main() {
  // LGL tables: weights sum to 2, nodes antisymmetric, endpoints +-1
  for (int N = 1; N <= 16; ++N) {
    std::vector<double> xi(N + 1), w(N + 1);
    EXPECT(dg_lgl(N, xi.data(), w.data()) == DG_OK);
    double s = 0.0;
    for (int i = 0; i <= N; ++i) {
      s += w[i];
      EXPECT(std::fabs(xi[i] + xi[N - i]) < 1e-14);
    }
    EXPECT(std::fabs(s - 2.0) < 1e-13);
    EXPECT(xi[0] == -1.0 && xi[N] == 1.0);
  }
  EXPECT(dg_lgl(0, nullptr, nullptr) != DG_OK);

  const dg_physics p = gas();
  dg_ctx* c = nullptr;
  // valid meshes of every kind; sizes and counts
  const int kinds[4][3] = {{0, 0, 0}, {0, 1, 0}, {2, 0, 2}, {1, 2, 1}};
  for (int N : {3, 5, 7}) {
    for (auto& b : kinds) {
      Mesh m(N, 3, 2, 4, b[0], b[1], b[2]);
      c = nullptr;
      EXPECT(dg_init_mesh(&m.d, &p, nullptr, &c) == DG_OK);
      if (!c) continue;
      long long ndof = 0, nw = 0;
      size_t fwd = 0, adj = 0;
      EXPECT(dg_n_dof(c, &ndof) == DG_OK && ndof == 24LL * (N + 1) * (N + 1) * (N + 1));
      EXPECT(dg_workspace_bytes(c, 0, &fwd) == DG_OK && dg_workspace_bytes(c, 1, &adj) == DG_OK);
      EXPECT(fwd >= 15 * sizeof(double) * ndof && adj > fwd);
      EXPECT(dg_wall_faces(c, &nw) == DG_OK);
      long long expect = 0;
      if (b[0]) expect += 2 * 2 * 4;
      if (b[1]) expect += 2 * 3 * 4;
      if (b[2]) expect += 2 * 3 * 2;
      EXPECT(nw == expect);
      // calls before a workspace is bound report DG_ESTATE without touching the device
      double dummy[5] = {0};
      EXPECT(dg_eval_rhs(c, dummy, dummy + 1, 0.0) == DG_ESTATE);
      EXPECT(dg_rk_step(c, 0.0, 1e-3, 1) == DG_ESTATE);
      EXPECT(dg_set_state(c, dummy) == DG_ESTATE);
      EXPECT(dg_eval_rhs_vjp(c, dummy, dummy, dummy + 1, 0.0) == DG_ESTATE);
      EXPECT(dg_wall_stress(c, dummy, 1, dummy) == DG_ESTATE);
      EXPECT(dg_get_state(c, dummy) == DG_ESTATE);
      EXPECT(dg_eval_lift(c, dummy, dummy + 1) == DG_ESTATE);
      EXPECT(dg_rk_step_vjp(c, dummy, 0.0, 1e-3, dummy, dummy + 1) == DG_ESTATE);
      EXPECT(dg_rk_record_stages(c, dummy, 0.0, 1e-3, 1, dummy + 1) == DG_ESTATE);
      EXPECT(dg_rk_step_vjp_stages(c, dummy, 0.0, 1e-3, dummy, dummy + 1) == DG_ESTATE);
      EXPECT(dg_kinetic_energy(c, dummy, dummy + 1) == DG_ESTATE);
      EXPECT(dg_kinetic_energy_grad(c, dummy, dummy + 1) == DG_ESTATE);
      EXPECT(dg_rk_graph_build(c, 1e-3, 2) == DG_ESTATE);
      EXPECT(dg_rk_graph_launch(c, 1) == DG_ESTATE);
      double ms[2];
      int cnt[2];
      EXPECT(dg_timing_end(c, ms, cnt) == DG_ESTATE);  // no dg_timing_begin
      EXPECT(dg_last_error(c) != nullptr);
      EXPECT(dg_free(c) == DG_OK);
    }
  }
  // curved elements: node coordinates copied on the host, faces optional
  {
    const int N = 5, nx = 2, ny = 3, nz = 2, NP = N + 1;
    const long long ndof = 1LL * nx * ny * nz * NP * NP * NP;
    std::vector<double> X(3 * ndof);
    for (long long q = 0; q < 3 * ndof; ++q) X[q] = 0.001 * static_cast<double>(q % 977);
    Mesh m(N, nx, ny, nz);
    for (int k = 0; k < 3; ++k) m.d.faces[k] = nullptr;
    m.d.nodes = X.data();
    c = nullptr;
    EXPECT(dg_init_mesh(&m.d, &p, nullptr, &c) == DG_OK);
    size_t plain = 0, curved = 0;
    if (c) {
      EXPECT(dg_workspace_bytes(c, 0, &curved) == DG_OK);
      dg_free(c);
    }
    Mesh m2(N, nx, ny, nz);
    c = nullptr;
    EXPECT(dg_init_mesh(&m2.d, &p, nullptr, &c) == DG_OK);
    if (c) {
      EXPECT(dg_workspace_bytes(c, 0, &plain) == DG_OK);
      dg_free(c);
    }
    EXPECT(curved >= plain + 10 * sizeof(double) * ndof);
    X[3 * ndof - 1] = NAN;
    c = nullptr;
    EXPECT(dg_init_mesh(&m.d, &p, nullptr, &c) == DG_EINVAL && c == nullptr);
    X[3 * ndof - 1] = 0.0;
    m.d.bc[1] = DG_BC_ISOTHERMAL_WALL;
    c = nullptr;
    EXPECT(dg_init_mesh(&m.d, &p, nullptr, &c) == DG_OK);
    if (c) dg_free(c);
    m.d.bc[1] = DG_BC_WALL_MODEL;
    EXPECT(dg_init_mesh(&m.d, &p, nullptr, &c) == DG_EUNSUPPORTED);
  }
  // invalid arguments
  {
    Mesh m(3, 2, 2, 2);
    EXPECT(dg_init_mesh(nullptr, &p, nullptr, &c) == DG_EINVAL);
    m.f[1][1] = m.f[1][0];  // not strictly increasing
    EXPECT(dg_init_mesh(&m.d, &p, nullptr, &c) == DG_EINVAL);
    Mesh m4(4, 2, 2, 2);
    EXPECT(dg_init_mesh(&m4.d, &p, nullptr, &c) == DG_EUNSUPPORTED);
    Mesh mw(3, 2, 2, 2, 0, 2, 0);
    mw.d.wm_node = 4;
    EXPECT(dg_init_mesh(&mw.d, &p, nullptr, &c) == DG_EINVAL);
    Mesh ok(3, 2, 2, 2);
    dg_physics q = gas();
    q.gamma = 1.0;
    EXPECT(dg_init_mesh(&ok.d, &q, nullptr, &c) == DG_EINVAL);
    q = gas(DG_MIXED_NOREF, DG_FLUX_EC_ROE);
    EXPECT(dg_init_mesh(&ok.d, &q, nullptr, &c) == DG_EUNSUPPORTED);
    q = gas(DG_MIXED, DG_FLUX_EC_ROE);
    c = nullptr;
    EXPECT(dg_init_mesh(&ok.d, &q, nullptr, &c) == DG_OK);
    if (c) dg_free(c);
    q = gas();
    q.viscosity = DG_VISC_SUTHERLAND;
    q.T_ref = 1.0;
    q.S = -0.5;
    EXPECT(dg_init_mesh(&ok.d, &q, nullptr, &c) == DG_EINVAL);
    q.S = 0.4;
    c = nullptr;
    EXPECT(dg_init_mesh(&ok.d, &q, nullptr, &c) == DG_OK);
    if (c) dg_free(c);
  }
  EXPECT(dg_free(nullptr) == DG_OK);
  if (failures) std::fprintf(stderr, "%d expectation(s) failed\n", failures);
  else std::printf("host driver: all expectations hold\n");
  return failures ? 1 : 0;
}
