// Stand-ins for the kernel launchers (defined in the .hip files) so that the
// host half of the library links into a CPU-only sanitizer build.  The
// driver only takes paths that end before any launch; reaching one aborts.
#include <cstdio>
#include <cstdlib>

#include "../../paper_2606_18927_amd/csrc/dg_internal.hpp"

namespace {
[[noreturn]] void reached(const char* what) {
  std::fprintf(stderr, "kernel launcher %s reached in a host-only build\n", what);
  std::abort();
}
}  // namespace

namespace dg {
hipError_t launch_face_flux(int, int, const DevMesh&, const DevPhys&, const DevBasis&, const double*, void*,
                            hipStream_t) { reached("face_flux"); }
hipError_t launch_rhs(int, int, const DevMesh&, const DevPhys&, const DevBasis&, const double*, const void*,
                      double*, int*, hipStream_t) { reached("rhs"); }
hipError_t launch_rk_stage(int, int, const DevMesh&, const DevPhys&, const DevBasis&, const double*, const void*,
                           double*, double*, const Stage&, int*, hipStream_t) { reached("rk_stage"); }
hipError_t launch_lift(int, const DevMesh&, const DevPhys&, const DevBasis&, const double*, double*,
                       hipStream_t) { reached("lift"); }
hipError_t launch_rhs_vjp(int, const DevMesh&, const DevPhys&, const DevBasis&, const double*, const double*,
                          double*, double*, double*, bool, double, hipStream_t, double*, double, double) {
  reached("rhs_vjp");
}
hipError_t launch_axpby(double*, const double*, double, double, long long, hipStream_t) { reached("axpby"); }
hipError_t launch_wall_stress(int, const DevMesh&, const DevPhys&, const double*, int, double, double, double*,
                              hipStream_t) { reached("wall_stress"); }
hipError_t launch_kinetic_energy(int, const DevMesh&, const double*, const double*, double*, int, double, double*,
                                 hipStream_t) { reached("kinetic_energy"); }
hipError_t launch_kinetic_energy_grad(int, const DevMesh&, const double*, const double*, double, double*,
                                      hipStream_t) { reached("kinetic_energy_grad"); }
hipError_t launch_triad(const double*, const double*, double, double*, long long, hipStream_t) {
  reached("triad");
}
hipError_t launch_metrics(int, const double*, double*, double*, bool, const DevBasis&, long long, int*,
                          hipStream_t) {
  reached("metrics");
}
hipError_t launch_face_flux_curv(int, int, const DevMesh&, const DevPhys&, const DevBasis&, const double*, void*,
                                 hipStream_t) { reached("face_flux_curv"); }
hipError_t launch_rhs_curv(int, int, const DevMesh&, const DevPhys&, const DevBasis&, const double*, const void*,
                           double*, int*, hipStream_t) { reached("rhs_curv"); }
hipError_t launch_rk_stage_curv(int, int, const DevMesh&, const DevPhys&, const DevBasis&, const double*,
                                const void*, double*, double*, const Stage&, int*, hipStream_t) {
  reached("rk_stage_curv");
}
}  // namespace dg
