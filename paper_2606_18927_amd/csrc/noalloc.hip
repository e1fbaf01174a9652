// dg_eval_rhs_noalloc: the right-hand side of dg_eval_rhs with its scratch
// memory (the derivative matrix, the element scale tables, the face viscous
// fluxes, the wall-model stress and the status word) in a file-scope device
// array instead of the caller's workspace, for callers that cannot allocate
// device memory.  The same kernels run in the same order, so the result is
// bitwise that of dg_eval_rhs.
//
// The array's device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept; host code uses
// that address only, never the array's name.  Every call on a device shares
// its array: the tables and the status word are rewritten by each call, and
// calls that overlap on one device race.
#include <mutex>

#include "dg_internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // per device
constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};

// Values of one table written by a kernel from its arguments (no host-to-
// device copy from pageable memory, so the call stays allocation-free and
// can be captured): at most kChunk values per launch.
constexpr int kChunk = 256;
struct Chunk {
  double v[kChunk];
  int n;
};

__global__ void k_put(double* __restrict__ dst, Chunk ch) {
  const int t = threadIdx.x;
  if (t < ch.n) dst[t] = ch.v[t];
}

__global__ void k_zero_status(int* status) {
  if (threadIdx.x == 0) status[0] = 0;
}

hipError_t put_table(double* dst, const double* src, size_t n, hipStream_t s) {
  for (size_t at = 0; at < n; at += kChunk) {
    Chunk ch{};
    ch.n = static_cast<int>(n - at < static_cast<size_t>(kChunk) ? n - at : kChunk);
    for (int q = 0; q < ch.n; ++q) ch.v[q] = src[at + q];
    hipLaunchKernelGGL(k_put, dim3(1), dim3(kChunk), 0, s, dst + at, ch);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

dg_status fail(dg_ctx* c, dg_status st, const std::string& msg) {
  c->err = msg;
  return st;
}

// Device address of `scratch` on the device of `stream`.
dg_status scratch_address(dg_ctx* c, unsigned char** out) {
  int dev = 0;
  hipError_t e = hipStreamGetDevice(c->stream, &dev);
  if (e != hipSuccess) return fail(c, DG_EHIP, std::string("hipStreamGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(c, DG_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    int cur = 0;
    if ((e = hipGetDevice(&cur)) != hipSuccess)
      return fail(c, DG_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess)
      return fail(c, DG_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr)
      return fail(c, DG_EHIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return DG_OK;
}

}  // namespace

extern "C" dg_status dg_eval_rhs_noalloc(dg_ctx* c, const double* U, double* Ut, double /*t*/,
                                         int* status_dev) {
  if (!c || !U || !Ut) return DG_EINVAL;
  if (c->curvilinear) return fail(c, DG_EUNSUPPORTED, "the allocation-free call covers axis-aligned elements");
  const size_t NP = c->N + 1;
  const size_t rsize = c->phys.precision == DG_FP64 ? sizeof(double) : sizeof(float);
  // scratch layout: D, s_x, s_y, s_z, status, face fluxes, wall stress
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t oD = take(NP * NP * sizeof(double));
  size_t os[3];
  for (int d = 0; d < 3; ++d) os[d] = take(static_cast<size_t>(c->nelem[d]) * sizeof(double));
  const size_t ostatus = take(sizeof(int));
  const size_t offv = c->phys.viscous
                          ? take(static_cast<size_t>(c->nE) * dg::face_flux_values_per_element(c->N) * rsize)
                          : off;
  const size_t otau = c->wall_model ? take(static_cast<size_t>(c->n_wall_faces) * 3 * NP * NP * sizeof(double)) : off;
  if (off > kScratchBytes)
    return fail(c, DG_EINVAL,
                "mesh too large for the allocation-free call: needs " + std::to_string(off) +
                    " bytes of scratch, the limit is " + std::to_string(kScratchBytes));
  unsigned char* base = nullptr;
  if (dg_status st = scratch_address(c, &base); st != DG_OK) return st;
  const auto hip = [&](hipError_t e, const char* what) {
    return e == hipSuccess ? DG_OK : fail(c, DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };

  double* dD = reinterpret_cast<double*>(base + oD);
  dg_status st = hip(put_table(dD, c->D.data(), NP * NP, c->stream), "table kernel");
  dg::DevMesh m{};
  for (int d = 0; d < 3 && st == DG_OK; ++d) {
    double* ds = reinterpret_cast<double*>(base + os[d]);
    st = hip(put_table(ds, c->s[d].data(), c->s[d].size(), c->stream), "table kernel");
    m.n[d] = c->nelem[d];
    m.bc[d] = c->bc[d];
    m.s[d] = ds;
  }
  if (st != DG_OK) return st;
  int* status = status_dev ? status_dev : reinterpret_cast<int*>(base + ostatus);
  if (!status_dev) {
    hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, c->stream, status);
    if ((st = hip(hipGetLastError(), "status kernel")) != DG_OK) return st;
  }
  m.T_wall = c->T_wall;
  m.nE = c->nE;
  m.tauw = c->wall_model ? reinterpret_cast<double*>(base + otau) : nullptr;
  m.geo = nullptr;
  const dg::DevPhys p = dg::device_physics(c);
  dg::DevBasis b{};
  b.D = dD;
  b.inv_w_end = 1.0 / c->w[0];
  void* ffv = base + offv;
  if (c->phys.viscous &&
      (st = hip(dg::launch_face_flux(c->N, c->phys.precision, m, p, b, U, ffv, c->stream), "face flux kernel")) !=
          DG_OK)
    return st;
  if (c->wall_model && c->phys.viscous &&
      (st = hip(dg::launch_wall_stress(c->N, m, p, U, c->wm_node, c->xi[c->wm_node] + 1.0, std::cbrt(c->phys.Pr),
                                       const_cast<double*>(m.tauw), c->stream),
                "wall stress kernel")) != DG_OK)
    return st;
  return hip(dg::launch_rhs(c->N, c->phys.precision, m, p, b, U, ffv, Ut, status, c->stream), "rhs kernel");
}
