// Guard-cell domain decomposition of the PSATD step on one device.
//
// The paper's parallel solver (Sec. II.A) splits the domain into subdomains
// extended by guard regions that hold copies of the neighbouring subdomains,
// and solves Maxwell's equations on each with local FFTs.  Here every
// subdomain is one patch of a batched PSATD plan.  One step:
//   scatter  global fields -> every local patch (interior and guards, the
//            guards read from the neighbours' current values: the exchange);
//   push     one step of the batched plan on all local patches;
//   gather   each local interior -> its box of the global E and B.
// On several GPUs the scatter is the halo exchange (face neighbours over
// xGMI) and the gather disappears (each rank owns its interior).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.hpp"
#include "psatd.h"

psatd_status set_last_error(psatd_status s, const std::string& msg);

namespace psatd {
namespace {

struct DomainGeom {
  long long n[3];   // global nx, ny, nz
  long long ns[3];  // subdomain box per axis
  long long nl[3];  // local patch per axis (box + 2 guards on split axes)
  long long g[3];   // guards per side (0 on unsplit axes)
  int parts[3];
  long long local_cells;
};

__device__ __forceinline__ long long wrap(long long i, long long n) {
  const long long r = i % n;
  return r < 0 ? r + n : r;
}

// local[c][p * local_cells + r] = global[c][periodic global position]
template <typename S>
__global__ void scatter_kernel(DomainGeom G, FieldPtrs global, FieldPtrs local, int ncomp,
                               long long total) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long p = i / G.local_cells;
    const long long r = i - p * G.local_cells;
    const long long lx = r % G.nl[0];
    const long long ly = (r / G.nl[0]) % G.nl[1];
    const long long lz = r / (G.nl[0] * G.nl[1]);
    const long long sx = p % G.parts[0];
    const long long sy = (p / G.parts[0]) % G.parts[1];
    const long long sz = p / ((long long)G.parts[0] * G.parts[1]);
    const long long gx = wrap(sx * G.ns[0] - G.g[0] + lx, G.n[0]);
    const long long gy = wrap(sy * G.ns[1] - G.g[1] + ly, G.n[1]);
    const long long gz = wrap(sz * G.ns[2] - G.g[2] + lz, G.n[2]);
    const long long src = (gz * G.n[1] + gy) * G.n[0] + gx;
    for (int c = 0; c < ncomp; ++c)
      static_cast<S*>(local.f[c])[i] = static_cast<const S*>(global.f[c])[src];
  }
}

// global[c][position] = interior cell of the patch that owns the position
template <typename S>
__global__ void gather_kernel(DomainGeom G, FieldPtrs local, FieldPtrs global, int ncomp,
                              long long total) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long gx = i % G.n[0];
    const long long gy = (i / G.n[0]) % G.n[1];
    const long long gz = i / (G.n[0] * G.n[1]);
    const long long sx = gx / G.ns[0], sy = gy / G.ns[1], sz = gz / G.ns[2];
    const long long lx = gx - sx * G.ns[0] + G.g[0];
    const long long ly = gy - sy * G.ns[1] + G.g[1];
    const long long lz = gz - sz * G.ns[2] + G.g[2];
    const long long p = (sz * G.parts[1] + sy) * G.parts[0] + sx;
    const long long j = p * G.local_cells + (lz * G.nl[1] + ly) * G.nl[0] + lx;
    for (int c = 0; c < ncomp; ++c)
      static_cast<S*>(global.f[c])[i] = static_cast<const S*>(local.f[c])[j];
  }
}

psatd_status fail(psatd_status s, const std::string& m) { return set_last_error(s, m); }

psatd_status hip_fail(hipError_t e, const char* what) {
  // reset the runtime's last-error state, which the failed call set, so that
  // it does not surface again at the caller's next, unrelated launch check
  (void)hipGetLastError();
  return fail(e == hipErrorOutOfMemory ? PSATD_ERR_OOM : PSATD_ERR_HIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace
}  // namespace psatd

using namespace psatd;

struct psatd_domain_s {
  psatd_plan_t plan = nullptr;
  psatd_config cfg{};
  int device = 0;
  int nin = 6;
  size_t elem = 4;
  DomainGeom geom{};
  long long npatch = 0;
  void* local = nullptr;  // nin components x npatch x local_cells
  FieldPtrs local_ptrs{};
};

namespace {

bool valid_len(long long n) {
  if (n < 2 || n > 4096 || n % 2) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

void destroy_domain(psatd_domain_s* d) {
  if (!d) return;
  if (d->plan) (void)psatd_destroy(d->plan);
  if (d->local) (void)hipFree(d->local);
  delete d;
}

template <typename S>
hipError_t launch_scatter(const DomainGeom& G, const FieldPtrs& g, const FieldPtrs& l, int ncomp,
                          long long total, hipStream_t s) {
  const int b = 256;
  const long long blocks = std::min<long long>((total + b - 1) / b, 65536);
  hipLaunchKernelGGL(scatter_kernel<S>, dim3(static_cast<unsigned>(blocks)), dim3(b), 0, s, G, g,
                     l, ncomp, total);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_gather(const DomainGeom& G, const FieldPtrs& l, const FieldPtrs& g, int ncomp,
                         long long total, hipStream_t s) {
  const int b = 256;
  const long long blocks = std::min<long long>((total + b - 1) / b, 65536);
  hipLaunchKernelGGL(gather_kernel<S>, dim3(static_cast<unsigned>(blocks)), dim3(b), 0, s, G, l,
                     g, ncomp, total);
  return hipGetLastError();
}

}  // namespace

extern "C" {

psatd_status psatd_domain_create(const psatd_config* cfg, const psatd_domain_desc* dom,
                                 int32_t device, psatd_domain_t* out) {
  try {
    if (!cfg || !dom || !out) return fail(PSATD_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (dom->ndim != 2 && dom->ndim != 3) return fail(PSATD_ERR_INVALID_ARG, "ndim must be 2 or 3");
    DomainGeom G{};
    long long npatch = 1;
    for (int a = 0; a < 3; ++a) {
      const bool used = !(dom->ndim == 2 && a == 1);
      const long long n = used ? dom->n[a] : 1;
      const int parts = used ? dom->parts[a] : 1;
      if (dom->ndim == 2 && a == 1 && (dom->n[1] != 1 || dom->parts[1] != 1))
        return fail(PSATD_ERR_INVALID_ARG, "2D domains need n[1] = 1 and parts[1] = 1");
      if (n < 1 || parts < 1 || n % parts != 0)
        return fail(PSATD_ERR_INVALID_ARG, "every axis must split into parts of equal size");
      if (dom->guard[a] < 0) return fail(PSATD_ERR_INVALID_ARG, "guard widths must be >= 0");
      G.n[a] = n;
      G.parts[a] = parts;
      G.ns[a] = n / parts;
      G.g[a] = parts > 1 ? dom->guard[a] : 0;
      G.nl[a] = G.ns[a] + 2 * G.g[a];
      if (used && !valid_len(G.nl[a]))
        return fail(PSATD_ERR_UNSUPPORTED_SIZE,
                    "local patch length " + std::to_string(G.nl[a]) + " on axis " +
                        std::to_string(a) + " (box + 2 guards) is not an even 2^a 3^b <= 4096");
      npatch *= parts;
    }
    G.local_cells = G.nl[0] * G.nl[1] * G.nl[2];
    if (npatch > (1 << 20)) return fail(PSATD_ERR_INVALID_ARG, "too many subdomains");

    std::vector<psatd_patch_desc> descs(static_cast<size_t>(npatch));
    for (long long p = 0; p < npatch; ++p) {
      psatd_patch_desc& d = descs[static_cast<size_t>(p)];
      d = psatd_patch_desc{};
      d.ndim = dom->ndim;
      for (int a = 0; a < 3; ++a) {
        d.n[a] = G.nl[a];
        d.d[a] = dom->d[a];
      }
      d.dt = dom->dt;
      d.offset = p * G.local_cells;
    }
    psatd_domain_s* D = new psatd_domain_s();
    D->cfg = *cfg;
    D->device = device;
    D->geom = G;
    D->npatch = npatch;
    D->nin = cfg->source_mode == PSATD_VACUUM ? 6 : (cfg->source_mode == PSATD_SOURCES_RHO ? 11 : 9);
    D->elem = cfg->precision == PSATD_FP64 ? 8 : 4;
    psatd_status st = psatd_plan(cfg, descs.data(), static_cast<int32_t>(npatch), device, &D->plan);
    if (st != PSATD_OK) {
      destroy_domain(D);
      return st;  // the plan has set the message
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(device);
    const size_t comp_bytes = static_cast<size_t>(npatch * G.local_cells) * D->elem;
    if (e == hipSuccess) e = hipMalloc(&D->local, comp_bytes * D->nin);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
      D->local = nullptr;
      destroy_domain(D);
      return hip_fail(e, "hipMalloc(local patches)");
    }
    for (int c = 0; c < D->nin; ++c) D->local_ptrs.f[c] = static_cast<char*>(D->local) + c * comp_bytes;
    *out = D;
    return PSATD_OK;
  } catch (const std::exception& ex) {
    return fail(PSATD_ERR_OOM, std::string("host exception: ") + ex.what());
  }
}

psatd_status psatd_domain_local_shape(psatd_domain_t dom, int64_t* npatch, int64_t local_n[3]) {
  if (!dom || !npatch || !local_n) return fail(PSATD_ERR_INVALID_ARG, "NULL argument");
  *npatch = dom->npatch;
  for (int a = 0; a < 3; ++a) local_n[a] = dom->geom.nl[a];
  return PSATD_OK;
}

psatd_status psatd_domain_push(psatd_domain_t dom, const psatd_fields* global, int32_t nsteps,
                               void* hip_stream) {
  if (!dom) return fail(PSATD_ERR_INVALID_ARG, "domain is NULL");
  if (!global) return fail(PSATD_ERR_INVALID_ARG, "fields is NULL");
  if (nsteps < 0) return fail(PSATD_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (nsteps > 1 && dom->cfg.source_mode != PSATD_VACUUM)
    return fail(PSATD_ERR_INVALID_ARG, "with sources, push one step at a time (nsteps = 1)");
  FieldPtrs g{};
  for (int i = 0; i < 3; ++i) {
    if (!global->E[i] || !global->B[i])
      return fail(PSATD_ERR_INVALID_ARG, "E and B pointers must be non-NULL");
    g.f[kEx + i] = global->E[i];
    g.f[kBx + i] = global->B[i];
  }
  if (dom->cfg.source_mode != PSATD_VACUUM) {
    for (int i = 0; i < 3; ++i) {
      if (!global->J[i]) return fail(PSATD_ERR_INVALID_ARG, "J pointers must be non-NULL with sources");
      g.f[kJx + i] = const_cast<void*>(global->J[i]);
    }
  }
  if (dom->cfg.source_mode == PSATD_SOURCES_RHO) {
    if (!global->rho_old || !global->rho_new)
      return fail(PSATD_ERR_INVALID_ARG, "rho_old and rho_new must be non-NULL in the rho form");
    g.f[kRhoOld] = const_cast<void*>(global->rho_old);
    g.f[kRhoNew] = const_cast<void*>(global->rho_new);
  }
  psatd_fields lf{};
  for (int i = 0; i < 3; ++i) {
    lf.E[i] = dom->local_ptrs.f[kEx + i];
    lf.B[i] = dom->local_ptrs.f[kBx + i];
    if (dom->nin > 6) lf.J[i] = dom->local_ptrs.f[kJx + i];
  }
  if (dom->nin > 9) {
    lf.rho_old = dom->local_ptrs.f[kRhoOld];
    lf.rho_new = dom->local_ptrs.f[kRhoNew];
  }
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(dom->device) != hipSuccess) return fail(PSATD_ERR_HIP, "hipSetDevice failed");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const DomainGeom& G = dom->geom;
  const long long local_total = dom->npatch * G.local_cells;
  const long long global_total = G.n[0] * G.n[1] * G.n[2];
  psatd_status st = PSATD_OK;
  for (int step = 0; step < nsteps && st == PSATD_OK; ++step) {
    hipError_t e = dom->elem == 8
                       ? launch_scatter<double>(G, g, dom->local_ptrs, dom->nin, local_total, s)
                       : launch_scatter<float>(G, g, dom->local_ptrs, dom->nin, local_total, s);
    if (e != hipSuccess) {
      st = hip_fail(e, "domain scatter");
      break;
    }
    st = psatd_push(dom->plan, &lf, 1, hip_stream);
    if (st != PSATD_OK) break;
    e = dom->elem == 8 ? launch_gather<double>(G, dom->local_ptrs, g, 6, global_total, s)
                       : launch_gather<float>(G, dom->local_ptrs, g, 6, global_total, s);
    if (e != hipSuccess) st = hip_fail(e, "domain gather");
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  return st;
}

psatd_status psatd_domain_destroy(psatd_domain_t dom) {
  if (!dom) return fail(PSATD_ERR_INVALID_ARG, "domain is NULL");
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(dom->device);
  destroy_domain(dom);
  if (prev >= 0) (void)hipSetDevice(prev);
  return PSATD_OK;
}

}  // extern "C"
