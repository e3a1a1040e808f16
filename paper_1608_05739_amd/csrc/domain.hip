// Guard-cell domain decomposition of the PSATD step on one device.
//
// The paper's parallel solver (Sec. II.A) splits the domain into subdomains
// extended by guard regions that hold copies of the neighbouring subdomains,
// and solves Maxwell's equations on each with local FFTs.  Here every
// subdomain is one patch of a batched PSATD plan whose patches know their
// place in the global grid (GlobalMap): the forward x pass reads each patch,
// interior and guards, straight from the global fields at the periodic
// positions (the guard exchange), and the inverse x pass writes each patch's
// interior straight back (the gather).  One step is one push of that plan;
// no local copy of the fields exists.  The x passes of every patch read
// before any writes (they are separate launches), so the in-place update of
// the global fields is safe.  On several GPUs the reads of the guards become
// the halo exchange with the face neighbours over xGMI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.hpp"
#include "psatd.h"

psatd_status set_last_error(psatd_status s, const std::string& msg);
// (api.cpp) a plan whose patches read and write a global grid
psatd_status plan_mapped(const psatd_config* cfg, const psatd_patch_desc* patches,
                         const psatd::GlobalMap* maps, int32_t npatches, int32_t device,
                         psatd_plan_t* out);

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
  delete d;
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
      if (a == 0 && parts > 1 && dom->guard[0] % 2 != 0)
        return fail(PSATD_ERR_INVALID_ARG, "the x guard width must be even (rows are read in pairs)");
      npatch *= parts;
    }
    G.local_cells = G.nl[0] * G.nl[1] * G.nl[2];
    if (npatch > (1 << 20)) return fail(PSATD_ERR_INVALID_ARG, "too many subdomains");

    std::vector<psatd_patch_desc> descs(static_cast<size_t>(npatch));
    std::vector<GlobalMap> maps(static_cast<size_t>(npatch));
    for (long long p = 0; p < npatch; ++p) {
      psatd_patch_desc& d = descs[static_cast<size_t>(p)];
      d = psatd_patch_desc{};
      d.ndim = dom->ndim;
      for (int a = 0; a < 3; ++a) {
        d.n[a] = G.nl[a];
        d.d[a] = dom->d[a];
      }
      d.dt = dom->dt;
      d.offset = p * G.local_cells;  // (unused: the x passes go through the map)
      // box (sx, sy, sz); local (0, 0, 0) sits at the box start minus the guards
      const long long sidx[3] = {p % G.parts[0], (p / G.parts[0]) % G.parts[1],
                                 p / (static_cast<long long>(G.parts[0]) * G.parts[1])};
      long long org[3];
      for (int a = 0; a < 3; ++a) {
        const long long o = (sidx[a] * G.ns[a] - G.g[a]) % G.n[a];
        org[a] = o < 0 ? o + G.n[a] : o;
      }
      GlobalMap& m = maps[static_cast<size_t>(p)];
      m.on = 1;
      m.gnx = static_cast<int>(G.n[0]);
      m.gny = static_cast<int>(G.n[1]);
      m.gnz = static_cast<int>(G.n[2]);
      m.ox = static_cast<int>(org[0]);
      m.oy = static_cast<int>(org[1]);
      m.oz = static_cast<int>(org[2]);
      m.ix0 = static_cast<int>(G.g[0]);
      m.ix1 = static_cast<int>(G.g[0] + G.ns[0]);
      m.iy0 = static_cast<int>(G.g[1]);
      m.iy1 = static_cast<int>(G.g[1] + G.ns[1]);
      m.iz0 = static_cast<int>(G.g[2]);
      m.iz1 = static_cast<int>(G.g[2] + G.ns[2]);
    }
    psatd_domain_s* D = new psatd_domain_s();
    D->cfg = *cfg;
    D->device = device;
    D->geom = G;
    D->npatch = npatch;
    D->nin = cfg->source_mode == PSATD_VACUUM ? 6 : (cfg->source_mode == PSATD_SOURCES_RHO ? 11 : 9);
    D->elem = cfg->precision == PSATD_FP64 ? 8 : 4;
    psatd_status st = plan_mapped(cfg, descs.data(), maps.data(), static_cast<int32_t>(npatch),
                                  device, &D->plan);
    if (st != PSATD_OK) {
      destroy_domain(D);
      return st;  // the plan has set the message
    }
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
  // the plan's x passes read and write the global fields through the maps
  return psatd_push(dom->plan, global, nsteps, hip_stream);
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
