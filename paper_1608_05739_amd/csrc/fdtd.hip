// FDTD contrast solvers on the Yee grid: Yee, order-p FDTD and CKC (Sec. III.A;
// Table 1, Yee, CKC and FDTD p-order rows).  The paper measures PSATD against
// these; they share no kernel with the PSATD path.
//
// Leapfrog: E at integer times, B at half-integer times.  One step
//   Faraday:  B^{n+1/2} = B^{n-1/2} - dt curl+ E^n
//   Ampere:   E^{n+1}   = E^n + dt (c^2 curl- B^{n+1/2} - J^{n+1/2} / eps0)
// Staggered positions (cells):  Ex (i+1/2, j, k)  Ey (i, j+1/2, k)  Ez (i, j, k+1/2)
//                               Bx (i, j+1/2, k+1/2)  By (i+1/2, j, k+1/2)  Bz (i+1/2, j+1/2, k)
// and J with E; element [k][j][i] of a component holds it at its own position.
// curl+ takes forward differences and curl- backward ones, with the staggered
// order-p weights C_l (p = 2: C_1 = 1):
//   D+ f[i] = sum_l C_l (f[i+l] - f[i-l+1]) / d,   D- f[i] = sum_l C_l (f[i+l-1] - f[i-l]) / d.
// CKC (2D, dx = dz, beta = 1/4): in curl+ only, each x-difference is averaged
// over z and each z-difference over x with weights (1 - beta, beta/2, beta/2).
// Grids are periodic.  Both updates are in place: a Faraday cell reads E and
// its own B, an Ampere cell B and its own E, so no cell reads a value the same
// launch writes.  Arithmetic is FP64 for either storage type.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.hpp"
#include "psatd.h"

psatd_status set_last_error(psatd_status s, const std::string& msg);

namespace psatd {
namespace {

constexpr int kMaxRadius = 16;  // orders up to 32
constexpr int kRowBlock = 256;  // threads per workgroup, one row segment each
constexpr double kBetaCKC = 0.25;

struct FdtdGeom {
  int nx, ny, nz;
  int r;             // stencil radius p / 2
  int xchunks;       // row segments of kRowBlock cells
  int pad0;
  long long off;     // element offset in the component buffers
  double dt;
  double c2dt;       // c^2 dt
  double dt_eps;     // dt / eps0
  double inv_d[3];   // 1 / dx, 1 / dy, 1 / dz
  double w[kMaxRadius];
};

enum Scheme : int { kYee = 0, kCKC = 1 };

__device__ __forceinline__ int wrap_up(int i, int l, int n) {
  const int j = i + l;
  return j >= n ? j - n : j;
}
__device__ __forceinline__ int wrap_dn(int i, int l, int n) {
  const int j = i - l;
  return j < 0 ? j + n : j;
}

// f at (x, y, z) shifted by s cells along axis a (|s| <= n_a)
template <typename S>
__device__ __forceinline__ double ld_shift(const S* f, const FdtdGeom& g, int x, int y, int z,
                                           int a, int s) {
  if (a == 0) x = s >= 0 ? wrap_up(x, s, g.nx) : wrap_dn(x, -s, g.nx);
  else if (a == 1) y = s >= 0 ? wrap_up(y, s, g.ny) : wrap_dn(y, -s, g.ny);
  else z = s >= 0 ? wrap_up(z, s, g.nz) : wrap_dn(z, -s, g.nz);
  return static_cast<double>(f[g.off + (static_cast<long long>(z) * g.ny + y) * g.nx + x]);
}

// D+ (FWD) or D- of f along axis a at (x, y, z); RAD > 0 is the radius at
// compile time, RAD = 0 takes g.r.
template <int RAD, bool FWD, typename S>
__device__ __forceinline__ double diff(const S* f, const FdtdGeom& g, int x, int y, int z, int a) {
  const int r = RAD > 0 ? RAD : g.r;
  double acc = 0.0;
#pragma unroll 4
  for (int l = 1; l <= r; ++l) {
    const double hi = ld_shift(f, g, x, y, z, a, FWD ? l : l - 1);
    const double lo = ld_shift(f, g, x, y, z, a, FWD ? -(l - 1) : -l);
    acc = fma(g.w[l - 1], hi - lo, acc);
  }
  return acc * g.inv_d[a];
}

// CKC forward difference along a (2D: a = 0 or 2), averaged over the other axis
template <typename S>
__device__ __forceinline__ double diff_ckc(const S* f, const FdtdGeom& g, int x, int y, int z,
                                           int a) {
  const int o = a == 0 ? 2 : 0;
  int xm = x, xp = x, zm = z, zp = z;
  if (o == 0) {
    xm = wrap_dn(x, 1, g.nx);
    xp = wrap_up(x, 1, g.nx);
  } else {
    zm = wrap_dn(z, 1, g.nz);
    zp = wrap_up(z, 1, g.nz);
  }
  const double d0 = diff<1, true>(f, g, x, y, z, a);
  const double dm = diff<1, true>(f, g, xm, y, zm, a);
  const double dp = diff<1, true>(f, g, xp, y, zp, a);
  return (1.0 - kBetaCKC) * d0 + 0.5 * kBetaCKC * (dm + dp);
}

// Row segment of the work: b -> (x, y, z); false past the row's end.
__device__ __forceinline__ bool cell_of(const FdtdGeom& g, long long b, int* x, int* y, int* z) {
  const long long row = b / g.xchunks;
  *x = static_cast<int>(b - row * g.xchunks) * kRowBlock + static_cast<int>(threadIdx.x);
  *y = static_cast<int>(row % g.ny);
  *z = static_cast<int>(row / g.ny);
  return *x < g.nx;
}

template <typename S, int DIM, int SCHEME, int RAD>
__global__ void __launch_bounds__(kRowBlock)
faraday_kernel(FdtdGeom g, FieldPtrs f, long long nblocks) {
  const S* Ex = static_cast<const S*>(f.f[kEx]);
  const S* Ey = static_cast<const S*>(f.f[kEy]);
  const S* Ez = static_cast<const S*>(f.f[kEz]);
  S* Bx = static_cast<S*>(f.f[kBx]);
  S* By = static_cast<S*>(f.f[kBy]);
  S* Bz = static_cast<S*>(f.f[kBz]);
  for (long long b = blockIdx.x; b < nblocks; b += gridDim.x) {
    int x, y, z;
    if (!cell_of(g, b, &x, &y, &z)) continue;
    double dzEy, dzEx, dxEz, dxEy;
    if constexpr (SCHEME == kCKC) {
      dzEy = diff_ckc(Ey, g, x, y, z, 2);
      dzEx = diff_ckc(Ex, g, x, y, z, 2);
      dxEz = diff_ckc(Ez, g, x, y, z, 0);
      dxEy = diff_ckc(Ey, g, x, y, z, 0);
    } else {
      dzEy = diff<RAD, true>(Ey, g, x, y, z, 2);
      dzEx = diff<RAD, true>(Ex, g, x, y, z, 2);
      dxEz = diff<RAD, true>(Ez, g, x, y, z, 0);
      dxEy = diff<RAD, true>(Ey, g, x, y, z, 0);
    }
    double dyEz = 0.0, dyEx = 0.0;
    if constexpr (DIM == 3) {
      dyEz = diff<RAD, true>(Ez, g, x, y, z, 1);
      dyEx = diff<RAD, true>(Ex, g, x, y, z, 1);
    }
    const long long i = g.off + (static_cast<long long>(z) * g.ny + y) * g.nx + x;
    Bx[i] = static_cast<S>(static_cast<double>(Bx[i]) - g.dt * (dyEz - dzEy));
    By[i] = static_cast<S>(static_cast<double>(By[i]) - g.dt * (dzEx - dxEz));
    Bz[i] = static_cast<S>(static_cast<double>(Bz[i]) - g.dt * (dxEy - dyEx));
  }
}

template <typename S, int DIM, int RAD, bool SRC>
__global__ void __launch_bounds__(kRowBlock)
ampere_kernel(FdtdGeom g, FieldPtrs f, long long nblocks) {
  S* Ex = static_cast<S*>(f.f[kEx]);
  S* Ey = static_cast<S*>(f.f[kEy]);
  S* Ez = static_cast<S*>(f.f[kEz]);
  const S* Bx = static_cast<const S*>(f.f[kBx]);
  const S* By = static_cast<const S*>(f.f[kBy]);
  const S* Bz = static_cast<const S*>(f.f[kBz]);
  for (long long b = blockIdx.x; b < nblocks; b += gridDim.x) {
    int x, y, z;
    if (!cell_of(g, b, &x, &y, &z)) continue;
    const double dzBy = diff<RAD, false>(By, g, x, y, z, 2);
    const double dzBx = diff<RAD, false>(Bx, g, x, y, z, 2);
    const double dxBz = diff<RAD, false>(Bz, g, x, y, z, 0);
    const double dxBy = diff<RAD, false>(By, g, x, y, z, 0);
    double dyBz = 0.0, dyBx = 0.0;
    if constexpr (DIM == 3) {
      dyBz = diff<RAD, false>(Bz, g, x, y, z, 1);
      dyBx = diff<RAD, false>(Bx, g, x, y, z, 1);
    }
    const long long i = g.off + (static_cast<long long>(z) * g.ny + y) * g.nx + x;
    double ex = static_cast<double>(Ex[i]) + g.c2dt * (dyBz - dzBy);
    double ey = static_cast<double>(Ey[i]) + g.c2dt * (dzBx - dxBz);
    double ez = static_cast<double>(Ez[i]) + g.c2dt * (dxBy - dyBx);
    if constexpr (SRC) {
      ex -= g.dt_eps * static_cast<double>(static_cast<const S*>(f.f[kJx])[i]);
      ey -= g.dt_eps * static_cast<double>(static_cast<const S*>(f.f[kJy])[i]);
      ez -= g.dt_eps * static_cast<double>(static_cast<const S*>(f.f[kJz])[i]);
    }
    Ex[i] = static_cast<S>(ex);
    Ey[i] = static_cast<S>(ey);
    Ez[i] = static_cast<S>(ez);
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

// Staggered weights C_1..C_{p/2}: C_l = L_l(0) / x_l for the Lagrange basis on
// the nodes +-1/2, ..., +-(p-1)/2 (the derivative at 0; Sec. III.B).
std::vector<double> staggered_weights(int p) {
  std::vector<double> w;
  for (int l = 1; l <= p / 2; ++l) {
    const double xl = (2.0 * l - 1.0) / 2.0;
    double L0 = 1.0;
    for (int j = 0; j < p; ++j) {
      const double xn = (2.0 * j - p + 1.0) / 2.0;
      if (xn != xl) L0 *= (0.0 - xn) / (xl - xn);
    }
    w.push_back(L0 / xl);
  }
  return w;
}

template <typename S, int DIM, int RAD>
hipError_t launch_step_r(int scheme, bool src, const FdtdGeom& g, const FieldPtrs& f,
                         long long nblocks, int grid, hipStream_t s) {
  if (scheme == kCKC)
    hipLaunchKernelGGL((faraday_kernel<S, DIM, kCKC, 1>), dim3(grid), dim3(kRowBlock), 0, s, g, f,
                       nblocks);
  else
    hipLaunchKernelGGL((faraday_kernel<S, DIM, kYee, RAD>), dim3(grid), dim3(kRowBlock), 0, s, g,
                       f, nblocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (src)
    hipLaunchKernelGGL((ampere_kernel<S, DIM, RAD, true>), dim3(grid), dim3(kRowBlock), 0, s, g, f,
                       nblocks);
  else
    hipLaunchKernelGGL((ampere_kernel<S, DIM, RAD, false>), dim3(grid), dim3(kRowBlock), 0, s, g,
                       f, nblocks);
  return hipGetLastError();
}

template <typename S, int DIM>
hipError_t launch_step_s(int scheme, bool src, const FdtdGeom& g, const FieldPtrs& f,
                         long long nblocks, int grid, hipStream_t s) {
  // second order (Yee, CKC) with the radius fixed at compile time; order p
  // with the radius read from the geometry
  if (g.r == 1) return launch_step_r<S, DIM, 1>(scheme, src, g, f, nblocks, grid, s);
  return launch_step_r<S, DIM, 0>(scheme, src, g, f, nblocks, grid, s);
}

}  // namespace
}  // namespace psatd

using namespace psatd;

struct psatd_fdtd_s {
  psatd_config cfg{};
  int scheme = 0;
  int device = 0;
  int ndim = 2;
  size_t elem = 4;
  FdtdGeom geom{};
  long long nblocks = 0;
  int grid = 0;
};

extern "C" {

psatd_status psatd_fdtd_plan(const psatd_config* cfg, int32_t scheme,
                             const psatd_patch_desc* patch, int32_t device, psatd_fdtd_t* out) {
  try {
    if (!cfg || !patch || !out) return fail(PSATD_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (scheme != PSATD_FDTD_YEE && scheme != PSATD_FDTD_CKC)
      return fail(PSATD_ERR_INVALID_ARG, "scheme must be PSATD_FDTD_YEE or PSATD_FDTD_CKC");
    if (cfg->precision != PSATD_FP32 && cfg->precision != PSATD_FP64)
      return fail(PSATD_ERR_INVALID_ARG, "precision must be PSATD_FP32 or PSATD_FP64");
    if (cfg->source_mode != PSATD_VACUUM && cfg->source_mode != PSATD_SOURCES_J)
      return fail(PSATD_ERR_INVALID_ARG, "FDTD takes J only: source_mode VACUUM or SOURCES_J");
    if (cfg->path != PSATD_PATH_FUSED || cfg->flags != 0)
      return fail(PSATD_ERR_INVALID_ARG, "FDTD: path and flags must be 0");
    const int p = cfg->order == 0 ? 2 : cfg->order;
    if (p < 2 || p % 2 != 0 || p > 2 * kMaxRadius)
      return fail(PSATD_ERR_INVALID_ARG, "FDTD order must be 0, or even in [2, 32]");
    if (scheme == PSATD_FDTD_CKC && p != 2)
      return fail(PSATD_ERR_INVALID_ARG, "CKC is the second-order scheme (order 0 or 2)");
    if (!(cfg->c > 0.0) || !std::isfinite(cfg->c)) return fail(PSATD_ERR_INVALID_ARG, "c must be > 0");
    if (!(cfg->eps0 > 0.0) || !std::isfinite(cfg->eps0))
      return fail(PSATD_ERR_INVALID_ARG, "eps0 must be > 0");
    const psatd_patch_desc& d = *patch;
    if (d.ndim != 2 && d.ndim != 3) return fail(PSATD_ERR_INVALID_ARG, "ndim must be 2 or 3");
    if (d.ndim == 2 && d.n[1] != 1) return fail(PSATD_ERR_INVALID_ARG, "2D patches need n[1] = 1");
    if (scheme == PSATD_FDTD_CKC && d.ndim != 2)
      return fail(PSATD_ERR_UNSUPPORTED_SIZE, "CKC is implemented in 2D (x, z)");
    long long cells = 1;
    for (int a = 0; a < 3; ++a) {
      if (d.ndim == 2 && a == 1) continue;
      if (d.n[a] < std::max(2, p) || d.n[a] > (int64_t(1) << 24))
        return fail(PSATD_ERR_UNSUPPORTED_SIZE, "FDTD: every axis needs max(2, p) <= n <= 2^24");
      if (!(d.d[a] > 0.0) || !std::isfinite(d.d[a]))
        return fail(PSATD_ERR_INVALID_ARG, "grid spacing must be > 0");
      cells *= d.n[a];
    }
    if (cells > (int64_t(1) << 31)) return fail(PSATD_ERR_UNSUPPORTED_SIZE, "more than 2^31 cells");
    if (!(d.dt > 0.0) || !std::isfinite(d.dt)) return fail(PSATD_ERR_INVALID_ARG, "dt must be > 0");
    if (d.offset < 0) return fail(PSATD_ERR_INVALID_ARG, "offset must be >= 0");
    if (scheme == PSATD_FDTD_CKC && d.d[0] != d.d[2])
      return fail(PSATD_ERR_INVALID_ARG, "CKC needs dx = dz");

    const std::vector<double> w = staggered_weights(p);
    // Courant condition (Table 1): Yee / order p: c dt sqrt(sum_a (sum_l |C_l| / d_a)^2) <= 1;
    // CKC: c dt <= dx
    double courant;
    if (scheme == PSATD_FDTD_CKC) {
      courant = cfg->c * d.dt / d.d[0];
    } else {
      double sw = 0.0;
      for (double x : w) sw += std::fabs(x);
      double s2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        if (d.ndim == 2 && a == 1) continue;
        s2 += (sw / d.d[a]) * (sw / d.d[a]);
      }
      courant = cfg->c * d.dt * std::sqrt(s2);
    }
    if (courant > 1.0 + 1e-12)
      return fail(PSATD_ERR_INVALID_ARG,
                  "dt exceeds the scheme's Courant limit (ratio " + std::to_string(courant) + ")");

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
      return fail(PSATD_ERR_HIP, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(PSATD_ERR_INVALID_ARG, "device index out of range");

    psatd_fdtd_s* F = new psatd_fdtd_s();
    F->cfg = *cfg;
    F->scheme = scheme;
    F->device = device;
    F->ndim = d.ndim;
    F->elem = cfg->precision == PSATD_FP64 ? 8 : 4;
    FdtdGeom& g = F->geom;
    g.nx = static_cast<int>(d.n[0]);
    g.ny = d.ndim == 3 ? static_cast<int>(d.n[1]) : 1;
    g.nz = static_cast<int>(d.n[2]);
    g.r = p / 2;
    g.xchunks = (g.nx + kRowBlock - 1) / kRowBlock;
    g.off = d.offset;
    g.dt = d.dt;
    g.c2dt = cfg->c * cfg->c * d.dt;
    g.dt_eps = d.dt / cfg->eps0;
    for (int a = 0; a < 3; ++a) g.inv_d[a] = 1.0 / d.d[a];
    for (int l = 0; l < kMaxRadius; ++l) g.w[l] = l < g.r ? w[l] : 0.0;
    F->nblocks = static_cast<long long>(g.xchunks) * g.ny * g.nz;
    int ncu = 256;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        ncu <= 0)
      ncu = 256;
    F->grid = static_cast<int>(std::min<long long>(F->nblocks, 64LL * ncu));
    *out = F;
    return PSATD_OK;
  } catch (const std::exception& ex) {
    return fail(PSATD_ERR_OOM, std::string("host exception: ") + ex.what());
  }
}

psatd_status psatd_fdtd_push(psatd_fdtd_t F, const psatd_fields* fields, int32_t nsteps,
                             void* hip_stream) {
  if (!F) return fail(PSATD_ERR_INVALID_ARG, "fdtd is NULL");
  if (!fields) return fail(PSATD_ERR_INVALID_ARG, "fields is NULL");
  if (nsteps < 0) return fail(PSATD_ERR_INVALID_ARG, "nsteps must be >= 0");
  const bool src = F->cfg.source_mode == PSATD_SOURCES_J;
  if (nsteps > 1 && src)
    return fail(PSATD_ERR_INVALID_ARG, "with sources, push one step at a time (nsteps = 1)");
  FieldPtrs f{};
  for (int i = 0; i < 3; ++i) {
    if (!fields->E[i] || !fields->B[i])
      return fail(PSATD_ERR_INVALID_ARG, "E and B pointers must be non-NULL");
    f.f[kEx + i] = fields->E[i];
    f.f[kBx + i] = fields->B[i];
    if (src) {
      if (!fields->J[i]) return fail(PSATD_ERR_INVALID_ARG, "J pointers must be non-NULL with sources");
      f.f[kJx + i] = const_cast<void*>(fields->J[i]);
    }
  }
  for (int i = 0; i < (src ? 9 : 6); ++i)
    if (reinterpret_cast<uintptr_t>(f.f[i]) % F->elem != 0)
      return fail(PSATD_ERR_INVALID_ARG, "field buffers must be aligned to their element size");
  if (nsteps == 0) return PSATD_OK;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(F->device) != hipSuccess) return fail(PSATD_ERR_HIP, "hipSetDevice failed");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSuccess;
  for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
    if (F->elem == 8)
      e = F->ndim == 2 ? launch_step_s<double, 2>(F->scheme, src, F->geom, f, F->nblocks, F->grid, s)
                       : launch_step_s<double, 3>(F->scheme, src, F->geom, f, F->nblocks, F->grid, s);
    else
      e = F->ndim == 2 ? launch_step_s<float, 2>(F->scheme, src, F->geom, f, F->nblocks, F->grid, s)
                       : launch_step_s<float, 3>(F->scheme, src, F->geom, f, F->nblocks, F->grid, s);
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  if (e != hipSuccess) return hip_fail(e, "fdtd step");
  return PSATD_OK;
}

psatd_status psatd_fdtd_destroy(psatd_fdtd_t F) {
  delete F;
  return PSATD_OK;
}

}  // extern "C"
