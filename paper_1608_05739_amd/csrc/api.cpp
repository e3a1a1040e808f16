// Host side of the PSATD library: validation, planning, tables, launches and
// the C ABI declared in include/psatd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "fast2d.hpp"
#include "internal.hpp"
#include "kernels.hpp"
#include "psatd.h"
#include "update.hpp"
#include "wave2d.hpp"

using namespace psatd;

// Device-resident workspace of psatd_push_scratch: one copy per GPU the
// library runs on, held until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: every host use goes
// through the device address that hipGetSymbolAddress returned for the
// current device (scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[PSATD_SCRATCH_BYTES];

namespace {

// Device address of `scratch` per device, looked up once per device at the
// first plan created on it (with that device current).
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

psatd_status lookup_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return PSATD_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return PSATD_ERR_HIP;
  }
  g_scratch_ptr[device] = ptr;
  return PSATD_OK;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

thread_local std::string g_last_error;

psatd_status fail(psatd_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

bool even_2a3b(int64_t n) {
  if (n < 2 || n > 4096 || (n % 2) != 0) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

// Radix schedule of a complex length L = 2^a 3^b (L = 1: no stages), largest
// radices first, none above max_radix (16, 8 or 4).
std::vector<int> radix_plan(int L, int max_radix) {
  int a = 0, b = 0;
  while (L % 2 == 0) { L /= 2; ++a; }
  while (L % 3 == 0) { L /= 3; ++b; }
  std::vector<int> r;
  const int big = max_radix >= 16 ? 4 : (max_radix >= 8 ? 3 : 2);
  while (a >= big) { r.push_back(1 << big); a -= big; }
  if (a == 3) r.push_back(8);
  if (a == 2) r.push_back(4);
  if (a == 1) r.push_back(2);
  for (int i = 0; i < b; ++i) r.push_back(3);
  return r;
}

bool has_radix3(int L) { return L % 3 == 0; }

// Points a thread may own in a stage when at most maxpts fit its registers:
// radix-3 stages hold 3 * floor(maxpts / 3).
int points_per_thread(int L, int maxpts) { return has_radix3(L) ? 3 * (maxpts / 3) : maxpts; }

// Threads needed so that no thread holds more than ppt points in a stage.
int threads_for(int points, int L, int ppt) {
  const int per = points_per_thread(L, ppt);
  int t = (points + per - 1) / per;
  t = ((t + 63) / 64) * 64;
  return std::max(64, t);
}

// Staggered-grid Fornberg weights C_1..C_{p/2}: C_l = L_l(0) / x_l for the
// Lagrange basis on nodes +-1/2, ..., +-(p-1)/2 (derivative at 0).
std::vector<double> fornberg_staggered(int p) {
  std::vector<double> nodes;
  for (int j = 0; j < p; ++j) nodes.push_back((2.0 * j - p + 1) / 2.0);
  std::vector<double> w;
  for (int l = 1; l <= p / 2; ++l) {
    const double xj = (2.0 * l - 1) / 2.0;
    double L0 = 1.0;
    for (double xn : nodes)
      if (xn != xj) L0 *= (0.0 - xn) / (xj - xn);
    w.push_back(L0 / xj);
  }
  return w;
}

// Centered first-derivative weights a_1..a_{p/2} on the integer nodes
// -p/2..p/2: a_l = (-1)^(l+1) (m!)^2 / ((m-l)! (m+l)! l), m = p/2, written as
// a running product so that no factorial is formed.
std::vector<double> fornberg_centered(int p) {
  const int m = p / 2;
  std::vector<double> w;
  double ratio = 1.0;  // (m!)^2 / ((m-l)! (m+l)!)
  for (int l = 1; l <= m; ++l) {
    ratio *= static_cast<double>(m - l + 1) / static_cast<double>(m + l);
    w.push_back(((l % 2) ? 1.0 : -1.0) * ratio / l);
  }
  return w;
}

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

enum PassType { kLine = 0, kFused = 1, kUpdate = 2, kFastXFwd = 3, kFastZ = 4, kFastXInv = 5,
                kWaveZ = 6, kWaveX = 7 };

// One launch of a pass compiled per length (compile-time line passes, the
// wave-resident x passes): the work items of one line length.
struct SubLaunch {
  int L = 0;
  int first = 0;  // index of its first work item within the pass's list
  int nitems = 0;
  LaunchShape shape{};
  int full = 0;    // workgroups that give every wave its own work (0: nitems)
  int region = 0;  // wave z pass: double2 elements of LDS per wavefront
};

struct Pass {
  PassType type;
  int line_kind;
  const char* name;
  LaunchShape shape;
  WorkItem* d_items = nullptr;
  int nitems = 0;
  double bytes = 0.0;
  int mpt = 0;             // fused pass: modes per thread
  int ppt = 0;             // line passes: points per thread per FFT stage
  double tuned_ms = -1.0;  // mean launch time at the chosen grid (autotune), else -1
  int grid_choice = -1;    // the grid code given to set_grid by tuning, -1: the default grid
  bool tuning_applied = false;  // chosen by a tuning string (psatd_plan_tuned)
  std::vector<int> comps;  // line passes: the components they transform
  int lines = 0;           // line passes: lines per workgroup (the tile)
  int region = 0;          // wave-resident passes: double2 elements of LDS per wavefront
  bool ct = false;         // line passes: the compile-time-length kernels (ct_line_kernel),
  std::vector<SubLaunch> subs;  // ct line and wave x passes: one launch per length
};

// One pass's choice in a tuning string: pass type, compile-time flag, lines
// per workgroup, modes per thread, points per thread, grid (-1: the plan's
// default grid).
struct Choice {
  int type, ct, lines, mpt, ppt, grid;
};

const char* line_pass_name(int kind) {
  switch (kind) {
    case kXFwd: return "x_r2c_fwd";
    case kXInv: return "x_c2r_inv";
    case kYFwd: return "y_c2c_fwd";
    case kYInv: return "y_c2c_inv";
    case kZFwd: return "z_c2c_fwd";
    default: return "z_c2c_inv";
  }
}

}  // namespace

psatd_status set_last_error(psatd_status s, const std::string& msg) { return fail(s, msg); }

struct psatd_plan_s {
  psatd_config cfg{};
  int device = 0;
  int num_cus = 256;  // compute units of the device (persistent grids)
  int ndim = 2;
  int nin = 6;      // input components
  int src_form = 0; // SourceForm run by the generic kernels (PSATD forms or PSTD)
  size_t elem = 4;  // sizeof storage scalar
  std::vector<psatd_patch_desc> desc;
  std::vector<Choice> tuning;  // kernel choices to apply instead of autotuning (psatd_plan_tuned)
  std::vector<PatchDev> host_patches;
  PatchDev* d_patches = nullptr;
  void* d_tables = nullptr;
  void* d_items = nullptr;
  void* ws = nullptr;
  bool ws_owned = false;
  size_t ws_bytes = 0;
  std::vector<Pass> passes;
  std::vector<void*> extra_items;  // work lists of passes the autotuner re-tiled
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  // one graph per pass (graph plans), for psatd_push_profiled to time each
  // pass as the step's graph runs it
  std::vector<hipGraphExec_t> pass_exec;
  std::vector<hipGraph_t> pass_graphs;
  FieldPtrs* d_fieldtab = nullptr;  // field pointers the graph's kernels read (FieldPtrs::table)
  // graph capture: the launches of a pass with one launch per length run on
  // side streams forked from the capture stream and joined back, so that the
  // graph holds them as parallel branches (their tails overlap)
  std::vector<hipStream_t> side_streams;
  std::vector<hipEvent_t> fork_events;
  std::string info;
  // host-only planning (psatd_plan_describe): no device call is made, the
  // table addresses point into this host block and are never dereferenced
  bool dry = false;
  std::vector<char> dry_tables;
  // guard-cell decomposition: each patch's place in the global grid (empty
  // for ordinary plans); the x passes then read and write the global fields
  std::vector<GlobalMap> maps;
};

namespace {

void free_pass_graphs(psatd_plan_s* p) {
  for (hipGraphExec_t x : p->pass_exec)
    if (x) (void)hipGraphExecDestroy(x);
  for (hipGraph_t g : p->pass_graphs)
    if (g) (void)hipGraphDestroy(g);
  p->pass_exec.clear();
  p->pass_graphs.clear();
}

void free_plan_memory(psatd_plan_s* p) {
  free_pass_graphs(p);
  for (hipEvent_t ev : p->fork_events) (void)hipEventDestroy(ev);
  for (hipStream_t st : p->side_streams) (void)hipStreamDestroy(st);
  p->fork_events.clear();
  p->side_streams.clear();
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->d_patches) (void)hipFree(p->d_patches);
  if (p->d_tables) (void)hipFree(p->d_tables);
  if (p->d_items) (void)hipFree(p->d_items);
  if (p->d_fieldtab) (void)hipFree(p->d_fieldtab);
  for (void* x : p->extra_items) (void)hipFree(x);
  p->extra_items.clear();
  if (p->ws && p->ws_owned) (void)hipFree(p->ws);
  p->graph_exec = nullptr;
  p->graph = nullptr;
  p->capture_stream = nullptr;
  p->d_patches = nullptr;
  p->d_tables = nullptr;
  p->d_items = nullptr;
  p->d_fieldtab = nullptr;
  p->ws = nullptr;
}

psatd_status hip_fail(hipError_t e, const char* what) {
  // reset the runtime's last-error state, which the failed call set, so that
  // it does not surface again at the caller's next, unrelated launch check
  (void)hipGetLastError();
  return fail(e == hipErrorOutOfMemory ? PSATD_ERR_OOM : PSATD_ERR_HIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

// Largest |k| of one axis table: the exact lattice k with Nyquist -> 0, or the
// order-p wavevector of the staggered or centered stencil at those k.
double axis_kmax(int n, double d, const std::vector<double>& w, bool centered) {
  double best = 0.0;
  for (int j = 0; j <= n / 2; ++j) {
    if (n % 2 == 0 && j == n / 2) continue;  // Nyquist -> 0
    const double k = 2.0 * M_PI * j / (n * d);
    double kp = k;
    if (!w.empty()) {
      kp = 0.0;
      for (size_t l = 1; l <= w.size(); ++l)
        kp += w[l - 1] * (2.0 / d) *
              (centered ? std::sin(l * k * d) : std::sin((2.0 * l - 1.0) * k * d / 2.0));
    }
    best = std::max(best, std::fabs(kp));
  }
  return best;
}

psatd_status validate(const psatd_config* cfg, const psatd_patch_desc* patches, int32_t np) {
  if (!cfg) return fail(PSATD_ERR_INVALID_ARG, "cfg is NULL");
  if (!patches) return fail(PSATD_ERR_INVALID_ARG, "patches is NULL");
  if (np < 1) return fail(PSATD_ERR_INVALID_ARG, "npatches must be >= 1");
  if (cfg->precision != PSATD_FP32 && cfg->precision != PSATD_FP64)
    return fail(PSATD_ERR_INVALID_ARG, "precision must be PSATD_FP32 or PSATD_FP64");
  if (cfg->source_mode < PSATD_VACUUM || cfg->source_mode > PSATD_SOURCES_J)
    return fail(PSATD_ERR_INVALID_ARG, "unknown source_mode");
  if (cfg->path != PSATD_PATH_FUSED && cfg->path != PSATD_PATH_PLAIN)
    return fail(PSATD_ERR_INVALID_ARG, "unknown path");
  if (cfg->order < 0 || cfg->order % 2 != 0 || cfg->order > 512)
    return fail(PSATD_ERR_INVALID_ARG, "order must be 0 or an even number in [2, 512]");
  if (!(cfg->c > 0.0) || !std::isfinite(cfg->c)) return fail(PSATD_ERR_INVALID_ARG, "c must be > 0");
  if (!(cfg->eps0 > 0.0) || !std::isfinite(cfg->eps0))
    return fail(PSATD_ERR_INVALID_ARG, "eps0 must be > 0");
  if (cfg->flags & ~(PSATD_FLAG_AUTOTUNE | PSATD_FLAG_GRAPH | PSATD_FLAG_NO_WORKSPACE |
                     PSATD_FLAG_GENERIC_KERNELS | PSATD_FLAG_CENTERED_STENCIL | PSATD_FLAG_PSTD |
                     PSATD_FLAG_RADIX4_LINES))
    return fail(PSATD_ERR_INVALID_ARG, "unknown flag bits");
  if ((cfg->flags & PSATD_FLAG_PSTD) && cfg->source_mode == PSATD_SOURCES_RHO)
    return fail(PSATD_ERR_INVALID_ARG, "PSTD takes J only: source_mode VACUUM or SOURCES_J");
  const int ndim = patches[0].ndim;
  std::vector<std::pair<int64_t, int64_t>> ranges;
  for (int i = 0; i < np; ++i) {
    const psatd_patch_desc& d = patches[i];
    const std::string tag = "patch " + std::to_string(i) + ": ";
    if (d.ndim != 2 && d.ndim != 3) return fail(PSATD_ERR_INVALID_ARG, tag + "ndim must be 2 or 3");
    if (d.ndim != ndim)
      return fail(PSATD_ERR_INVALID_ARG, tag + "all patches of a plan must have the same ndim");
    if (d.ndim == 2 && d.n[1] != 1) return fail(PSATD_ERR_INVALID_ARG, tag + "2D patches need n[1] = 1");
    for (int a = 0; a < 3; ++a) {
      if (d.ndim == 2 && a == 1) continue;
      if (!even_2a3b(d.n[a]))
        return fail(PSATD_ERR_UNSUPPORTED_SIZE,
                    tag + "axis " + std::to_string(a) + " length " + std::to_string(d.n[a]) +
                        " is not an even 2^a 3^b in [2, 4096]");
      if (!(d.d[a] > 0.0) || !std::isfinite(d.d[a]))
        return fail(PSATD_ERR_INVALID_ARG, tag + "grid spacing must be > 0");
    }
    if (!(d.dt > 0.0) || !std::isfinite(d.dt)) return fail(PSATD_ERR_INVALID_ARG, tag + "dt must be > 0");
    if (d.offset < 0 || (d.offset % 2) != 0)
      return fail(PSATD_ERR_INVALID_ARG, tag + "offset must be a non-negative even element index");
    const int64_t cells = d.n[0] * (d.ndim == 3 ? d.n[1] : 1) * d.n[2];
    if (cells > (int64_t(1) << 31))
      return fail(PSATD_ERR_UNSUPPORTED_SIZE, tag + "more than 2^31 cells in one patch");
    ranges.emplace_back(d.offset, d.offset + cells);
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second)
      return fail(PSATD_ERR_INVALID_ARG, "patches overlap in the component buffers");
  if (cfg->flags & PSATD_FLAG_PSTD) {
    // the leapfrog is stable while c dt |k|max / 2 <= 1 (Table 1, PSTD row)
    const bool centered = (cfg->flags & PSATD_FLAG_CENTERED_STENCIL) != 0;
    std::vector<double> fw;
    if (cfg->order > 0) fw = centered ? fornberg_centered(cfg->order) : fornberg_staggered(cfg->order);
    for (int i = 0; i < np; ++i) {
      const psatd_patch_desc& d = patches[i];
      double k2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        if (d.ndim == 2 && a == 1) continue;
        const double k = axis_kmax(static_cast<int>(d.n[a]), d.d[a], fw, centered);
        k2 += k * k;
      }
      const double r = 0.5 * cfg->c * d.dt * std::sqrt(k2);
      if (r > 1.0 + 1e-12)
        return fail(PSATD_ERR_INVALID_ARG,
                    "patch " + std::to_string(i) + ": PSTD needs c dt |k|max / 2 <= 1, got " +
                        std::to_string(r) + " (Courant condition)");
    }
  }
  return PSATD_OK;
}

int inputs_for(int src) { return src == PSATD_VACUUM ? 6 : (src == PSATD_SOURCES_J ? 9 : 11); }


// Lines of a line pass for one patch and its FFT length.
void line_geometry(int kind, const PatchDev& P, int* nlines, int* L) {
  switch (kind) {
    case kXFwd:
    case kXInv:
      *nlines = P.nz * P.ny;
      *L = P.mx;
      break;
    case kYFwd:
    case kYInv:
      *nlines = P.mx * P.nz;
      *L = P.ny;
      break;
    default:
      *nlines = P.mx * P.ny;
      *L = P.nz;
      break;
  }
}

// Points per thread of the plan's generic line passes.
int line_ppt(const psatd_plan_s* plan) {
  return (plan->cfg.flags & PSATD_FLAG_RADIX4_LINES) ? 4 : kMaxPts;
}

// Lines of a line pass between which a tile of the compile-time kernels may
// not cross: the strided side of the x and y passes is placed by one division
// per tile (the tile map's A), so a tile stays inside one run of A lines.
int tile_period(int kind, const PatchDev& P) {
  if (kind == kXFwd || kind == kXInv) return P.ndim == 2 ? P.nz : P.ny;
  if (kind == kYFwd || kind == kYInv) return P.nz;
  return 0;
}

// The compile-time line kernels take every patch of the plan if each line
// length is compiled.
bool ct_line_eligible(int kind, const psatd_plan_s* plan) {
  // (PSATD_FLAG_RADIX4_LINES asks for the generic radix-4 schedule)
  if (plan->cfg.flags & (PSATD_FLAG_GENERIC_KERNELS | PSATD_FLAG_RADIX4_LINES)) return false;
  if (!plan->maps.empty() && (kind == kXFwd || kind == kXInv)) return false;  // (see GlobalMap)
  for (const PatchDev& P : plan->host_patches) {
    int nlines, L;
    line_geometry(kind, P, &nlines, &L);
    if (!ct_line_supported(L)) return false;
  }
  return true;
}

Pass make_ct_line_pass(int kind, const psatd_plan_s* plan, const std::vector<int>& comps,
                       std::vector<WorkItem>& items) {
  Pass ps;
  ps.type = kLine;
  ps.ct = true;
  ps.line_kind = kind;
  ps.ppt = 0;
  ps.name = line_pass_name(kind);
  size_t lds = 0;
  const size_t first = items.size();
  double bytes = 0.0;
  std::set<int> lengths;
  for (const PatchDev& P : plan->host_patches) {
    int nlines, L;
    line_geometry(kind, P, &nlines, &L);
    lengths.insert(L);
  }
  for (int Lc : lengths) {
    SubLaunch sub;
    sub.L = Lc;
    sub.first = static_cast<int>(items.size() - first);
    for (size_t pi = 0; pi < plan->host_patches.size(); ++pi) {
      const PatchDev& P = plan->host_patches[pi];
      int nlines, L;
      line_geometry(kind, P, &nlines, &L);
      if (L != Lc) continue;
      const int R = std::min(ct_line_tile(L), nlines);
      ps.lines = std::max(ps.lines, R);
      // tiles of R lines inside each run of A lines (the last one shorter
      // where R does not divide A)
      const int A = tile_period(kind, P) > 0 ? tile_period(kind, P) : nlines;
      for (int c : comps)
        for (int a0 = 0; a0 < nlines; a0 += A)
          for (int l = a0; l < std::min(a0 + A, nlines); l += R)
            items.push_back(
                WorkItem{static_cast<int>(pi), l, std::min(R, std::min(a0 + A, nlines) - l), c});
      const double cells = static_cast<double>(P.nx) * P.ny * P.nz;
      bytes += comps.size() * 2.0 * cells * plan->elem;
    }
    sub.nitems = static_cast<int>(items.size() - first) - sub.first;
    const size_t sub_lds = static_cast<size_t>(lpad_size(ct_line_tile(Lc) * Lc)) * sizeof(double2);
    sub.shape = LaunchShape{sub.nitems, kCtBlock, sub_lds};
    lds = std::max(lds, sub_lds);
    ps.subs.push_back(sub);
  }
  ps.nitems = static_cast<int>(items.size() - first);
  ps.shape = LaunchShape{ps.nitems, kCtBlock, lds};
  ps.bytes = bytes;
  ps.comps = comps;
  ps.d_items = reinterpret_cast<WorkItem*>(first);
  return ps;
}

// Wave-resident x passes (wavex.hip): 2D or 3D, FP32 storage, every row
// length compiled.  (PSATD_FLAG_RADIX4_LINES asks for the generic radix-4
// schedule.)
bool wave_x_eligible(const psatd_plan_s* plan) {
  const psatd_config& c = plan->cfg;
  if (c.flags & (PSATD_FLAG_GENERIC_KERNELS | PSATD_FLAG_RADIX4_LINES)) return false;
  if (!plan->maps.empty()) return false;  // (see GlobalMap)
  if (c.precision != PSATD_FP32) return false;
  for (const PatchDev& P : plan->host_patches)
    if (!wave2d::x_supported(P.mx)) return false;
  return true;
}

// Wave-resident y passes (wavex.hip): 3D, FP32 storage, every y length
// compiled.
bool wave_y_eligible(const psatd_plan_s* plan) {
  const psatd_config& c = plan->cfg;
  if (c.flags & (PSATD_FLAG_GENERIC_KERNELS | PSATD_FLAG_RADIX4_LINES)) return false;
  if (plan->ndim != 3 || c.precision != PSATD_FP32) return false;
  for (const PatchDev& P : plan->host_patches)
    if (!wave2d::x_supported(P.ny)) return false;
  return true;
}

bool wave_line_eligible(int kind, const psatd_plan_s* plan) {
  if (kind == kXFwd || kind == kXInv) return wave_x_eligible(plan);
  if (kind == kYFwd || kind == kYInv) return wave_y_eligible(plan);
  return false;
}

// Line length, lines, and the run of lines a tile stays in, of the
// wave-resident x and y passes: x rows (L = nx / 2) in runs of nz (2D) or ny
// (3D) rows; y lines (L = ny) l = kx nz + z in runs of nz.
void wave_line_geometry(int kind, const PatchDev& P, int* L, int* nlines, int* run) {
  if (kind == kYFwd || kind == kYInv) {
    *L = P.ny;
    *nlines = P.mx * P.nz;
    *run = P.nz;
  } else {
    *L = P.mx;
    *nlines = P.ny * P.nz;
    *run = P.ndim == 2 ? P.nz : P.ny;
  }
}

// Work items of up to x_rows_per_item(L) consecutive lines of one component
// inside one run (wave_line_geometry), one launch per line length.
Pass make_wave_x_pass(int kind, const psatd_plan_s* plan, const std::vector<int>& comps,
                      std::vector<WorkItem>& items) {
  Pass ps;
  ps.type = kWaveX;
  ps.line_kind = kind;
  ps.name = line_pass_name(kind);
  const size_t first = items.size();
  double bytes = 0.0;
  std::set<int> lengths;
  for (const PatchDev& P : plan->host_patches) {
    int L, nl, run;
    wave_line_geometry(kind, P, &L, &nl, &run);
    lengths.insert(L);
  }
  size_t lds = 0;
  int block = 64;
  for (int L : lengths) {
    SubLaunch sub;
    sub.L = L;
    sub.first = static_cast<int>(items.size() - first);
    const int T = wave2d::x_rows_per_item(L);
    for (size_t pi = 0; pi < plan->host_patches.size(); ++pi) {
      const PatchDev& P = plan->host_patches[pi];
      int Lp, nrows, A;
      wave_line_geometry(kind, P, &Lp, &nrows, &A);
      if (Lp != L) continue;
      for (int c : comps)
        for (int r0 = 0; r0 < nrows; r0 += A)
          for (int a = 0; a < A; a += T)
            items.push_back(WorkItem{static_cast<int>(pi), r0 + a, std::min(T, A - a), c});
      const double cells = static_cast<double>(P.nx) * P.ny * P.nz;
      bytes += comps.size() * 2.0 * cells * plan->elem;
    }
    sub.nitems = static_cast<int>(items.size() - first) - sub.first;
    const size_t sub_lds = wave2d::x_lds(L);
    sub.shape = LaunchShape{sub.nitems, wave2d::x_block(L), sub_lds};
    lds = std::max(lds, sub_lds);
    block = std::max(block, wave2d::x_block(L));
    ps.lines = std::max(ps.lines, T);
    ps.subs.push_back(sub);
  }
  ps.nitems = static_cast<int>(items.size() - first);
  ps.shape = LaunchShape{ps.nitems, block, lds};
  ps.bytes = bytes;
  ps.comps = comps;
  ps.d_items = reinterpret_cast<WorkItem*>(first);
  return ps;
}

// Launch grid of a pass: g workgroups, or for the passes launched per length
// g = 0 for every item in a workgroup of its own and g = k for at most k
// workgroups per CU in each launch.
void set_grid(const psatd_plan_s* plan, Pass& ps, int g) {
  if (ps.subs.empty()) {
    ps.shape.grid = g;
    return;
  }
  int total = 0;
  for (SubLaunch& sub : ps.subs) {
    const int full = sub.full > 0 ? sub.full : sub.nitems;
    sub.shape.grid = g == 0 ? full : std::min(full, g * plan->num_cus);
    total += sub.shape.grid;
  }
  ps.shape.grid = total;
}

Pass make_line_pass(int kind, const psatd_plan_s* plan, const std::vector<int>& comps,
                    std::vector<WorkItem>& items, int lines_override = 0, int ppt_override = 0) {
  int ppt = ppt_override > 0 ? ppt_override : line_ppt(plan);
  // a line longer than the threads of a workgroup can hold at this many
  // points each runs at the default points per thread
  for (const PatchDev& P : plan->host_patches) {
    int nlines, L;
    line_geometry(kind, P, &nlines, &L);
    if (L > kLineBlockMax * points_per_thread(L, ppt)) ppt = kMaxPts;
  }
  Pass ps;
  ps.type = kLine;
  ps.line_kind = kind;
  ps.ppt = ppt;
  ps.name = line_pass_name(kind);
  const bool transposing = kind == kXFwd || kind == kXInv || kind == kYFwd || kind == kYInv;
  const int want = lines_override > 0 ? lines_override : (plan->elem == 4 ? 8 : 4);
  int block = 64;
  size_t lds = 0;
  const size_t first = items.size();
  double bytes = 0.0;
  for (size_t pi = 0; pi < plan->host_patches.size(); ++pi) {
    const PatchDev& P = plan->host_patches[pi];
    int nlines, L;
    line_geometry(kind, P, &nlines, &L);
    int R;
    if (lines_override > 0) {
      R = lines_override;
    } else if (transposing) {
      R = want;
    } else {
      R = std::max(1, 4096 / L);
    }
    R = std::min(R, nlines);
    // LDS holds R lines (<= 8192 points, 136 KB padded) and 512 threads own
    // every stage's points
    const int max_pts = std::min(8192, kLineBlockMax * points_per_thread(L, ppt));
    R = std::max(1, std::min(R, max_pts / L));
    block = std::max(block, threads_for(R * L, L, ppt));
    lds = std::max(lds, static_cast<size_t>(lpad_size(R * L)) * sizeof(double2));
    ps.lines = std::max(ps.lines, R);
    for (int c : comps)
      for (int l = 0; l < nlines; l += R)
        items.push_back(WorkItem{static_cast<int>(pi), l, std::min(R, nlines - l), c});
    const double cells = static_cast<double>(P.nx) * P.ny * P.nz;
    bytes += comps.size() * 2.0 * cells * plan->elem;
  }
  ps.nitems = static_cast<int>(items.size() - first);
  ps.shape = LaunchShape{ps.nitems, std::min(block, kLineBlockMax), lds};
  ps.bytes = bytes;
  ps.comps = comps;
  ps.d_items = reinterpret_cast<WorkItem*>(first);  // offset, fixed up after upload
  return ps;
}

// Modes per thread the fused pass is compiled for, smallest first.  Fewer
// held inputs per thread leave room for more waves per SIMD; the larger
// choice takes z lines the smaller one cannot hold.
std::vector<int> fused_mpt_choices(int precision, int ndim) {
  if (precision == PSATD_FP32) return ndim == 2 ? std::vector<int>{2, 4, 8} : std::vector<int>{2, 4};
  return ndim == 2 ? std::vector<int>{2, 4} : std::vector<int>{2};
}

psatd_status make_fused_pass_mpt(const psatd_plan_s* plan, std::vector<WorkItem>& items, Pass* out,
                                 int lines_cap, int mpt) {
  Pass ps;
  ps.type = kFused;
  ps.name = "z_fused";
  ps.mpt = mpt;
  const int block = kFusedBlock;
  const int modes = block * ps.mpt;
  const int sl = fused_slots(ps.mpt);
  const size_t first = items.size();
  size_t lds = 0;
  double bytes = 0.0;
  int threads = 64;
  for (size_t pi = 0; pi < plan->host_patches.size(); ++pi) {
    const PatchDev& P = plan->host_patches[pi];
    const int nlines = P.mx * P.ny;
    if (P.nz > modes)
      return fail(PSATD_ERR_UNSUPPORTED_SIZE,
                  "fused path: nz = " + std::to_string(P.nz) + " exceeds " + std::to_string(modes) +
                      " modes per workgroup at this precision; use PSATD_PATH_PLAIN");
    // lines per workgroup: all modes must fit T * MPT, and every FFT stage over
    // the fused_slots(mpt) tiles transformed together must leave at most
    // kMaxPtsFused points per thread
    const int cap = std::min(modes, block * points_per_thread(P.nz, kMaxPtsFused) / sl);
    if (P.nz > cap)
      return fail(PSATD_ERR_UNSUPPORTED_SIZE,
                  "fused path: nz = " + std::to_string(P.nz) + " does not fit one workgroup");
    int W = std::max(1, std::min(nlines, cap / P.nz));
    if (lines_cap > 0) W = std::min(W, lines_cap);
    // the block shrinks to the threads the tile needs (at most mpt modes each,
    // and at most ppt points of the sl stacked tiles each in a stage): small
    // tiles run as several workgroups per CU, whose barriers do not stall
    // each other
    const int ppt = points_per_thread(P.nz, kMaxPtsFused);
    const int t_modes = (W * P.nz + ps.mpt - 1) / ps.mpt;      // W nz <= T mpt
    const int t_stage = (sl * W * P.nz + ppt - 1) / ppt;       // sl W nz <= T ppt
    const int need = (std::max(t_modes, t_stage) + 63) / 64 * 64;
    threads = std::max(threads, std::min(block, need));
    lds = std::max(lds, static_cast<size_t>(lpad_size(sl * W * P.nz)) * sizeof(double2));
    ps.lines = std::max(ps.lines, W);
    for (int l = 0; l < nlines; l += W)
      items.push_back(WorkItem{static_cast<int>(pi), l, std::min(W, nlines - l), -1});
    const double cells = static_cast<double>(P.nx) * P.ny * P.nz;
    bytes += (plan->nin + 6) * cells * plan->elem;
  }
  ps.nitems = static_cast<int>(items.size() - first);
  ps.shape = LaunchShape{ps.nitems, threads, lds};
  ps.bytes = bytes;
  ps.d_items = reinterpret_cast<WorkItem*>(first);
  *out = ps;
  return PSATD_OK;
}

// The fused pass at `mpt` modes per thread, or (mpt = 0) at the smallest
// compiled choice whose workgroups hold every patch's z lines.
psatd_status make_fused_pass(const psatd_plan_s* plan, std::vector<WorkItem>& items, Pass* out,
                             int lines_cap = 0, int mpt = 0) {
  if (mpt > 0) return make_fused_pass_mpt(plan, items, out, lines_cap, mpt);
  psatd_status st = PSATD_ERR_UNSUPPORTED_SIZE;
  const size_t n0 = items.size();
  const std::string before = g_last_error;  // a choice that does not fit is no error
  for (int m : fused_mpt_choices(plan->cfg.precision, plan->ndim)) {
    items.resize(n0);
    st = make_fused_pass_mpt(plan, items, out, lines_cap, m);
    if (st == PSATD_OK) {
      g_last_error = before;
      return st;
    }
  }
  return st;
}

// Does the fused pass hold every patch's z lines at some compiled choice?
// (Longer lines run as the plain z passes instead: transform, update,
// transform.)  Leaves items and the last error as they were.
bool fused_fits(const psatd_plan_s* plan, std::vector<WorkItem>& items) {
  const size_t n0 = items.size();
  const std::string before = g_last_error;
  Pass probe;
  const bool ok = make_fused_pass(plan, items, &probe) == PSATD_OK;
  items.resize(n0);
  g_last_error = before;
  return ok;
}

Pass make_update_pass(const psatd_plan_s* plan, std::vector<WorkItem>& items) {
  Pass ps;
  ps.type = kUpdate;
  ps.name = "update";
  const size_t first = items.size();
  const int chunk = 4096;
  double bytes = 0.0;
  for (size_t pi = 0; pi < plan->host_patches.size(); ++pi) {
    const PatchDev& P = plan->host_patches[pi];
    const long long modes = P.comp_stride;
    for (long long m = 0; m < modes; m += chunk)
      items.push_back(WorkItem{static_cast<int>(pi), static_cast<int>(m),
                               static_cast<int>(std::min<long long>(chunk, modes - m)), -1});
    const double cells = static_cast<double>(P.nx) * P.ny * P.nz;
    bytes += (plan->nin + 6) * cells * plan->elem;
  }
  ps.nitems = static_cast<int>(items.size() - first);
  ps.shape = LaunchShape{ps.nitems, 256, 0};
  ps.bytes = bytes;
  ps.d_items = reinterpret_cast<WorkItem*>(first);
  return ps;
}

// Host check of the invariants every kernel relies on, run once per plan
// before anything can be launched: work items stay inside their patch, LDS
// holds every item, and in each FFT stage the block owns all butterflies
// within the per-thread register budget.
psatd_status verify_pass(const psatd_plan_s* plan, const Pass& ps, const WorkItem* items) {
  const int maxpts = ps.type == kFused ? kMaxPtsFused : ps.ppt;
  if (ps.type == kLine && !ps.ct && !line_ppt_supported(ps.ppt))
    return fail(PSATD_ERR_STATE, std::string(ps.name) + ": points per thread not compiled");
  for (int i = 0; i < ps.nitems; ++i) {
    const WorkItem& w = items[i];
    if (w.patch < 0 || w.patch >= static_cast<int>(plan->host_patches.size()))
      return fail(PSATD_ERR_STATE, std::string(ps.name) + ": bad patch index");
    const PatchDev& P = plan->host_patches[w.patch];
    if (ps.type == kFastXFwd || ps.type == kFastXInv || ps.type == kFastZ) {
      if (P.nx != fast2d::kNX || P.nz != fast2d::kNZfast || P.ndim != 2)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": patch shape not specialized");
      const int lim = ps.type == kFastZ ? P.mx : fast2d::kTilesZ;
      if (w.first < 0 || w.first >= lim || w.count != 1)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": item out of range");
      if (ps.type != kFastZ && (w.comp < 0 || w.comp >= plan->nin))
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": bad component");
      if (ps.shape.block != fast2d::kBlock)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": bad block size");
      continue;
    }
    if (ps.type == kWaveX) {
      int L, nrows, A;
      wave_line_geometry(ps.line_kind, P, &L, &nrows, &A);
      if (!wave2d::x_supported(L) || ((ps.line_kind == kYFwd || ps.line_kind == kYInv) && P.ndim != 3))
        return fail(PSATD_ERR_STATE, std::string(ps.name) + " (wave): line length not compiled");
      if (w.comp < 0 || w.comp >= plan->nin)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + " (wave): bad component");
      if (w.count < 1 || w.first < 0 || w.first + w.count > nrows ||
          w.count > wave2d::x_rows_per_item(L) || w.first / A != (w.first + w.count - 1) / A)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + " (wave): item out of range");
      bool in_sub = false;
      for (const SubLaunch& sub : ps.subs)
        in_sub = in_sub ||
                 (i >= sub.first && i < sub.first + sub.nitems && sub.L == L &&
                  sub.shape.block == wave2d::x_block(L) && sub.shape.lds_bytes >= wave2d::x_lds(L));
      if (!in_sub)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + " (wave): item outside its length's launch");
      continue;
    }
    if (ps.type == kWaveZ) {
      if (P.ndim == 2 ? !wave2d::z_supported(P.nz) : !wave2d::z3_supported(P.nz))
        return fail(PSATD_ERR_STATE, "z_fused (wave): z length not compiled");
      if (w.count < 1 || w.first < 0 || w.first + w.count > P.mx * P.ny ||
          w.count > wave2d::z_lines_per_item(P.nz))
        return fail(PSATD_ERR_STATE, "z_fused (wave): item out of range");
      if (P.ndim == 2) {
        // each item in the launch of its z length, whose LDS holds a region
        // of that length per wavefront
        bool in_sub = false;
        for (const SubLaunch& sub : ps.subs)
          in_sub = in_sub ||
                   (i >= sub.first && i < sub.first + sub.nitems && sub.L == P.nz &&
                    sub.region >= wave2d::z_region(P.nz) && sub.shape.block == wave2d::kBlock &&
                    static_cast<size_t>(sub.region) * wave2d::kWavesPerBlock * sizeof(double2) <=
                        sub.shape.lds_bytes);
        if (!in_sub) return fail(PSATD_ERR_STATE, "z_fused (wave): item outside its length's launch");
        continue;
      }
      if ((P.ndim == 2 ? wave2d::z_region(P.nz) : wave2d::z3_region(P.nz)) > ps.region ||
          static_cast<size_t>(ps.region) * wave2d::kWavesPerBlock * sizeof(double2) > ps.shape.lds_bytes)
        return fail(PSATD_ERR_STATE, "z_fused (wave): LDS region too small");
      if (ps.shape.block != wave2d::kBlock)
        return fail(PSATD_ERR_STATE, "z_fused (wave): bad block size");
      continue;
    }
    if (w.count < 1 || w.first < 0) return fail(PSATD_ERR_STATE, std::string(ps.name) + ": empty item");
    if (ps.type == kUpdate) {
      if (static_cast<long long>(w.first) + w.count > P.comp_stride)
        return fail(PSATD_ERR_STATE, "update: item past the spectrum");
      continue;
    }
    if (ps.type == kLine && ps.ct) {
      int nlines, L;
      line_geometry(ps.line_kind, P, &nlines, &L);
      bool in_sub = false;
      for (const SubLaunch& sub : ps.subs)
        in_sub = in_sub || (i >= sub.first && i < sub.first + sub.nitems && sub.L == L &&
                            sub.shape.lds_bytes >= static_cast<size_t>(lpad_size(ct_line_tile(L) * L)) *
                                                       sizeof(double2));
      if (!in_sub) return fail(PSATD_ERR_STATE, std::string(ps.name) + ": item outside its length's launch");
      if (!ct_line_supported(L)) return fail(PSATD_ERR_STATE, std::string(ps.name) + ": length not compiled");
      if (w.comp < 0 || w.comp >= plan->nin)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": bad component");
      if (w.count < 1 || w.first < 0 || w.first + w.count > nlines || w.count > ct_line_tile(L))
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": item out of range");
      const int A = tile_period(ps.line_kind, P);
      if (A > 0 && w.first / A != (w.first + w.count - 1) / A)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": tile straddles the tile map");
      if (static_cast<size_t>(lpad_size(ct_line_tile(L) * L)) * sizeof(double2) > ps.shape.lds_bytes)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": item exceeds LDS");
      if (ps.shape.block != kCtBlock) return fail(PSATD_ERR_STATE, std::string(ps.name) + ": bad block size");
      continue;
    }
    int nlines, L;
    const FFTPlanDev* f;
    if (ps.type == kFused) {
      nlines = P.mx * P.ny;
      L = P.nz;
      f = &P.fz;
    } else {
      line_geometry(ps.line_kind, P, &nlines, &L);
      f = (ps.line_kind == kXFwd || ps.line_kind == kXInv)   ? &P.fx
          : (ps.line_kind == kYFwd || ps.line_kind == kYInv) ? &P.fy
                                                             : &P.fz;
      if (w.comp < 0 || w.comp >= plan->nin)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": bad component");
    }
    if (w.first + w.count > nlines)
      return fail(PSATD_ERR_STATE, std::string(ps.name) + ": item past the last line");
    // points of one FFT: a fused pass transforms fused_slots tiles together
    const long long pts =
        static_cast<long long>(w.count) * L * (ps.type == kFused ? fused_slots(ps.mpt) : 1);
    if (static_cast<long long>(lpad_size(static_cast<int>(pts))) * static_cast<long long>(sizeof(double2)) >
        static_cast<long long>(ps.shape.lds_bytes))
      return fail(PSATD_ERR_STATE, std::string(ps.name) + ": item exceeds LDS");
    if (ps.type == kLine && pts > static_cast<long long>(ps.shape.block) * ps.ppt)
      return fail(PSATD_ERR_STATE, std::string(ps.name) + ": tile exceeds the loads a thread holds");
    if (ps.type == kFused &&
        static_cast<long long>(w.count) * L > static_cast<long long>(ps.shape.block) * ps.mpt)
      return fail(PSATD_ERR_STATE, "z_fused: modes exceed registers");
    // the stages the kernel runs: the plan's radices, or at 4 points per
    // thread the radix-4 schedule it derives from the length
    std::vector<int> radices(f->radix, f->radix + f->nstages);
    if (ps.type == kLine && ps.ppt == 4) radices = radix_plan(L, 4);
    for (int r : radices) {
      if (r > maxpts) return fail(PSATD_ERR_STATE, std::string(ps.name) + ": radix too large");
      const long long bpt = maxpts / r;
      if (pts / r > bpt * ps.shape.block)
        return fail(PSATD_ERR_STATE, std::string(ps.name) + ": too few threads for a stage");
    }
  }
  if (ps.shape.lds_bytes > 160 * 1024) return fail(PSATD_ERR_STATE, std::string(ps.name) + ": LDS > 160 KB");
  if (ps.shape.block < 64 || ps.shape.block > 1024)
    return fail(PSATD_ERR_STATE, std::string(ps.name) + ": bad block size");
  return PSATD_OK;
}

// Shape-specialized 2D passes (fast2d.hip): every patch nx = nz = 4096,
// FP32 storage, fused path.
bool fast2d_eligible(const psatd_plan_s* plan) {
  const psatd_config& c = plan->cfg;
  if (c.flags & (PSATD_FLAG_GENERIC_KERNELS | PSATD_FLAG_PSTD)) return false;
  if (!plan->maps.empty()) return false;  // only the generic x passes read through a map
  if (plan->ndim != 2 || c.precision != PSATD_FP32 || c.path != PSATD_PATH_FUSED) return false;
  for (const PatchDev& P : plan->host_patches)
    if (P.nx != fast2d::kNX || P.nz != fast2d::kNZfast) return false;
  return true;
}

Pass make_fast_pass(PassType type, const psatd_plan_s* plan, const std::vector<int>& comps,
                    std::vector<WorkItem>& items) {
  Pass ps;
  ps.type = type;
  ps.line_kind = -1;
  ps.name = type == kFastXFwd ? "x_r2c_fwd" : (type == kFastXInv ? "x_c2r_inv" : "z_fused");
  const size_t first = items.size();
  double bytes = 0.0;
  for (size_t pi = 0; pi < plan->host_patches.size(); ++pi) {
    const PatchDev& P = plan->host_patches[pi];
    const double cells = static_cast<double>(P.nx) * P.ny * P.nz;
    if (type == kFastZ) {
      for (int kx = 0; kx < P.mx; ++kx) items.push_back(WorkItem{static_cast<int>(pi), kx, 1, -1});
      bytes += (plan->nin + 6) * cells * plan->elem;
    } else {
      for (int c : comps)
        for (int z1 = 0; z1 < fast2d::kTilesZ; ++z1)
          items.push_back(WorkItem{static_cast<int>(pi), z1, 1, c});
      bytes += comps.size() * 2.0 * cells * plan->elem;
    }
  }
  ps.nitems = static_cast<int>(items.size() - first);
  const size_t lds = type == kFastZ      ? fast2d::z_lds_bytes()
                     : type == kFastXFwd ? fast2d::x_fwd_lds_bytes()
                                         : fast2d::x_inv_lds_bytes();
  // Each kernel fits one workgroup per CU (LDS) and loops over its items when
  // the grid is smaller than the item count.  Default grids as measured at
  // 4096x4096: the z pass walks its columns (prefetching the next one); the x
  // passes do better with one workgroup per item, handed out by the hardware
  // as CUs free up.  PSATD_FLAG_AUTOTUNE re-measures.
  const int grid = type == kFastZ ? std::min(ps.nitems, plan->num_cus) : ps.nitems;
  ps.shape = LaunchShape{grid, fast2d::kBlock, lds};
  ps.bytes = bytes;
  ps.mpt = type == kFastZ ? 8 : 0;
  ps.d_items = reinterpret_cast<WorkItem*>(first);
  return ps;
}

// Wave-resident fused z pass: 2D (wave2d.hip) in the vacuum forms, 3D
// (wave3d.hip) in the PSATD forms; FP32 storage, every z length compiled.
bool wave_z_eligible(const psatd_plan_s* plan) {
  const psatd_config& c = plan->cfg;
  if (c.flags & PSATD_FLAG_GENERIC_KERNELS) return false;
  if (c.precision != PSATD_FP32 || c.path != PSATD_PATH_FUSED) return false;
  if (plan->ndim == 2) {
    if (plan->src_form != kVacuum && plan->src_form != kPstdVacuum) return false;
    for (const PatchDev& P : plan->host_patches)
      if (!wave2d::z_supported(P.nz)) return false;
    return true;
  }
  if (src_is_pstd(plan->src_form)) return false;
  for (const PatchDev& P : plan->host_patches)
    if (!wave2d::z3_supported(P.nz)) return false;
  return true;
}

// One work item per wavefront: the z lines (kx columns) one wave holds.  In
// 2D, one launch per z length: lengths at 8 points per lane run one set per
// wavefront (two wavefronts per item), the others both sets.
Pass make_wave_z_pass(const psatd_plan_s* plan, std::vector<WorkItem>& items) {
  Pass ps;
  ps.type = kWaveZ;
  ps.name = "z_fused";
  const size_t first = items.size();
  double bytes = 0.0;
  if (plan->ndim == 2) {
    std::set<int> lengths;
    for (const PatchDev& P : plan->host_patches) lengths.insert(P.nz);
    size_t lds = 0;
    for (int L : lengths) {
      SubLaunch sub;
      sub.L = L;
      sub.first = static_cast<int>(items.size() - first);
      const int G = wave2d::z_lines_per_item(L);
      for (size_t pi = 0; pi < plan->host_patches.size(); ++pi) {
        const PatchDev& P = plan->host_patches[pi];
        if (P.nz != L) continue;
        const int nlines = P.mx * P.ny;
        for (int l = 0; l < nlines; l += G)
          items.push_back(WorkItem{static_cast<int>(pi), l, std::min(G, nlines - l), -1});
        const double cells = static_cast<double>(P.nx) * P.ny * P.nz;
        bytes += (plan->nin + 6) * cells * plan->elem;
      }
      sub.nitems = static_cast<int>(items.size() - first) - sub.first;
      sub.region = wave2d::z_region(L);
      const int waves = wave2d::z_set_supported(L) ? 2 * sub.nitems : sub.nitems;
      sub.full = (waves + wave2d::kWavesPerBlock - 1) / wave2d::kWavesPerBlock;
      const size_t sub_lds = static_cast<size_t>(sub.region) * wave2d::kWavesPerBlock * sizeof(double2);
      sub.shape = LaunchShape{sub.full, wave2d::kBlock, sub_lds};
      lds = std::max(lds, sub_lds);
      ps.region = std::max(ps.region, sub.region);
      ps.lines = std::max(ps.lines, G);
      ps.subs.push_back(sub);
    }
    ps.nitems = static_cast<int>(items.size() - first);
    int total = 0;
    for (const SubLaunch& sub : ps.subs) total += sub.shape.grid;
    ps.shape = LaunchShape{total, wave2d::kBlock, lds};
    ps.bytes = bytes;
    ps.d_items = reinterpret_cast<WorkItem*>(first);
    return ps;
  }
  for (size_t pi = 0; pi < plan->host_patches.size(); ++pi) {
    const PatchDev& P = plan->host_patches[pi];
    const int G = wave2d::z_lines_per_item(P.nz);
    const int nlines = P.mx * P.ny;
    for (int l = 0; l < nlines; l += G)
      items.push_back(WorkItem{static_cast<int>(pi), l, std::min(G, nlines - l), -1});
    ps.region = std::max(ps.region, P.ndim == 2 ? wave2d::z_region(P.nz) : wave2d::z3_region(P.nz));
    ps.lines = std::max(ps.lines, G);
    const double cells = static_cast<double>(P.nx) * P.ny * P.nz;
    bytes += (plan->nin + 6) * cells * plan->elem;
  }
  ps.nitems = static_cast<int>(items.size() - first);
  const int blocks = (ps.nitems + wave2d::kWavesPerBlock - 1) / wave2d::kWavesPerBlock;
  ps.shape = LaunchShape{blocks, wave2d::kBlock,
                         static_cast<size_t>(ps.region) * wave2d::kWavesPerBlock * sizeof(double2)};
  ps.bytes = bytes;
  ps.d_items = reinterpret_cast<WorkItem*>(first);
  return ps;
}

// Streams and events that let the launches of a per-length pass run as
// parallel branches of a captured graph: ev[0] forks, ev[1 + i] joins launch i.
struct Fork {
  const hipStream_t* side = nullptr;
  const hipEvent_t* ev = nullptr;
};

// Run launch(sub, stream) for every per-length launch of a pass: in order on
// s, or (fork given, several launches) each on its own side stream that
// waits for s and that s waits for.
template <typename F>
hipError_t for_subs(const Pass& ps, hipStream_t s, const Fork* fork, F&& launch) {
  if (!fork || ps.subs.size() < 2) {
    for (const SubLaunch& sub : ps.subs) {
      const hipError_t e = launch(sub, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipError_t e = hipEventRecord(fork->ev[0], s);
  for (size_t i = 0; i < ps.subs.size() && e == hipSuccess; ++i) {
    hipStream_t t = fork->side[i];
    e = hipStreamWaitEvent(t, fork->ev[0], 0);
    if (e == hipSuccess) e = launch(ps.subs[i], t);
    if (e == hipSuccess) e = hipEventRecord(fork->ev[1 + i], t);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, fork->ev[1 + i], 0);
  }
  return e;
}

psatd_status enqueue_pass(const psatd_plan_s* plan, const Pass& ps, const FieldPtrs& f,
                          hipStream_t s, void* ws, const Fork* fork = nullptr) {
  hipError_t e;
  const Physics ph{plan->cfg.c, plan->cfg.eps0};
  switch (ps.type) {
    case kLine:
      if (ps.ct) {
        e = for_subs(ps, s, fork, [&](const SubLaunch& sub, hipStream_t t) {
          return launch_ct_line(ps.line_kind, plan->cfg.precision, sub.L, sub.shape, t,
                                plan->d_patches, ps.d_items + sub.first, sub.nitems, f, ws);
        });
      } else {
        e = launch_line_pass(ps.line_kind, plan->cfg.precision, ps.ppt, ps.shape, s,
                             plan->d_patches, ps.d_items, ps.nitems, f, ws);
      }
      break;
    case kFused:
      e = launch_fused_z(plan->cfg.precision, plan->ndim, plan->src_form, ps.mpt, ps.shape,
                         s, plan->d_patches, ps.d_items, ps.nitems, ws, ph);
      break;
    case kUpdate:
      e = launch_update(plan->cfg.precision, plan->src_form, ps.shape, s, plan->d_patches,
                        ps.d_items, ps.nitems, ws, ph);
      break;
    case kWaveX:
      e = for_subs(ps, s, fork, [&](const SubLaunch& sub, hipStream_t t) {
        return wave2d::launch_x(ps.line_kind, sub.L, sub.shape, t, plan->d_patches,
                                ps.d_items + sub.first, sub.nitems, f, ws);
      });
      break;
    case kWaveZ:
      if (plan->ndim == 2) {
        e = for_subs(ps, s, fork, [&](const SubLaunch& sub, hipStream_t t) {
          return wave2d::z_set_supported(sub.L)
                     ? wave2d::launch_z_set(plan->src_form, sub.L, sub.shape, t, plan->d_patches,
                                            ps.d_items + sub.first, sub.nitems, ws, ph, sub.region)
                     : wave2d::launch_z_fused(plan->src_form, sub.shape, t, plan->d_patches,
                                              ps.d_items + sub.first, sub.nitems, ws, ph, sub.region);
        });
      } else {
        e = wave2d::launch_z3_fused(plan->src_form, ps.shape, s, plan->d_patches, ps.d_items,
                                    ps.nitems, ws, ph, ps.region);
      }
      break;
    case kFastXFwd:
      e = fast2d::launch_x_fwd(ps.shape, s, plan->d_patches, ps.d_items, ps.nitems, f, ws);
      break;
    case kFastXInv:
      e = fast2d::launch_x_inv(ps.shape, s, plan->d_patches, ps.d_items, ps.nitems, f, ws);
      break;
    default:
      e = fast2d::launch_z_fused(plan->cfg.source_mode, plan->cfg.order == 0, ps.shape, s,
                                 plan->d_patches, ps.d_items, ps.nitems, ws, ph);
      break;
  }
  if (e != hipSuccess) return hip_fail(e, ps.name);
  return PSATD_OK;
}

psatd_status check_fields(const psatd_plan_s* plan, const psatd_fields* f, FieldPtrs* out) {
  if (!f) return fail(PSATD_ERR_INVALID_ARG, "fields is NULL");
  for (int i = 0; i < 3; ++i) {
    if (!f->E[i] || !f->B[i]) return fail(PSATD_ERR_INVALID_ARG, "E and B pointers must be non-NULL");
  }
  const int src = plan->cfg.source_mode;
  if (src != PSATD_VACUUM) {
    for (int i = 0; i < 3; ++i)
      if (!f->J[i]) return fail(PSATD_ERR_INVALID_ARG, "J pointers must be non-NULL with sources");
  }
  if (src == PSATD_SOURCES_RHO && (!f->rho_old || !f->rho_new))
    return fail(PSATD_ERR_INVALID_ARG, "rho_old and rho_new must be non-NULL in the rho form");
  const size_t align = plan->elem * 2;
  auto misaligned = [&](const void* p) { return (reinterpret_cast<uintptr_t>(p) % align) != 0; };
  FieldPtrs fp{};
  for (int i = 0; i < 3; ++i) {
    fp.f[kEx + i] = f->E[i];
    fp.f[kBx + i] = f->B[i];
    fp.f[kJx + i] = const_cast<void*>(f->J[i]);
  }
  fp.f[kRhoOld] = const_cast<void*>(f->rho_old);
  fp.f[kRhoNew] = const_cast<void*>(f->rho_new);
  for (int i = 0; i < plan->nin; ++i)
    if (misaligned(fp.f[i]))
      return fail(PSATD_ERR_INVALID_ARG, "field buffers must be aligned to two elements");
  *out = fp;
  return PSATD_OK;
}

psatd_status enqueue_step(const psatd_plan_s* plan, const FieldPtrs& fp, hipStream_t s, void* ws,
                          const std::vector<Fork>* forks = nullptr) {
  for (size_t i = 0; i < plan->passes.size(); ++i) {
    const Fork* fk = (forks && (*forks)[i].side) ? &(*forks)[i] : nullptr;
    psatd_status st = enqueue_pass(plan, plan->passes[i], fp, s, ws, fk);
    if (st != PSATD_OK) return st;
  }
  return PSATD_OK;
}

// The fork of each pass launched per length, on the plan's side streams and
// events (made with the graph; no fork where there are none).
std::vector<Fork> plan_forks(const psatd_plan_s* plan) {
  std::vector<Fork> forks(plan->passes.size());
  size_t need = 0;
  for (const Pass& ps : plan->passes)
    if (ps.subs.size() > 1) need += 1 + ps.subs.size();
  if (need == 0 || plan->fork_events.size() < need) return forks;
  for (size_t i = 0, k = 0; i < plan->passes.size(); ++i)
    if (plan->passes[i].subs.size() > 1) {
      if (plan->side_streams.size() < plan->passes[i].subs.size()) return std::vector<Fork>(plan->passes.size());
      forks[i].side = plan->side_streams.data();
      forks[i].ev = plan->fork_events.data() + k;
      k += 1 + plan->passes[i].subs.size();
    }
  return forks;
}

// PSATD_FLAG_GRAPH: capture one step into a graph whose kernels read the
// field pointers from the plan's device table, and instantiate it.  Runs at
// plan time and in psatd_set_workspace (the step needs the workspace), so
// that a push only writes the table and launches the graph: no allocation,
// no capture, for any fields.
psatd_status build_graph(psatd_plan_s* plan) {
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  plan->graph_exec = nullptr;
  plan->graph = nullptr;
  free_pass_graphs(plan);
  if (!plan->ws) return PSATD_OK;  // built when the workspace arrives
  hipError_t e = hipSuccess;
  if (!plan->d_fieldtab) {
    e = hipMalloc(&plan->d_fieldtab, sizeof(FieldPtrs));
    if (e != hipSuccess) {
      plan->d_fieldtab = nullptr;
      return hip_fail(e, "hipMalloc(field table)");
    }
    e = hipMemset(plan->d_fieldtab, 0, sizeof(FieldPtrs));
    if (e != hipSuccess) return hip_fail(e, "hipMemset(field table)");
  }
  if (!plan->capture_stream) {
    e = hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      plan->capture_stream = nullptr;
      return hip_fail(e, "capture stream");
    }
  }
  // side streams and fork/join events for the per-length passes
  size_t nside = 0, nev = 0;
  for (const Pass& ps : plan->passes)
    if (ps.subs.size() > 1) {
      nside = std::max(nside, ps.subs.size());
      nev += 1 + ps.subs.size();
    }
  while (plan->side_streams.size() < nside) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "side stream");
    plan->side_streams.push_back(st);
  }
  while (plan->fork_events.size() < nev) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "fork event");
    plan->fork_events.push_back(ev);
  }
  const std::vector<Fork> forks = plan_forks(plan);
  FieldPtrs fp{};
  fp.table = plan->d_fieldtab;
  e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  psatd_status cs = enqueue_step(plan, fp, plan->capture_stream, plan->ws, &forks);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(plan->capture_stream, &graph);
  if (cs != PSATD_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return cs;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&plan->graph_exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    plan->graph_exec = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  plan->graph = graph;
  // each pass alone, captured the same way
  for (size_t i = 0; i < plan->passes.size(); ++i) {
    e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    cs = enqueue_pass(plan, plan->passes[i], fp, plan->capture_stream, plan->ws,
                      forks[i].side ? &forks[i] : nullptr);
    hipGraph_t pg = nullptr;
    e = hipStreamEndCapture(plan->capture_stream, &pg);
    if (cs != PSATD_OK) {
      if (pg) (void)hipGraphDestroy(pg);
      return cs;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t px = nullptr;
    e = hipGraphInstantiate(&px, pg, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(pg);
      return hip_fail(e, "hipGraphInstantiate");
    }
    plan->pass_graphs.push_back(pg);
    plan->pass_exec.push_back(px);
  }
  return PSATD_OK;
}

// ---------------------------------------------------------------- tuning
// The candidates of one pass: the plan's own choice first, then other tiles
// (lines per workgroup), modes or points per thread, radix schedules and
// kernel families.  Each keeps its host work list, checked against the plan
// by verify_pass; it is uploaded only when timed or chosen.
struct Cand {
  Pass pass;
  std::vector<WorkItem> its;  // empty for the plan's own choice (already on the device)
};

std::vector<Cand> pass_candidates(const psatd_plan_s* plan, const Pass& ps) {
  std::vector<Cand> cands;
  cands.push_back(Cand{ps, {}});
  // (fused passes: also at every compiled modes-per-thread choice that holds
  // the z lines; these run the same arithmetic per line)
  // (line passes: also at both radix schedules, radix-4 stages at 4 points
  // per thread and radices up to 8 at 8; they round differently, and each
  // is checked against the oracle by the tests)
  // (the wave-resident z pass: also the generic fused pass, at every choice)
  // (line passes: also the compile-time and the wave-resident kernels where
  // they apply)
  const bool linelike = ps.type == kLine || ps.type == kWaveX;
  std::vector<int> vars = {0};
  if (ps.type == kFused || ps.type == kWaveZ) vars = fused_mpt_choices(plan->cfg.precision, plan->ndim);
  if (linelike) vars = {4, kMaxPts};
  auto add = [&](Pass c, std::vector<WorkItem>& its) {
    for (const Cand& x : cands)
      if (x.pass.type == c.type && x.pass.ct == c.ct && x.pass.lines == c.lines &&
          x.pass.mpt == c.mpt && x.pass.ppt == c.ppt)
        return;
    c.d_items = nullptr;
    if (verify_pass(plan, c, its.data()) != PSATD_OK) return;
    cands.push_back(Cand{c, std::move(its)});
  };
  if (linelike && !(ps.type == kLine && ps.ct) && ct_line_eligible(ps.line_kind, plan)) {
    std::vector<WorkItem> its;
    add(make_ct_line_pass(ps.line_kind, plan, ps.comps, its), its);
  }
  if (linelike && ps.type != kWaveX && wave_line_eligible(ps.line_kind, plan)) {
    std::vector<WorkItem> its;
    add(make_wave_x_pass(ps.line_kind, plan, ps.comps, its), its);
  }
  if (linelike || ps.type == kFused || ps.type == kWaveZ) {
    for (int m : vars) {
      for (int R : {1, 2, 4, 8, 16, 32}) {
        std::vector<WorkItem> its;
        Pass c;
        if (linelike) {
          c = make_line_pass(ps.line_kind, plan, ps.comps, its, R, m);
        } else if (make_fused_pass(plan, its, &c, R, m) != PSATD_OK) {
          continue;
        }
        add(c, its);
      }
    }
  }
  return cands;
}

// The launch grids a candidate is timed at: one workgroup per item (the wave
// z pass: one wavefront per item), or a persistent grid of k workgroups per
// CU; per-length launches take a code (0: every item its own workgroup, k: k
// per CU) that set_grid turns into each launch's grid.
std::vector<int> grid_choices(const psatd_plan_s* plan, const Pass& c) {
  if (!c.subs.empty()) return {0, 1, 2, 4, 8};
  const int full = c.type == kWaveZ ? c.shape.grid : c.nitems;
  std::vector<int> grids = {full};
  for (int k : {1, 2, 4, 8})
    if (k * plan->num_cus < full) grids.push_back(k * plan->num_cus);
  return grids;
}

bool parse_tuning(const char* text, std::vector<Choice>* out) {
  out->clear();
  const char* p = text;
  if (std::strncmp(p, "psatd-tuning-1", 14) != 0) return false;
  p += 14;
  while (*p == ';') {
    ++p;
    Choice c{};
    int used = 0;
    if (std::sscanf(p, "%d,%d,%d,%d,%d,%d%n", &c.type, &c.ct, &c.lines, &c.mpt, &c.ppt, &c.grid,
                    &used) != 6)
      return false;
    out->push_back(c);
    p += used;
  }
  return *p == '\0' && !out->empty();
}

// Upload a candidate's work list into plan-owned device memory.
psatd_status upload_items(psatd_plan_s* plan, Cand& c, WorkItem** d) {
  *d = nullptr;
  if (c.its.empty()) return PSATD_OK;
  hipError_t e = hipMalloc(d, sizeof(WorkItem) * c.its.size());
  if (e == hipSuccess)
    e = hipMemcpy(*d, c.its.data(), sizeof(WorkItem) * c.its.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (*d) (void)hipFree(*d);
    *d = nullptr;
    return hip_fail(e, "tuning: work list upload");
  }
  c.pass.d_items = *d;
  return PSATD_OK;
}

// Apply the choices of a tuning string (from psatd_plan_tuning of a plan with
// the same configuration and patches): no timing launch.
psatd_status apply_tuning(psatd_plan_s* plan, const std::vector<Choice>& choice) {
  if (choice.size() != plan->passes.size())
    return fail(PSATD_ERR_INVALID_ARG, "tuning: " + std::to_string(choice.size()) +
                                           " choices for a plan of " +
                                           std::to_string(plan->passes.size()) + " passes");
  for (size_t i = 0; i < plan->passes.size(); ++i) {
    Pass& ps = plan->passes[i];
    const Choice& ch = choice[i];
    std::vector<Cand> cands = pass_candidates(plan, ps);
    int pick = -1;
    for (size_t ci = 0; ci < cands.size() && pick < 0; ++ci) {
      const Pass& c = cands[ci].pass;
      if (c.type == ch.type && static_cast<int>(c.ct) == ch.ct && c.lines == ch.lines &&
          c.mpt == ch.mpt && c.ppt == ch.ppt)
        pick = static_cast<int>(ci);
    }
    if (pick < 0)
      return fail(PSATD_ERR_INVALID_ARG,
                  std::string("tuning: no such kernel choice for pass ") + ps.name);
    Cand& c = cands[pick];
    if (ch.grid >= 0) {
      const std::vector<int> grids = grid_choices(plan, c.pass);
      if (std::find(grids.begin(), grids.end(), ch.grid) == grids.end())
        return fail(PSATD_ERR_INVALID_ARG, std::string("tuning: grid not offered for pass ") + ps.name);
    }
    if (!plan->dry) {
      WorkItem* d = nullptr;
      psatd_status st = upload_items(plan, c, &d);
      if (st != PSATD_OK) return st;
      if (d) plan->extra_items.push_back(d);
    }
    ps = c.pass;
    if (ch.grid >= 0) set_grid(plan, ps, ch.grid);
    ps.grid_choice = ch.grid;
    ps.tuning_applied = true;
  }
  return PSATD_OK;
}

// Launch-shape autotuning (PSATD_FLAG_AUTOTUNE).  Every kernel loops over its
// work list, so any grid size is correct; what changes is whether one
// workgroup per CU walks the list (and prefetches its next item) or the
// hardware hands out items as CUs free up.  Each pass is timed alone, at each
// candidate grid, on zero-filled scratch fields (the work does not depend on
// the values), and keeps the fastest.
psatd_status autotune_passes(psatd_plan_s* plan) {
  long long total = 0;
  for (const psatd_patch_desc& d : plan->desc)
    total = std::max<long long>(total, d.offset + d.n[0] * d.n[1] * d.n[2]);
  const size_t comp_bytes = static_cast<size_t>(total) * plan->elem;
  void* fields = nullptr;
  void* tmp_ws = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  psatd_status st = PSATD_OK;
  auto cleanup = [&]() {
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (fields) (void)hipFree(fields);
    if (tmp_ws) {
      (void)hipFree(tmp_ws);
      plan->ws = nullptr;
    }
  };
  hipError_t e = hipMalloc(&fields, comp_bytes * plan->nin);
  if (e != hipSuccess) {
    fields = nullptr;
    cleanup();
    return fail(PSATD_ERR_OOM, "autotune: scratch fields");
  }
  e = hipMemset(fields, 0, comp_bytes * plan->nin);
  if (e == hipSuccess && !plan->ws) {
    e = hipMalloc(&tmp_ws, plan->ws_bytes);
    if (e == hipSuccess) {
      plan->ws = tmp_ws;
      e = hipMemset(tmp_ws, 0, plan->ws_bytes);
    } else {
      tmp_ws = nullptr;
    }
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "autotune setup");
  }
  FieldPtrs f{};
  for (int c = 0; c < plan->nin; ++c) f.f[c] = static_cast<char*>(fields) + c * comp_bytes;
  constexpr int kReps = 3;
  // Mean ms of one launch of `ps` (warm-up first), or a negative value on error.
  auto time_pass = [&](const Pass& ps) -> double {
    st = enqueue_pass(plan, ps, f, s, plan->ws);
    if (st != PSATD_OK) return -1.0;
    e = hipEventRecord(e0, s);
    for (int r = 0; r < kReps && st == PSATD_OK && e == hipSuccess; ++r) st = enqueue_pass(plan, ps, f, s, plan->ws);
    if (st != PSATD_OK) return -1.0;
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    return e == hipSuccess ? ms / kReps : -1.0;
  };
  for (Pass& ps : plan->passes) {
    std::vector<Cand> cands = pass_candidates(plan, ps);
    std::vector<WorkItem*> dev(cands.size(), nullptr);
    int best_c = 0, best_g = ps.shape.grid;
    double best_ms = 1e300;
    for (size_t ci = 0; ci < cands.size() && st == PSATD_OK && e == hipSuccess; ++ci) {
      st = upload_items(plan, cands[ci], &dev[ci]);
      if (st != PSATD_OK) break;
      Pass& c = cands[ci].pass;
      for (int g : grid_choices(plan, c)) {
        set_grid(plan, c, g);
        const double ms = time_pass(c);
        if (ms < 0.0) break;
        if (ms < best_ms) {
          best_ms = ms;
          best_c = static_cast<int>(ci);
          best_g = g;
        }
      }
    }
    for (size_t ci = 0; ci < cands.size(); ++ci)
      if (dev[ci] && (static_cast<int>(ci) != best_c || st != PSATD_OK || e != hipSuccess))
        (void)hipFree(dev[ci]);
    if (st != PSATD_OK || e != hipSuccess) break;
    if (best_c != 0) {
      ps = cands[best_c].pass;
      plan->extra_items.push_back(dev[best_c]);
    }
    set_grid(plan, ps, best_g);
    ps.grid_choice = best_g;
    ps.tuned_ms = best_ms;
  }
  cleanup();
  if (st != PSATD_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "autotune");
  return PSATD_OK;
}

psatd_status build_plan(psatd_plan_s* plan) {
  const psatd_config& cfg = plan->cfg;
  plan->ndim = plan->desc[0].ndim;
  plan->nin = inputs_for(cfg.source_mode);
  const bool pstd = (cfg.flags & PSATD_FLAG_PSTD) != 0;
  plan->src_form = !pstd ? cfg.source_mode
                         : (cfg.source_mode == PSATD_VACUUM ? kPstdVacuum : kPstdJ);
  plan->elem = cfg.precision == PSATD_FP32 ? 4 : 8;

  // ---- tables layout (bytes): per patch kx, ky, kz, post; per FFT length twiddles
  std::map<int, size_t> tw_off;
  size_t tb = 0;
  auto take = [&](size_t bytes) {
    size_t o = tb;
    tb += (bytes + 255) / 256 * 256;
    return o;
  };
  struct PT { size_t kx, ky, kz, kz_b, post; };
  std::vector<PT> pt;
  for (const psatd_patch_desc& d : plan->desc) {
    const int nx = static_cast<int>(d.n[0]);
    const int ny = plan->ndim == 3 ? static_cast<int>(d.n[1]) : 1;
    const int nz = static_cast<int>(d.n[2]);
    const int mx = nx / 2;
    PT t;
    t.kx = take(sizeof(double) * mx);
    t.ky = take(sizeof(double) * ny);
    t.kz = take(sizeof(double) * nz);
    t.kz_b = take(sizeof(double) * nz);
    t.post = take(sizeof(double2) * mx);
    pt.push_back(t);
    for (int L : {mx, ny, nz})
      if (!tw_off.count(L)) tw_off[L] = take(sizeof(double2) * L);
  }
  std::vector<double> fw;
  const int centered = (cfg.flags & PSATD_FLAG_CENTERED_STENCIL) ? 1 : 0;
  if (cfg.order > 0) fw = centered ? fornberg_centered(cfg.order) : fornberg_staggered(cfg.order);
  // The device sincos is accurate for |theta/2| <= kSincosMax; bound |k| per
  // axis by pi/d (exact k) or (2/d) sum |C_l| (order p).
  {
    double wsum = 0.0;
    for (double x : fw) wsum += std::fabs(x);
    const double per = cfg.order > 0 ? 2.0 * wsum : M_PI;
    for (const psatd_patch_desc& d : plan->desc) {
      double k2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        if (plan->ndim == 2 && a == 1) continue;
        const double k = per / d.d[a];
        k2 += k * k;
      }
      if (0.5 * cfg.c * d.dt * std::sqrt(k2) > kSincosMax)
        return fail(PSATD_ERR_INVALID_ARG,
                    "c |k|max dt / 2 exceeds " + std::to_string(kSincosMax) +
                        " (time step too large for the coefficient evaluation)");
    }
  }
  const size_t fw_off = take(sizeof(double) * std::max<size_t>(1, fw.size()));

  const bool dry = plan->dry;
  hipError_t e = hipSuccess;
  if (dry) {
    plan->dry_tables.assign(tb, 0);
  } else {
    e = hipMalloc(&plan->d_tables, tb);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(tables)");
  }
  char* T = dry ? plan->dry_tables.data() : static_cast<char*>(plan->d_tables);
  if (!fw.empty() && !dry) {
    e = hipMemcpy(T + fw_off, fw.data(), sizeof(double) * fw.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(fornberg)");
  }
  const double* d_fw = reinterpret_cast<const double*>(T + fw_off);
  const int nfw = static_cast<int>(fw.size());

  for (auto& kv : tw_off) {
    if (dry) break;
    e = launch_twiddles(reinterpret_cast<double2*>(T + kv.second), kv.first, kv.first, nullptr);
    if (e != hipSuccess) return hip_fail(e, "twiddle table");
  }

  // ---- patch descriptors and workspace layout
  long long spec_off = 0;
  plan->host_patches.clear();
  for (size_t i = 0; i < plan->desc.size(); ++i) {
    const psatd_patch_desc& d = plan->desc[i];
    PatchDev P{};
    P.ndim = plan->ndim;
    P.nx = static_cast<int>(d.n[0]);
    P.ny = plan->ndim == 3 ? static_cast<int>(d.n[1]) : 1;
    P.nz = static_cast<int>(d.n[2]);
    P.mx = P.nx / 2;
    P.dt = d.dt;
    P.inv_n = 1.0 / (static_cast<double>(P.nx) * P.ny * P.nz);
    P.dkz = cfg.order == 0 ? 6.283185307179586476925286766559 / (static_cast<double>(P.nz) * d.d[2])
                           : 0.0;
    P.off_real = d.offset;
    P.comp_stride = static_cast<long long>(P.mx) * P.ny * P.nz;
    P.off_spec = spec_off;
    spec_off += (P.comp_stride * plan->nin + 63) / 64 * 64;
    P.kx = reinterpret_cast<const double*>(T + pt[i].kx);
    P.ky = reinterpret_cast<const double*>(T + pt[i].ky);
    P.kz = reinterpret_cast<const double*>(T + pt[i].kz);
    P.kz_b = reinterpret_cast<const double*>(T + pt[i].kz_b);
    P.post = reinterpret_cast<const double2*>(T + pt[i].post);
    if (!plan->maps.empty()) P.map = plan->maps[i];
    auto fill = [&](FFTPlanDev& f, int L, int max_radix) {
      const std::vector<int> r = radix_plan(L, max_radix);
      f.n = L;
      f.nstages = static_cast<int>(r.size());
      for (size_t s = 0; s < r.size(); ++s) f.radix[s] = r[s];
      f.tw = reinterpret_cast<const double2*>(T + tw_off[L]);
    };
    fill(P.fx, P.mx, kMaxPts);
    fill(P.fy, P.ny, kMaxPts);
    fill(P.fz, P.nz, kMaxRadixZ);
    plan->host_patches.push_back(P);
    if (dry) continue;

    e = launch_ktable(const_cast<double*>(P.kx), P.nx, d.d[0], P.mx, 1, d_fw, nfw, centered, nullptr);
    if (e == hipSuccess && plan->ndim == 3)
      e = launch_ktable(const_cast<double*>(P.ky), P.ny, d.d[1], P.ny, 0, d_fw, nfw, centered, nullptr);
    if (e == hipSuccess && plan->ndim == 2) {
      const double zero = 0.0;
      e = hipMemcpy(const_cast<double*>(P.ky), &zero, sizeof(double), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
      e = launch_ktable(const_cast<double*>(P.kz), P.nz, d.d[2], P.nz, 0, d_fw, nfw, centered, nullptr);
    if (e == hipSuccess)
      e = launch_twiddles(const_cast<double2*>(P.post), P.nx, P.mx, nullptr);
    if (e != hipSuccess) return hip_fail(e, "k tables");
    if (P.nz == fast2d::kNZfast) {
      // mode order of the specialized z pass (see PatchDev::kz_b)
      std::vector<double> kz(P.nz), kzb(P.nz);
      e = hipMemcpy(kz.data(), P.kz, sizeof(double) * P.nz, hipMemcpyDeviceToHost);
      for (int q = 0; q < 8; ++q)
        for (int k2 = 0; k2 < 8; ++k2)
          for (int j = 0; j < 64; ++j) kzb[64 * k2 + j + 512 * q] = kz[8 * j + k2 + 512 * q];
      if (e == hipSuccess)
        e = hipMemcpy(const_cast<double*>(P.kz_b), kzb.data(), sizeof(double) * P.nz,
                      hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "kz table (z pass order)");
    }
  }
  // 3D: a second block of the same size for the z passes (see PatchDev::off_z)
  for (PatchDev& P : plan->host_patches) P.off_z = plan->ndim == 3 ? spec_off + P.off_spec : P.off_spec;
  if (plan->ndim == 3) spec_off *= 2;
  plan->ws_bytes = static_cast<size_t>(spec_off) * 2 * plan->elem;

  if (!dry) {
    e = hipMalloc(&plan->d_patches, sizeof(PatchDev) * plan->host_patches.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(patches)");
    e = hipMemcpy(plan->d_patches, plan->host_patches.data(),
                  sizeof(PatchDev) * plan->host_patches.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(patches)");
  }

  // ---- passes
  std::vector<int> in_comps, out_comps;
  for (int c = 0; c < plan->nin; ++c) in_comps.push_back(c);
  for (int c = 0; c < 6; ++c) out_comps.push_back(c);
  std::vector<WorkItem> items;
  plan->passes.clear();
  if (fast2d_eligible(plan)) {
    plan->passes.push_back(make_fast_pass(kFastXFwd, plan, in_comps, items));
    plan->passes.push_back(make_fast_pass(kFastZ, plan, in_comps, items));
    plan->passes.push_back(make_fast_pass(kFastXInv, plan, out_comps, items));
  } else {
    // compile-time line kernels where every length is compiled, else the
    // generic ones (the autotuner times both)
    auto line = [&](int kind, const std::vector<int>& comps) {
      if (wave_line_eligible(kind, plan)) return make_wave_x_pass(kind, plan, comps, items);
      return ct_line_eligible(kind, plan) ? make_ct_line_pass(kind, plan, comps, items)
                                          : make_line_pass(kind, plan, comps, items);
    };
    plan->passes.push_back(line(kXFwd, in_comps));
  if (plan->ndim == 3) plan->passes.push_back(line(kYFwd, in_comps));
  if (cfg.path == PSATD_PATH_FUSED && wave_z_eligible(plan)) {
    plan->passes.push_back(make_wave_z_pass(plan, items));
  } else if (cfg.path == PSATD_PATH_FUSED && fused_fits(plan, items)) {
    Pass fz;
    psatd_status st = make_fused_pass(plan, items, &fz);
    if (st != PSATD_OK) return st;
    plan->passes.push_back(fz);
  } else {
    // the plain z passes: asked for, or the fused pass cannot hold a z line
    plan->passes.push_back(line(kZFwd, in_comps));
    plan->passes.push_back(make_update_pass(plan, items));
    plan->passes.push_back(line(kZInv, out_comps));
  }
  if (plan->ndim == 3) plan->passes.push_back(line(kYInv, out_comps));
  plan->passes.push_back(line(kXInv, out_comps));
  }

  for (const Pass& ps : plan->passes) {
    psatd_status st = verify_pass(plan, ps, items.data() + reinterpret_cast<size_t>(ps.d_items));
    if (st != PSATD_OK) return st;
  }
  if (!dry) {
    e = hipMalloc(&plan->d_items, sizeof(WorkItem) * items.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(work items)");
    e = hipMemcpy(plan->d_items, items.data(), sizeof(WorkItem) * items.size(),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(work items)");
    for (Pass& ps : plan->passes)
      ps.d_items = static_cast<WorkItem*>(plan->d_items) + reinterpret_cast<size_t>(ps.d_items);

    if (!(cfg.flags & PSATD_FLAG_NO_WORKSPACE)) {
      e = hipMalloc(&plan->ws, plan->ws_bytes);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
      plan->ws_owned = true;
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "plan tables");
    if (!plan->tuning.empty()) {
      psatd_status st = apply_tuning(plan, plan->tuning);
      if (st != PSATD_OK) return st;
    } else if (cfg.flags & PSATD_FLAG_AUTOTUNE) {
      psatd_status st = autotune_passes(plan);
      if (st != PSATD_OK) return st;
    }
    if (cfg.flags & PSATD_FLAG_GRAPH) {
      psatd_status st = build_graph(plan);
      if (st != PSATD_OK) return st;
    }
  }

  char buf[512];
  plan->info.clear();
  std::snprintf(buf, sizeof(buf),
                "ndim=%d patches=%zu solver=%s precision=%s source=%d path=%s order=%d ws=%zu\n",
                plan->ndim, plan->host_patches.size(), pstd ? "pstd" : "psatd",
                cfg.precision == PSATD_FP32 ? "fp32" : "fp64", cfg.source_mode,
                cfg.path == PSATD_PATH_FUSED ? "fused" : "plain", cfg.order, plan->ws_bytes);
  plan->info += buf;
  for (const Pass& ps : plan->passes) {
    std::snprintf(buf, sizeof(buf),
                  "  %-10s items=%d grid=%d block=%d lds=%zu mpt=%d ppt=%d lines=%d bytes=%.0f kernel=%s%s\n",
                  ps.name, ps.nitems, ps.shape.grid, ps.shape.block, ps.shape.lds_bytes, ps.mpt,
                  ps.ppt, ps.lines, ps.bytes,
                  (ps.type == kWaveZ || ps.type == kWaveX)
                      ? "wave"
                      : (ps.ct ? "compile-time" : (ps.type >= kFastXFwd ? "4096" : "generic")),
                  ps.tuning_applied ? " (tuning applied)" : (ps.tuned_ms >= 0.0 ? " (autotuned)" : ""));
    plan->info += buf;
  }
  return PSATD_OK;
}

psatd_status create_plan(const psatd_config* cfg, const psatd_patch_desc* patches, int32_t npatches,
                         int32_t device, const GlobalMap* maps, psatd_plan_t* out,
                         const char* tuning = nullptr) {
  try {
    if (!out) return fail(PSATD_ERR_INVALID_ARG, "out is NULL");
    psatd_status st = validate(cfg, patches, npatches);
    if (st != PSATD_OK) return st;
    std::vector<Choice> choices;
    if (tuning && !parse_tuning(tuning, &choices))
      return fail(PSATD_ERR_INVALID_ARG, "tuning string does not parse");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
      return fail(PSATD_ERR_HIP, "no HIP device available");
    if (device < 0 || device >= ndev)
      return fail(PSATD_ERR_INVALID_ARG, "device index out of range");
    DeviceGuard g(device);
    if (!g.ok) return fail(PSATD_ERR_HIP, "hipSetDevice failed");
    {
      // the dynamic-LDS limit of every kernel, raised once per device
      static std::mutex mu;
      static std::set<int> configured;
      std::lock_guard<std::mutex> lock(mu);
      if (!configured.count(device)) {
        hipError_t e = configure_kernel_attributes();
        if (e == hipSuccess) e = fast2d::configure_attributes();
        if (e == hipSuccess) e = wave2d::configure_attributes();
        if (e == hipSuccess) e = wave2d::configure_x_attributes();
        if (e == hipSuccess) e = wave2d::configure_z3_attributes();
        if (e != hipSuccess) return hip_fail(e, "kernel attributes");
        if (lookup_scratch(device) != PSATD_OK)
          return fail(PSATD_ERR_HIP, "hipGetSymbolAddress(scratch) failed");
        configured.insert(device);
      }
    }
    psatd_plan_s* plan = new psatd_plan_s();
    plan->cfg = *cfg;
    plan->device = device;
    {
      int ncu = 0;
      if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) ==
              hipSuccess &&
          ncu > 0)
        plan->num_cus = ncu;
    }
    plan->desc.assign(patches, patches + npatches);
    if (maps) plan->maps.assign(maps, maps + npatches);
    plan->tuning = choices;
    st = build_plan(plan);
    if (st != PSATD_OK) {
      free_plan_memory(plan);
      delete plan;
      return st;
    }
    *out = plan;
    return PSATD_OK;
  } catch (const std::exception& ex) {
    return fail(PSATD_ERR_OOM, std::string("host allocation failed: ") + ex.what());
  } catch (...) {
    return fail(PSATD_ERR_INVALID_ARG, "unexpected host exception");
  }
}

}  // namespace

// A plan whose patches are boxes of a guard-cell decomposition of one global
// grid (domain.hip): the x passes read each patch from the global fields and
// write its interior back (GlobalMap).  maps[i] describes patches[i].
psatd_status plan_mapped(const psatd_config* cfg, const psatd_patch_desc* patches,
                         const GlobalMap* maps, int32_t npatches, int32_t device,
                         psatd_plan_t* out) {
  if (!maps) return fail(PSATD_ERR_INVALID_ARG, "maps is NULL");
  return create_plan(cfg, patches, npatches, device, maps, out);
}

// ====================================================================== C ABI
extern "C" {

psatd_status psatd_plan(const psatd_config* cfg, const psatd_patch_desc* patches, int32_t npatches,
                        int32_t device, psatd_plan_t* out) {
  return create_plan(cfg, patches, npatches, device, nullptr, out);
}

psatd_status psatd_plan_tuned(const psatd_config* cfg, const psatd_patch_desc* patches,
                              int32_t npatches, int32_t device, const char* tuning,
                              psatd_plan_t* out) {
  if (!tuning) return fail(PSATD_ERR_INVALID_ARG, "tuning is NULL");
  return create_plan(cfg, patches, npatches, device, nullptr, out, tuning);
}

psatd_status psatd_plan_tuning(psatd_plan_t plan, char* buf, size_t len, size_t* needed) {
  if (!plan) return fail(PSATD_ERR_INVALID_ARG, "plan is NULL");
  std::string t = "psatd-tuning-1";
  char tok[96];
  for (const Pass& ps : plan->passes) {
    std::snprintf(tok, sizeof(tok), ";%d,%d,%d,%d,%d,%d", static_cast<int>(ps.type),
                  ps.ct ? 1 : 0, ps.lines, ps.mpt, ps.ppt, ps.grid_choice);
    t += tok;
  }
  if (needed) *needed = t.size() + 1;
  if (buf) {
    if (len < t.size() + 1) return fail(PSATD_ERR_INVALID_ARG, "tuning buffer too small");
    std::memcpy(buf, t.c_str(), t.size() + 1);
  }
  return PSATD_OK;
}

psatd_status psatd_plan_describe(const psatd_config* cfg, const psatd_patch_desc* patches,
                                 int32_t npatches, size_t* ws_bytes, char* info, size_t len) {
  try {
    psatd_status st = validate(cfg, patches, npatches);
    if (st != PSATD_OK) return st;
    psatd_plan_s plan;
    plan.cfg = *cfg;
    plan.dry = true;
    plan.desc.assign(patches, patches + npatches);
    st = build_plan(&plan);
    if (st != PSATD_OK) return st;
    if (ws_bytes) *ws_bytes = plan.ws_bytes;
    if (info && len > 0) std::snprintf(info, len, "%s", plan.info.c_str());
    return PSATD_OK;
  } catch (const std::exception& ex) {
    return fail(PSATD_ERR_OOM, std::string("host allocation failed: ") + ex.what());
  } catch (...) {
    return fail(PSATD_ERR_INVALID_ARG, "unexpected host exception");
  }
}

psatd_status psatd_workspace_size(psatd_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(PSATD_ERR_INVALID_ARG, "NULL argument");
  *bytes = plan->ws_bytes;
  return PSATD_OK;
}

psatd_status psatd_set_workspace(psatd_plan_t plan, void* ptr, size_t bytes) {
  if (!plan || !ptr) return fail(PSATD_ERR_INVALID_ARG, "NULL argument");
  if (bytes < plan->ws_bytes)
    return fail(PSATD_ERR_WORKSPACE, "workspace of " + std::to_string(bytes) + " bytes < required " +
                                         std::to_string(plan->ws_bytes));
  if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
    return fail(PSATD_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  DeviceGuard g(plan->device);
  if (plan->ws && plan->ws_owned) (void)hipFree(plan->ws);
  plan->ws = ptr;
  plan->ws_owned = false;
  if (plan->cfg.flags & PSATD_FLAG_GRAPH) return build_graph(plan);
  return PSATD_OK;
}

static psatd_status push_impl(psatd_plan_t plan, const psatd_fields* fields, int32_t nsteps,
                              void* hip_stream, double* ms_per_pass, int32_t max_pass) {
  if (!plan) return fail(PSATD_ERR_INVALID_ARG, "plan is NULL");
  if (nsteps < 0) return fail(PSATD_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (nsteps > 1 && plan->cfg.source_mode != PSATD_VACUUM && !ms_per_pass)
    return fail(PSATD_ERR_INVALID_ARG, "with sources, push one step at a time (nsteps = 1)");
  if (!plan->ws) return fail(PSATD_ERR_WORKSPACE, "no workspace: call psatd_set_workspace");
  FieldPtrs fp;
  psatd_status st = check_fields(plan, fields, &fp);
  if (st != PSATD_OK) return st;
  if (nsteps == 0) return PSATD_OK;
  DeviceGuard g(plan->device);
  if (!g.ok) return fail(PSATD_ERR_HIP, "hipSetDevice failed");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);

  if (ms_per_pass) {
    const int np = static_cast<int>(plan->passes.size());
    if (max_pass < np) return fail(PSATD_ERR_INVALID_ARG, "ms_per_pass holds fewer than npass entries");
    std::vector<hipEvent_t> ev(2 * np * nsteps);
    for (auto& x : ev)
      if (hipEventCreate(&x) != hipSuccess) return fail(PSATD_ERR_HIP, "hipEventCreate");
    // a graph plan runs each pass's own graph (captured like the step's), so
    // each pass is timed as the step's graph runs it
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    const bool graphs = (plan->cfg.flags & PSATD_FLAG_GRAPH) &&
                        static_cast<int>(plan->pass_exec.size()) == np &&
                        hipStreamIsCapturing(s, &cst) == hipSuccess && cst == hipStreamCaptureStatusNone;
    psatd_status rs = PSATD_OK;
    if (graphs && launch_store_fields(fp, plan->d_fieldtab, s) != hipSuccess)
      rs = fail(PSATD_ERR_HIP, "field table");
    for (int n = 0; n < nsteps && rs == PSATD_OK; ++n)
      for (int i = 0; i < np && rs == PSATD_OK; ++i) {
        (void)hipEventRecord(ev[2 * (n * np + i)], s);
        if (graphs) {
          const hipError_t ge = hipGraphLaunch(plan->pass_exec[i], s);
          if (ge != hipSuccess) rs = hip_fail(ge, "hipGraphLaunch");
        } else {
          rs = enqueue_pass(plan, plan->passes[i], fp, s, plan->ws);
        }
        (void)hipEventRecord(ev[2 * (n * np + i) + 1], s);
      }
    hipError_t e = hipStreamSynchronize(s);
    for (int i = 0; i < np; ++i) ms_per_pass[i] = 0.0;
    if (rs == PSATD_OK && e == hipSuccess) {
      for (int n = 0; n < nsteps; ++n)
        for (int i = 0; i < np; ++i) {
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, ev[2 * (n * np + i)], ev[2 * (n * np + i) + 1]);
          ms_per_pass[i] += ms / nsteps;
        }
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (rs != PSATD_OK) return rs;
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    return PSATD_OK;
  }

  if (plan->cfg.flags & PSATD_FLAG_GRAPH) {
    // A stream the caller is capturing records the kernels themselves;
    // otherwise write the field table and replay the plan's graph.
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cst);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cst == hipStreamCaptureStatusNone) {
      if (!plan->graph_exec) return fail(PSATD_ERR_STATE, "graph plan without its graph");
      e = launch_store_fields(fp, plan->d_fieldtab, s);
      if (e != hipSuccess) return hip_fail(e, "field table");
      for (int n = 0; n < nsteps; ++n) {
        e = hipGraphLaunch(plan->graph_exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      }
      return PSATD_OK;
    }
  }

  for (int n = 0; n < nsteps; ++n) {
    st = enqueue_step(plan, fp, s, plan->ws);
    if (st != PSATD_OK) return st;
  }
  return PSATD_OK;
}

psatd_status psatd_push(psatd_plan_t plan, const psatd_fields* fields, int32_t nsteps,
                        void* hip_stream) {
  try {
    return push_impl(plan, fields, nsteps, hip_stream, nullptr, 0);
  } catch (...) {
    return fail(PSATD_ERR_INVALID_ARG, "unexpected host exception");
  }
}

psatd_status psatd_push_scratch(psatd_plan_t plan, const psatd_fields* fields, int32_t nsteps,
                                void* hip_stream) {
  try {
    if (!plan) return fail(PSATD_ERR_INVALID_ARG, "plan is NULL");
    if (nsteps < 0) return fail(PSATD_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (nsteps > 1 && plan->cfg.source_mode != PSATD_VACUUM)
      return fail(PSATD_ERR_INVALID_ARG, "with sources, push one step at a time (nsteps = 1)");
    if (plan->ws_bytes > static_cast<size_t>(PSATD_SCRATCH_BYTES))
      return fail(PSATD_ERR_WORKSPACE,
                  "the plan needs " + std::to_string(plan->ws_bytes) +
                      " bytes of workspace; psatd_push_scratch holds at most " +
                      std::to_string(static_cast<size_t>(PSATD_SCRATCH_BYTES)));
    FieldPtrs fp;
    psatd_status st = check_fields(plan, fields, &fp);
    if (st != PSATD_OK) return st;
    if (nsteps == 0) return PSATD_OK;
    void* ws = scratch_ptr(plan->device);
    if (!ws) return fail(PSATD_ERR_STATE, "no scratch address for the plan's device");
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(PSATD_ERR_HIP, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    for (int n = 0; n < nsteps; ++n) {
      st = enqueue_step(plan, fp, s, ws);
      if (st != PSATD_OK) return st;
    }
    return PSATD_OK;
  } catch (...) {
    return fail(PSATD_ERR_INVALID_ARG, "unexpected host exception");
  }
}

psatd_status psatd_push_profiled(psatd_plan_t plan, const psatd_fields* fields, int32_t nsteps,
                                 void* hip_stream, double* ms_per_pass, int32_t max_pass) {
  if (!ms_per_pass) return fail(PSATD_ERR_INVALID_ARG, "ms_per_pass is NULL");
  if (nsteps < 1) return fail(PSATD_ERR_INVALID_ARG, "nsteps must be >= 1");
  try {
    return push_impl(plan, fields, nsteps, hip_stream, ms_per_pass, max_pass);
  } catch (...) {
    return fail(PSATD_ERR_INVALID_ARG, "unexpected host exception");
  }
}

psatd_status psatd_pass_count(psatd_plan_t plan, int32_t* npass) {
  if (!plan || !npass) return fail(PSATD_ERR_INVALID_ARG, "NULL argument");
  *npass = static_cast<int32_t>(plan->passes.size());
  return PSATD_OK;
}

const char* psatd_pass_name(psatd_plan_t plan, int32_t i) {
  if (!plan || i < 0 || i >= static_cast<int32_t>(plan->passes.size())) return nullptr;
  return plan->passes[i].name;
}

psatd_status psatd_pass_bytes(psatd_plan_t plan, int32_t i, double* bytes) {
  if (!plan || !bytes) return fail(PSATD_ERR_INVALID_ARG, "NULL argument");
  if (i < 0 || i >= static_cast<int32_t>(plan->passes.size()))
    return fail(PSATD_ERR_INVALID_ARG, "pass index out of range");
  *bytes = plan->passes[i].bytes;
  return PSATD_OK;
}

psatd_status psatd_plan_info(psatd_plan_t plan, char* buf, size_t len) {
  if (!plan || !buf || len == 0) return fail(PSATD_ERR_INVALID_ARG, "NULL argument");
  std::snprintf(buf, len, "%s", plan->info.c_str());
  return PSATD_OK;
}

psatd_status psatd_destroy(psatd_plan_t plan) {
  if (!plan) return PSATD_OK;
  {
    DeviceGuard g(plan->device);
    free_plan_memory(plan);
  }
  delete plan;
  return PSATD_OK;
}

const char* psatd_status_string(psatd_status s) {
  switch (s) {
    case PSATD_OK: return "PSATD_OK";
    case PSATD_ERR_INVALID_ARG: return "PSATD_ERR_INVALID_ARG";
    case PSATD_ERR_UNSUPPORTED_SIZE: return "PSATD_ERR_UNSUPPORTED_SIZE";
    case PSATD_ERR_OOM: return "PSATD_ERR_OOM";
    case PSATD_ERR_HIP: return "PSATD_ERR_HIP";
    case PSATD_ERR_WORKSPACE: return "PSATD_ERR_WORKSPACE";
    case PSATD_ERR_STATE: return "PSATD_ERR_STATE";
  }
  return "PSATD_ERR_UNKNOWN";
}

const char* psatd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
