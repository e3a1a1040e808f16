// Host-side exerciser of the planner (psatd_plan_describe) and of argument
// validation, built with AddressSanitizer and UndefinedBehaviorSanitizer on
// the host code.  No GPU is needed: psatd_plan_describe makes no HIP call.
//
// Each valid case must plan (status PSATD_OK, a non-zero workspace, a pass
// description); each invalid case must return its documented status with a
// message in psatd_last_error().  Exit status 0 only if every case did.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "psatd.h"

namespace {

int g_fail = 0, g_cases = 0;

void expect(bool ok, const std::string& what) {
  ++g_cases;
  if (!ok) {
    ++g_fail;
    std::printf("FAIL %s (last error: %s)\n", what.c_str(), psatd_last_error());
  }
}

psatd_config config(int precision, int source, int path, int order, uint32_t flags) {
  psatd_config c;
  std::memset(&c, 0, sizeof(c));
  c.precision = precision;
  c.source_mode = source;
  c.path = path;
  c.order = order;
  c.c = 1.0;
  c.eps0 = 1.0;
  c.flags = flags;
  return c;
}

psatd_patch_desc patch(int ndim, int64_t nx, int64_t ny, int64_t nz, double dt, int64_t offset) {
  psatd_patch_desc p;
  std::memset(&p, 0, sizeof(p));
  p.ndim = ndim;
  p.n[0] = nx;
  p.n[1] = ndim == 3 ? ny : 1;
  p.n[2] = nz;
  p.d[0] = p.d[1] = p.d[2] = 1.0;
  p.dt = dt;
  p.offset = offset;
  return p;
}

// Packs the patches in order (even offsets) and plans them on the host.
psatd_status describe(const psatd_config& c, std::vector<psatd_patch_desc> ps, size_t* ws,
                      std::string* info) {
  int64_t off = 0;
  for (auto& p : ps) {
    p.offset = off;
    const int64_t cells = p.n[0] * p.n[1] * p.n[2];
    off += cells + (cells & 1);
  }
  std::vector<char> buf(1 << 14, 'x');
  const psatd_status st = psatd_plan_describe(&c, ps.data(), static_cast<int32_t>(ps.size()), ws,
                                              buf.data(), buf.size());
  if (info) *info = st == PSATD_OK ? std::string(buf.data()) : std::string();
  return st;
}

void valid(const psatd_config& c, const std::vector<psatd_patch_desc>& ps, const std::string& tag) {
  size_t ws = 0;
  std::string info;
  const psatd_status st = describe(c, ps, &ws, &info);
  expect(st == PSATD_OK, tag + ": status " + std::to_string(st));
  if (st != PSATD_OK) return;
  expect(ws > 0 && ws % 256 == 0, tag + ": workspace " + std::to_string(ws));
  expect(info.rfind("ndim=", 0) == 0 && info.find("items=") != std::string::npos,
         tag + ": pass description");
}

void invalid(const psatd_config& c, const std::vector<psatd_patch_desc>& ps, psatd_status want,
             const std::string& tag) {
  // offsets as given (the overlap cases depend on them)
  size_t ws = 12345;
  const psatd_status st = psatd_plan_describe(&c, ps.data(), static_cast<int32_t>(ps.size()), &ws,
                                              nullptr, 0);
  expect(st == want, tag + ": status " + std::to_string(st) + ", want " + std::to_string(want));
  expect(ws == 12345, tag + ": *ws_bytes written on failure");
  expect(std::strlen(psatd_last_error()) > 0, tag + ": empty error message");
}

}  // namespace

int main() {
  const int lengths[] = {2, 4, 6, 8, 12, 16, 18, 24, 32, 36, 48, 54, 64, 96, 128, 162, 192,
                         256, 384, 486, 512, 768, 1024, 1536, 2048, 4096};
  const int orders[] = {0, 2, 16, 64};
  const uint32_t flag_sets[] = {0u, PSATD_FLAG_GENERIC_KERNELS, PSATD_FLAG_RADIX4_LINES,
                                PSATD_FLAG_CENTERED_STENCIL, PSATD_FLAG_GENERIC_KERNELS |
                                PSATD_FLAG_RADIX4_LINES};

  // ---- 2D single patches: every length pair x precision x sources x path
  for (int nx : lengths)
    for (int nz : lengths) {
      if (static_cast<int64_t>(nx) * nz > (int64_t(1) << 24)) continue;
      for (int prec : {PSATD_FP32, PSATD_FP64})
        for (int src : {PSATD_VACUUM, PSATD_SOURCES_RHO, PSATD_SOURCES_J})
          for (int path : {PSATD_PATH_FUSED, PSATD_PATH_PLAIN}) {
            const auto c = config(prec, src, path, 0, 0u);
            valid(c, {patch(2, nx, 1, nz, 0.5, 0)},
                  "2d " + std::to_string(nx) + "x" + std::to_string(nz));
          }
    }
  // ---- orders, stencils and kernel-choice flags on a few shapes
  for (int order : orders)
    for (uint32_t fl : flag_sets)
      for (int path : {PSATD_PATH_FUSED, PSATD_PATH_PLAIN}) {
        const auto c = config(PSATD_FP32, PSATD_SOURCES_J, path, order, fl);
        const std::string t = " order " + std::to_string(order) + " flags " + std::to_string(fl);
        valid(c, {patch(2, 4096, 1, 4096, 0.5, 0)}, "2d 4096^2" + t);
        valid(c, {patch(2, 256, 1, 512, 0.5, 0)}, "2d 256x512" + t);
        valid(c, {patch(3, 64, 48, 96, 0.3, 0)}, "3d 64x48x96" + t);
        valid(c, {patch(3, 6, 4, 2, 0.3, 0)}, "3d 6x4x2" + t);
      }
  // ---- 3D shapes up to the workload sizes (no device memory is touched)
  const int l3[][3] = {{2, 2, 2},     {4, 6, 8},      {32, 32, 32},     {64, 64, 64},
                       {128, 96, 48}, {512, 512, 512}, {1024, 1024, 512}, {4096, 2, 4096},
                       {2, 4096, 2},  {1536, 12, 1024}};
  for (const auto& s : l3)
    for (int prec : {PSATD_FP32, PSATD_FP64})
      for (int path : {PSATD_PATH_FUSED, PSATD_PATH_PLAIN}) {
        const auto c = config(prec, PSATD_SOURCES_RHO, path, 0, 0u);
        valid(c, {patch(3, s[0], s[1], s[2], 0.3, 0)},
              "3d " + std::to_string(s[0]) + "x" + std::to_string(s[1]) + "x" + std::to_string(s[2]));
      }
  // ---- batched, ragged patch lists
  {
    std::vector<psatd_patch_desc> ps;
    for (int i = 0; i < 256; ++i) ps.push_back(patch(2, 128, 1, 128, 0.5, 0));
    for (int path : {PSATD_PATH_FUSED, PSATD_PATH_PLAIN})
      valid(config(PSATD_FP32, PSATD_VACUUM, path, 0, 0u), ps, "256 patches 128^2");
    std::vector<psatd_patch_desc> mix;
    for (int i = 0; i < 40; ++i)
      mix.push_back(patch(2, lengths[i % 20 + 2], 1, lengths[(7 * i) % 22 + 1], 0.5, 0));
    for (int path : {PSATD_PATH_FUSED, PSATD_PATH_PLAIN})
      for (uint32_t fl : flag_sets)
        valid(config(PSATD_FP64, PSATD_SOURCES_J, path, 16, fl), mix, "40 mixed 2d patches");
    std::vector<psatd_patch_desc> mix3;
    for (int i = 0; i < 12; ++i)
      mix3.push_back(patch(3, lengths[i % 9 + 1], lengths[(5 * i) % 10 + 1], lengths[(3 * i) % 11 + 1],
                           0.3, 0));
    for (int path : {PSATD_PATH_FUSED, PSATD_PATH_PLAIN})
      valid(config(PSATD_FP32, PSATD_SOURCES_RHO, path, 0, 0u), mix3, "12 mixed 3d patches");
  }
  // ---- PSTD within its Courant condition
  valid(config(PSATD_FP32, PSATD_SOURCES_J, PSATD_PATH_FUSED, 0, PSATD_FLAG_PSTD),
        {patch(2, 256, 1, 256, 0.45, 0)}, "pstd");
  // ---- info truncation and NULL outputs
  {
    const auto c = config(PSATD_FP32, PSATD_VACUUM, PSATD_PATH_FUSED, 0, 0u);
    const auto p = patch(2, 64, 1, 64, 0.5, 0);
    char small[8];
    std::memset(small, 'y', sizeof(small));
    expect(psatd_plan_describe(&c, &p, 1, nullptr, small, sizeof(small)) == PSATD_OK &&
               std::strlen(small) == sizeof(small) - 1,
           "info truncated to len");
    expect(psatd_plan_describe(&c, &p, 1, nullptr, nullptr, 0) == PSATD_OK, "NULL outputs");
  }

  // ---- invalid arguments
  const auto ok = config(PSATD_FP32, PSATD_VACUUM, PSATD_PATH_FUSED, 0, 0u);
  const auto p64 = patch(2, 64, 1, 64, 0.5, 0);
  expect(psatd_plan_describe(nullptr, &p64, 1, nullptr, nullptr, 0) == PSATD_ERR_INVALID_ARG,
         "NULL config");
  expect(psatd_plan_describe(&ok, nullptr, 1, nullptr, nullptr, 0) == PSATD_ERR_INVALID_ARG,
         "NULL patches");
  invalid(ok, std::vector<psatd_patch_desc>{}, PSATD_ERR_INVALID_ARG, "no patches");
  invalid(config(7, PSATD_VACUUM, PSATD_PATH_FUSED, 0, 0u), {p64}, PSATD_ERR_INVALID_ARG, "precision");
  invalid(config(PSATD_FP32, 9, PSATD_PATH_FUSED, 0, 0u), {p64}, PSATD_ERR_INVALID_ARG, "source mode");
  invalid(config(PSATD_FP32, PSATD_VACUUM, 5, 0, 0u), {p64}, PSATD_ERR_INVALID_ARG, "path");
  invalid(config(PSATD_FP32, PSATD_VACUUM, PSATD_PATH_FUSED, 3, 0u), {p64}, PSATD_ERR_INVALID_ARG,
          "odd order");
  invalid(config(PSATD_FP32, PSATD_VACUUM, PSATD_PATH_FUSED, 514, 0u), {p64}, PSATD_ERR_INVALID_ARG,
          "order too high");
  invalid(config(PSATD_FP32, PSATD_VACUUM, PSATD_PATH_FUSED, 0, 0x1000u), {p64}, PSATD_ERR_INVALID_ARG,
          "unknown flag");
  invalid(config(PSATD_FP32, PSATD_SOURCES_RHO, PSATD_PATH_FUSED, 0, PSATD_FLAG_PSTD), {p64},
          PSATD_ERR_INVALID_ARG, "pstd with rho");
  invalid(config(PSATD_FP32, PSATD_VACUUM, PSATD_PATH_FUSED, 0, PSATD_FLAG_PSTD),
          {patch(2, 64, 1, 64, 0.9, 0)}, PSATD_ERR_INVALID_ARG, "pstd beyond Courant");
  {
    auto c = ok;
    c.c = 0.0;
    invalid(c, {p64}, PSATD_ERR_INVALID_ARG, "c = 0");
    c = ok;
    c.eps0 = -1.0;
    invalid(c, {p64}, PSATD_ERR_INVALID_ARG, "eps0 < 0");
  }
  for (int64_t bad : {0, 1, 3, 10, 14, 8192, -4, 6144})
    invalid(ok, {patch(2, bad, 1, 64, 0.5, 0)}, PSATD_ERR_UNSUPPORTED_SIZE,
            "axis length " + std::to_string(bad));
  {
    auto p = p64;
    p.ndim = 4;
    invalid(ok, {p}, PSATD_ERR_INVALID_ARG, "ndim 4");
    p = p64;
    p.n[1] = 2;
    invalid(ok, {p}, PSATD_ERR_INVALID_ARG, "2d with n[1] = 2");
    p = p64;
    p.d[2] = 0.0;
    invalid(ok, {p}, PSATD_ERR_INVALID_ARG, "zero spacing");
    p = p64;
    p.dt = -1.0;
    invalid(ok, {p}, PSATD_ERR_INVALID_ARG, "negative dt");
    p = p64;
    p.offset = 3;
    invalid(ok, {p}, PSATD_ERR_INVALID_ARG, "odd offset");
    invalid(ok, {p64, patch(3, 8, 8, 8, 0.5, 8192)}, PSATD_ERR_INVALID_ARG, "mixed ndim");
    invalid(ok, {p64, patch(2, 64, 1, 64, 0.5, 4000)}, PSATD_ERR_INVALID_ARG, "overlapping patches");
    invalid(ok, {patch(3, 4096, 4096, 4096, 0.5, 0)}, PSATD_ERR_UNSUPPORTED_SIZE, "2^36 cells");
    invalid(ok, {patch(2, 4096, 1, 4096, 1.0e5, 0)}, PSATD_ERR_INVALID_ARG, "dt beyond sincos range");
  }
  // ---- status strings
  for (int s = -8; s <= 1; ++s) expect(psatd_status_string(static_cast<psatd_status>(s)) != nullptr,
                                       "status string " + std::to_string(s));

  // ---- tuning strings are parsed before any device is touched
  {
    const auto c = config(PSATD_FP32, PSATD_VACUUM, PSATD_PATH_FUSED, 0, 0u);
    const psatd_patch_desc p1 = patch(2, 64, 1, 96, 0.5, 0);
    const std::string longest(100000, '9');
    const char* bad[] = {"", "psatd-tuning-1", "psatd-tuning-1;", "psatd-tuning-1;1,2,3",
                         "psatd-tuning-1;1,0,8,0,8,-1;", "psatd-tuning-1;1,0,8,0,8,-1x",
                         "psatd-tuning-0;1,0,8,0,8,-1", longest.c_str()};
    for (const char* t : bad) {
      psatd_plan_t out = nullptr;
      expect(psatd_plan_tuned(&c, &p1, 1, 0, t, &out) == PSATD_ERR_INVALID_ARG && out == nullptr,
             std::string("malformed tuning \"") + std::string(t).substr(0, 40) + "\"");
    }
    psatd_plan_t out = nullptr;
    expect(psatd_plan_tuned(&c, &p1, 1, 0, nullptr, &out) == PSATD_ERR_INVALID_ARG, "NULL tuning");
    size_t n = 0;
    expect(psatd_plan_tuning(nullptr, nullptr, 0, &n) == PSATD_ERR_INVALID_ARG, "tuning of NULL plan");
  }
  std::printf("%d cases, %d failed\n", g_cases, g_fail);
  return g_fail == 0 ? 0 : 1;
}
