// Wave-resident kernels for batched 2D patches (FP32 storage, FP64
// arithmetic).
//
// Fused z pass: one wavefront per work item, which is a group of G kx columns
// (z lines of length L = nz, G = 64 / (L / P)) of one patch.  For each
// polarization group (s: Ey, Bx, Bz; p: Ex, Ez, By, with their sources) the
// wave loads every input's lines (lane s of line g holds z = s + S m), runs
// the forward FFT of each in registers with exchanges through its own LDS
// region (wfft.hpp), updates every mode, and runs the inverse FFT of each
// output.  No workgroup barrier: the waves of a block work on their own
// items.  The spectra keep the layout of the generic kernels ([kx][z], FP32,
// column 0 carrying the DC and Nyquist columns packed; both have kx = 0), so
// these passes combine with the generic x passes.
//
// Two kernels.  wave_z_fused_kernel (every compiled length, one launch over
// all of them) has each wave run both sets of its lines, the second set's
// loads in flight during the first set's inverse transforms: about 460
// registers, one wave per SIMD, speed from the work each wave keeps in
// flight.  wave_z_set_kernel<L> (the lengths at 8 points per lane, one launch
// per length) gives each wave one set of its lines, so that a wave's state
// fits 256 registers and two waves share each SIMD; the other wave hides
// each one's LDS and memory waits.  Both compute every mode the same way, so
// their results are identical.
#include <hip/hip_runtime.h>

#include "groups.hpp"
#include "update.hpp"
#include "wave2d.hpp"
#include "wfft.hpp"

namespace psatd {
namespace wave2d {

__device__ __forceinline__ double2 f2d(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ float2 d2f(double2 v) {
  return make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
}

// Per-item state of a wave: its lines, the lane's position, and the values
// it requests once per item (twiddle bases, kx).
template <int L>
struct ZItem {
  using LN = wfft::Line<L>;
  static constexpr int NP = LN::P;
  static constexpr int S = LN::S;
  const PatchDev* P;
  int g, s;
  bool active;
  // wave-uniform base of the item's first line (scalar registers) and the
  // lane's 32-bit element offset, so that loads and stores address as
  // scalar base + lane offset + immediate
  float2* base;
  int loff;
  long long cs;
  wfft::Twiddles<L> tw;
  double kx;

  __device__ __forceinline__ ZItem(const PatchDev* p, const WorkItem& wi, float* ws, int lane)
      : P(p), g(lane / S), s(lane % S) {
    active = g < wi.count;
    base = reinterpret_cast<float2*>(ws) + P->off_z + static_cast<long long>(wi.first) * L;
    loff = (active ? g : 0) * L + s;  // inactive lanes: a valid line
    cs = P->comp_stride;
    tw.load(P->fz.tw, s);
    kx = gload(P->kx, wi.first + (active ? g : 0));
  }
};

// One polarization set: its inputs' loads (all requested at once), their
// forward transforms and the per-mode update, and the inverse transforms of
// the outputs with their stores.  The phases are separate so that the next
// set's loads can be issued while this set's inverse transforms run.
// BAR: scheduling barriers between the transforms and between the modes, so
// that the compiler does not overlap them (and hold their registers at once);
// for the kernel that runs at two waves per SIMD.
template <int L, int SRC, int GR, bool BAR>
struct ZSet {
  using Gr = Group<GR, SRC>;
  static constexpr int NP = wfft::Line<L>::P;
  static constexpr int NIN = Gr::nin;
  float2 held[NIN][NP];

  __device__ __forceinline__ void load(const ZItem<L>& it) {
    static_for<0, NIN>([&](auto sc) __attribute__((always_inline)) {
      constexpr int slot = decltype(sc)::value;
      const float2* src = it.base + Gr::in[slot] * it.cs;
#pragma unroll
      for (int m = 0; m < NP; ++m) held[slot][m] = src[it.loff + ZItem<L>::S * m];
    });
  }

  // forward transforms one at a time (kept in FP32 until the update), then
  // the update of every mode (kx of the line, kz of mode s + S m)
  __device__ __forceinline__ void forward_update(const ZItem<L>& it, const Physics& ph,
                                                 double2* region) {
    static_for<0, NIN>([&](auto sc) __attribute__((always_inline)) {
      constexpr int slot = decltype(sc)::value;
      double2 v[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) v[m] = f2d(held[slot][m]);
      wfft::fft<L, -1>(v, region, it.g, it.s, it.tw);
#pragma unroll
      for (int m = 0; m < NP; ++m) held[slot][m] = d2f(v[m]);
      if constexpr (BAR) __builtin_amdgcn_sched_barrier(0);
    });
    const double dt = it.P->dt;
    // the modes' kz, requested here rather than held through the transforms
    double kzv[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) kzv[m] = gload(it.P->kz, it.s + ZItem<L>::S * m);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      const double kz = kzv[m];
      double2 E[3] = {}, B[3] = {}, J[3] = {};
      double2 ro = make_double2(0.0, 0.0), rn = make_double2(0.0, 0.0);
      static_for<0, NIN>([&](auto sc) __attribute__((always_inline)) {
        constexpr int slot = decltype(sc)::value;
        constexpr int comp = Gr::in[slot];
        const double2 v = f2d(held[slot][m]);
        if constexpr (comp < 3) E[comp] = v;
        else if constexpr (comp < 6) B[comp - 3] = v;
        else if constexpr (comp < 9) J[comp - 6] = v;
        else if constexpr (comp == kRhoOld) ro = v;
        else rn = v;
      });
      double2 Eo[3], Bo[3];
      if constexpr (src_is_pstd(SRC)) {
        pstd_update_mode<SRC>(it.kx, 0.0, kz, dt, ph.c, ph.eps0, it.P->inv_n, E, B, J, Eo, Bo);
      } else {
        const double K = sqrt(it.kx * it.kx + kz * kz);
        const Coef q = psatd_coef(K, dt, ph.c, ph.eps0, it.P->inv_n);
        update_mode<SRC>(it.kx, 0.0, kz, q, ph.c, ph.eps0, dt, E, B, J, ro, rn, Eo, Bo);
      }
      static_for<0, Gr::nout>([&](auto oc) __attribute__((always_inline)) {
        constexpr int o = decltype(oc)::value;
        constexpr int comp = Gr::in[Gr::out_slot[o]];
        if constexpr (comp < 3) held[Gr::out_slot[o]][m] = d2f(Eo[comp]);
        else held[Gr::out_slot[o]][m] = d2f(Bo[comp - 3]);
      });
      if constexpr (BAR) __builtin_amdgcn_sched_barrier(0);
    }
  }

  // inverse transforms of the outputs, written over their inputs
  __device__ __forceinline__ void inverse_store(const ZItem<L>& it, double2* region) {
    static_for<0, Gr::nout>([&](auto oc) __attribute__((always_inline)) {
      constexpr int o = decltype(oc)::value;
      constexpr int slot = Gr::out_slot[o];
      double2 v[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) v[m] = f2d(held[slot][m]);
      wfft::fft<L, 1>(v, region, it.g, it.s, it.tw);
      if (it.active) {
        float2* dst = it.base + Gr::in[slot] * it.cs;
#pragma unroll
        for (int m = 0; m < NP; ++m) dst[it.loff + ZItem<L>::S * m] = d2f(v[m]);
      }
      if constexpr (BAR) __builtin_amdgcn_sched_barrier(0);
    });
  }
};

template <int L, int SRC>
__device__ __forceinline__ void z_item(const PatchDev* P, const WorkItem& wi, float* ws,
                                       const Physics& ph, double2* region, int lane) {
  const ZItem<L> it(P, wi, ws, lane);
  ZSet<L, SRC, 0, false> s0;
  ZSet<L, SRC, 1, false> s1;
  s0.load(it);
  s0.forward_update(it, ph, region);
  // at 8 points per lane the second set's loads are in flight during the
  // first set's inverse transforms; at 12 the registers are not there
  if constexpr (wfft::Line<L>::P <= 8) s1.load(it);
  s0.inverse_store(it, region);
  if constexpr (wfft::Line<L>::P > 8) s1.load(it);
  s1.forward_update(it, ph, region);
  s1.inverse_store(it, region);
}

template <int SRC>
__global__ void __launch_bounds__(kBlock)
wave_z_fused_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
                    int nitems, float* __restrict__ ws, Physics ph, int region_elems) {
  extern __shared__ double2 lds[];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double2* region = lds + wave * region_elems;
  for (int it = blockIdx.x * kWavesPerBlock + wave; it < nitems; it += gridDim.x * kWavesPerBlock) {
    const WorkItem wi = items[it];
    const PatchDev* P = patches + wi.patch;
    switch (P->nz) {
      case 32: z_item<32, SRC>(P, wi, ws, ph, region, lane); break;
      case 48: z_item<48, SRC>(P, wi, ws, ph, region, lane); break;
      case 64: z_item<64, SRC>(P, wi, ws, ph, region, lane); break;
      case 96: z_item<96, SRC>(P, wi, ws, ph, region, lane); break;
      case 128: z_item<128, SRC>(P, wi, ws, ph, region, lane); break;
      case 192: z_item<192, SRC>(P, wi, ws, ph, region, lane); break;
      case 256: z_item<256, SRC>(P, wi, ws, ph, region, lane); break;
      case 384: z_item<384, SRC>(P, wi, ws, ph, region, lane); break;
      default: z_item<512, SRC>(P, wi, ws, ph, region, lane); break;
    }
  }
}

// One set of one item's lines per wavefront: wave w of the launch takes
// item w / 2 and set w % 2 (the two sets of an item run on neighbouring
// waves).  L has 8 points per lane (z_set_supported).
template <int SRC, int L>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2)))
wave_z_set_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
                  int nitems, float* __restrict__ ws, Physics ph, int region_elems) {
  static_assert(wfft::Line<L>::P == 8, "one set per wave is for 8 points per lane");
  extern __shared__ double2 lds[];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double2* region = lds + wave * region_elems;
  const int nwork = 2 * nitems;
  for (int w = blockIdx.x * kWavesPerBlock + wave; w < nwork; w += gridDim.x * kWavesPerBlock) {
    const WorkItem wi = items[w >> 1];
    const PatchDev* P = patches + wi.patch;
    const ZItem<L> it(P, wi, ws, lane);
    if ((w & 1) == 0) {
      ZSet<L, SRC, 0, true> set;
      set.load(it);
      set.forward_update(it, ph, region);
      set.inverse_store(it, region);
    } else {
      ZSet<L, SRC, 1, true> set;
      set.load(it);
      set.forward_update(it, ph, region);
      set.inverse_store(it, region);
    }
  }
}

bool z_set_supported(int nz) {
  return nz == 32 || nz == 64 || nz == 128 || nz == 256 || nz == 512;
}

bool z_supported(int nz) {
  return nz == 32 || nz == 48 || nz == 64 || nz == 96 || nz == 128 || nz == 192 || nz == 256 ||
         nz == 384 || nz == 512;
}

int z_lines_per_item(int nz) { return 64 / (nz / wfft::points(nz)); }

int z_region(int nz) { return z_lines_per_item(nz) * wfft::stride_of(nz); }

hipError_t launch_z_fused(int src, const LaunchShape& sh, hipStream_t stream,
                          const PatchDev* patches, const WorkItem* items, int nitems, void* ws,
                          Physics ph, int region) {
  float* w = static_cast<float*>(ws);
  switch (src) {
    case kVacuum:
      hipLaunchKernelGGL((wave_z_fused_kernel<kVacuum>), dim3(sh.grid), dim3(kBlock), sh.lds_bytes,
                         stream, patches, items, nitems, w, ph, region);
      break;
    case kPstdVacuum:
      hipLaunchKernelGGL((wave_z_fused_kernel<kPstdVacuum>), dim3(sh.grid), dim3(kBlock),
                         sh.lds_bytes, stream, patches, items, nitems, w, ph, region);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int L>
hipError_t launch_set_len(int src, const LaunchShape& sh, hipStream_t stream,
                          const PatchDev* patches, const WorkItem* items, int nitems, float* w,
                          Physics ph, int region) {
  switch (src) {
    case kVacuum:
      hipLaunchKernelGGL((wave_z_set_kernel<kVacuum, L>), dim3(sh.grid), dim3(kBlock), sh.lds_bytes,
                         stream, patches, items, nitems, w, ph, region);
      break;
    case kPstdVacuum:
      hipLaunchKernelGGL((wave_z_set_kernel<kPstdVacuum, L>), dim3(sh.grid), dim3(kBlock),
                         sh.lds_bytes, stream, patches, items, nitems, w, ph, region);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_z_set(int src, int nz, const LaunchShape& sh, hipStream_t stream,
                        const PatchDev* patches, const WorkItem* items, int nitems, void* ws,
                        Physics ph, int region) {
  float* w = static_cast<float*>(ws);
  switch (nz) {
    case 32: return launch_set_len<32>(src, sh, stream, patches, items, nitems, w, ph, region);
    case 64: return launch_set_len<64>(src, sh, stream, patches, items, nitems, w, ph, region);
    case 128: return launch_set_len<128>(src, sh, stream, patches, items, nitems, w, ph, region);
    case 256: return launch_set_len<256>(src, sh, stream, patches, items, nitems, w, ph, region);
    case 512: return launch_set_len<512>(src, sh, stream, patches, items, nitems, w, ph, region);
    default: return hipErrorInvalidValue;
  }
}

hipError_t configure_attributes() {
  const int lim = 160 * 1024;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&wave_z_fused_kernel<kVacuum>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void*>(&wave_z_fused_kernel<kPstdVacuum>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  return e != hipSuccess ? e : r;
}

}  // namespace wave2d
}  // namespace psatd
