// Wave-resident fused z pass for 3D patches (FP32 storage, FP64 arithmetic),
// PSATD forms (vacuum, rho form, J form), z lines of 32 to 512 points.
//
// One wavefront per work item of G z lines of the [kx][y][z] spectra (line
// l = kx ny + y; lane s of line g holds modes z = s + S m, wfft.hpp).  In 3D
// every component couples with every other, so instead of holding all
// transformed inputs the wave accumulates the six outputs: each input is
// loaded, transformed, and its contribution to each output (the update is
// linear in the inputs) added mode by mode into the accumulators; then the
// six outputs are transformed back and stored over E and B.  The per-mode
// coefficients C, S, X1, X2, X3 are evaluated once per item and kept in LDS.  Each
// contribution is formed in FP64 and added to FP32 accumulators (the
// registers of FP64 ones are not there), one rounding per contribution.  With
// E' = C E + i c^2 S (k x B) - (S / eps0) J + i k (X3 rho_old - X2 rho_new)
// and B' = C B - i S (k x E) + i X1 (k x J) (rho form; the J form replaces the
// rho term by eps0 c^2 X1 k (k . E) - dt X2 k (k . J)), input by input:
//   E_a  -> E'_a += C E_a;  B' += -i S (k x e_a) E_a
//   B_a  -> B'_a += C B_a;  E' += i c^2 S (k x e_a) B_a
//   J_a  -> E'_a += -(S / eps0) J_a;  B' += i X1 (k x e_a) J_a
//   rho_old -> E' += i X3 k rho_old,  rho_new -> E' += -i X2 k rho_new
// (J form: E_a -> E' += eps0 c^2 X1 k_a k E_a,  J_a -> E' += -dt X2 k_a k J_a).
#include <hip/hip_runtime.h>

#include "update.hpp"
#include "wave2d.hpp"
#include "wfft.hpp"

namespace psatd {
namespace wave2d {

namespace {

__device__ __forceinline__ double2 f2d(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ float2 d2f(double2 v) {
  return make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
}
// acc += a z,  acc += i a z  (FP32 accumulator, FP64 product and sum)
__device__ __forceinline__ void add_re(float2& acc, double a, double2 z) {
  acc.x = static_cast<float>(fma(a, z.x, static_cast<double>(acc.x)));
  acc.y = static_cast<float>(fma(a, z.y, static_cast<double>(acc.y)));
}
__device__ __forceinline__ void add_im(float2& acc, double a, double2 z) {
  acc.x = static_cast<float>(fma(-a, z.y, static_cast<double>(acc.x)));
  acc.y = static_cast<float>(fma(a, z.x, static_cast<double>(acc.y)));
}

template <int NP>
__device__ __forceinline__ void take(double2 (&v)[NP], const float2 (&a)[NP]) {
#pragma unroll
  for (int m = 0; m < NP; ++m) v[m] = f2d(a[m]);
}

// The contribution of input c (transformed: v) to the accumulated outputs,
// mode by mode; coef holds the mode's C, S, X1, X2, X3 and kz (see z3_item).
template <int SRC, int c, int NP>
__device__ __forceinline__ void contribute(float2 (&E)[3][NP], float2 (&B)[3][NP],
                                           const double2 (&v)[NP], const double* coef, double kx,
                                           double ky, double c2, double dt, double eps0,
                                           double ie0) {
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const double k[3] = {kx, ky, coef[(5 * NP + m) * 64]};
    const double Cm = coef[(0 * NP + m) * 64], Sm = coef[(1 * NP + m) * 64];
    const double2 z = v[m];
    if constexpr (c < 3) {
      // E_c: C E_c, and B' -= i S (k x e_c) E_c with k x e_c = k_{c+2} e_{c+1} - k_{c+1} e_{c+2}
      constexpr int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
      add_re(E[c][m], Cm, z);
      add_im(B[a1][m], -Sm * k[a2], z);
      add_im(B[a2][m], Sm * k[a1], z);
      if constexpr (SRC == kJForm) {
        const double f = eps0 * c2 * coef[(2 * NP + m) * 64] * k[c];
#pragma unroll
        for (int a = 0; a < 3; ++a) add_re(E[a][m], f * k[a], z);
      }
    } else if constexpr (c < 6) {
      constexpr int b = c - 3, a1 = (b + 1) % 3, a2 = (b + 2) % 3;
      const double cS = c2 * Sm;
      add_re(B[b][m], Cm, z);
      add_im(E[a1][m], cS * k[a2], z);
      add_im(E[a2][m], -cS * k[a1], z);
    } else if constexpr (c < 9) {
      constexpr int j = c - 6, a1 = (j + 1) % 3, a2 = (j + 2) % 3;
      const double X1m = coef[(2 * NP + m) * 64];
      add_re(E[j][m], -Sm * ie0, z);
      add_im(B[a1][m], X1m * k[a2], z);
      add_im(B[a2][m], -X1m * k[a1], z);
      if constexpr (SRC == kJForm) {
        const double f = -dt * coef[(3 * NP + m) * 64] * k[j];
#pragma unroll
        for (int a = 0; a < 3; ++a) add_re(E[a][m], f * k[a], z);
      }
    } else {
      const double f = c == kRhoOld ? coef[(4 * NP + m) * 64] : -coef[(3 * NP + m) * 64];
#pragma unroll
      for (int a = 0; a < 3; ++a) add_im(E[a][m], f * k[a], z);
    }
  }
}

template <int L, int SRC>
__device__ __forceinline__ void z3_item(const PatchDev* __restrict__ P, const WorkItem& wi,
                                        float* __restrict__ ws, const Physics& ph,
                                        double2* region, int lane) {
  using LN = wfft::Line<L>;
  constexpr int NP = LN::P;
  constexpr int S = LN::S;
  constexpr int NIN = SRC == kVacuum ? 6 : (SRC == kRho ? 11 : 9);
  const int g = lane / S;
  const int s = lane % S;
  const bool active = g < wi.count;
  const int line = wi.first + (active ? g : 0);  // inactive lanes: a valid line
  float2* const base = reinterpret_cast<float2*>(ws) + P->off_z + static_cast<long long>(wi.first) * L;
  const int loff = (active ? g : 0) * L + s;
  const long long cs = P->comp_stride;

  wfft::Twiddles<L> tw;
  tw.load(P->fz.tw, s);
  int ix, iy;
  udivmod(line, P->ny, ix, iy);
  const double kx = gload(P->kx, ix);
  const double ky = gload(P->ky, iy);
  const double dt = P->dt;
  const double c2 = ph.c * ph.c;

  // per-mode coefficients C, S, X1, X2, X3 and kz, evaluated once and kept
  // in the wave's LDS after its exchange region: coefficient q of mode m of
  // this lane at coef[(q P + m) 64] (consecutive lanes, consecutive banks)
  const double ie0 = 1.0 / ph.eps0;
  double* const coef = reinterpret_cast<double*>(region + LN::REGION) + lane;
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const double kz = gload(P->kz, s + S * m);
    const double K = sqrt(kx * kx + ky * ky + kz * kz);
    const Coef q = psatd_coef(K, dt, ph.c, ph.eps0, P->inv_n);
    coef[(0 * NP + m) * 64] = q.C;
    coef[(1 * NP + m) * 64] = q.S;
    coef[(2 * NP + m) * 64] = q.X1;
    coef[(3 * NP + m) * 64] = q.X2;
    coef[(4 * NP + m) * 64] = q.X3;
    coef[(5 * NP + m) * 64] = kz;
  }

  float2 E[3][NP], B[3][NP];  // accumulated outputs
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      E[a][m] = make_float2(0.f, 0.f);
      B[a][m] = make_float2(0.f, 0.f);
    }

  // inputs one at a time, in a loop that is not unrolled (so that one
  // transform's code serves every input and the scheduler cannot hold
  // several inputs' transforms at once); the next input's loads are issued
  // before this input's transform
  float2 nxt[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) nxt[m] = base[loff + S * m];
#pragma unroll 1
  for (int c = 0; c < NIN; ++c) {
    double2 v[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) v[m] = f2d(nxt[m]);
    if (c + 1 < NIN) {
      const float2* src = base + (c + 1) * cs;
#pragma unroll
      for (int m = 0; m < NP; ++m) nxt[m] = src[loff + S * m];
    }
    wfft::fft<L, -1>(v, region, g, s, tw);
    switch (c) {
      case 0: contribute<SRC, 0, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      case 1: contribute<SRC, 1, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      case 2: contribute<SRC, 2, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      case 3: contribute<SRC, 3, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      case 4: contribute<SRC, 4, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      case 5: contribute<SRC, 5, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      case 6: contribute<SRC, 6, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      case 7: contribute<SRC, 7, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      case 8: contribute<SRC, 8, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      case 9: contribute<SRC, 9, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
      default: contribute<SRC, 10, NP>(E, B, v, coef, kx, ky, c2, dt, ph.eps0, ie0); break;
    }
  }

  // the six outputs back along z, over E and B (one transform's code)
#pragma unroll 1
  for (int o = 0; o < 6; ++o) {
    double2 v[NP];
    switch (o) {
      case 0: take(v, E[0]); break;
      case 1: take(v, E[1]); break;
      case 2: take(v, E[2]); break;
      case 3: take(v, B[0]); break;
      case 4: take(v, B[1]); break;
      default: take(v, B[2]); break;
    }
    wfft::fft<L, 1>(v, region, g, s, tw);
    if (active) {
      float2* dst = base + o * cs;
#pragma unroll
      for (int m = 0; m < NP; ++m) dst[loff + S * m] = d2f(v[m]);
    }
  }
}

template <int SRC>
__global__ void __launch_bounds__(kBlock)
wave_z3_fused_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
                     int nitems, float* __restrict__ ws, Physics ph, int region_elems) {
  extern __shared__ double2 lds[];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double2* region = lds + wave * region_elems;
  for (int it = blockIdx.x * kWavesPerBlock + wave; it < nitems; it += gridDim.x * kWavesPerBlock) {
    const WorkItem wi = items[it];
    const PatchDev* P = patches + wi.patch;
    switch (P->nz) {
      case 32: z3_item<32, SRC>(P, wi, ws, ph, region, lane); break;
      case 64: z3_item<64, SRC>(P, wi, ws, ph, region, lane); break;
      case 128: z3_item<128, SRC>(P, wi, ws, ph, region, lane); break;
      case 256: z3_item<256, SRC>(P, wi, ws, ph, region, lane); break;
      default: z3_item<512, SRC>(P, wi, ws, ph, region, lane); break;
    }
  }
}

template <int SRC>
hipError_t set_z3_lds_limit() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&wave_z3_fused_kernel<SRC>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

}  // namespace

bool z3_supported(int nz) { return nz == 32 || nz == 64 || nz == 128 || nz == 256 || nz == 512; }

int z3_region(int nz) {
  // the exchange region and six FP64 values per mode and lane (in double2)
  return z_lines_per_item(nz) * wfft::stride_of(nz) + 6 * wfft::points(nz) * 64 / 2;
}

hipError_t launch_z3_fused(int src, const LaunchShape& sh, hipStream_t stream,
                           const PatchDev* patches, const WorkItem* items, int nitems, void* ws,
                           Physics ph, int region) {
  float* w = static_cast<float*>(ws);
  switch (src) {
    case kVacuum:
      hipLaunchKernelGGL((wave_z3_fused_kernel<kVacuum>), dim3(sh.grid), dim3(kBlock),
                         sh.lds_bytes, stream, patches, items, nitems, w, ph, region);
      break;
    case kRho:
      hipLaunchKernelGGL((wave_z3_fused_kernel<kRho>), dim3(sh.grid), dim3(kBlock), sh.lds_bytes,
                         stream, patches, items, nitems, w, ph, region);
      break;
    case kJForm:
      hipLaunchKernelGGL((wave_z3_fused_kernel<kJForm>), dim3(sh.grid), dim3(kBlock),
                         sh.lds_bytes, stream, patches, items, nitems, w, ph, region);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t configure_z3_attributes() {
  const hipError_t r[] = {set_z3_lds_limit<kVacuum>(), set_z3_lds_limit<kRho>(),
                          set_z3_lds_limit<kJForm>()};
  for (hipError_t e : r)
    if (e != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace wave2d
}  // namespace psatd
