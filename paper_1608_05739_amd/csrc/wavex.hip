// Wave-resident x passes for batched 2D patches (FP32 storage, FP64
// arithmetic): the r2c transform of the field rows into the [kx][z] spectra
// and the c2r transform back.
//
// A workgroup of kWavesPerBlock wavefronts takes a tile of T = 4 G
// consecutive rows z of one component of one patch (G rows per wave, as the
// wave-resident FFT lays them out: lane s of row g holds points s + S m).
// Each wave transforms its rows in registers with exchanges through its own
// LDS region (wfft.hpp, no workgroup barrier inside the transform).  The
// spectra are column-major ([kx][z]), so the tile crosses the workgroup once
// through LDS: T consecutive z per kx, written (or read) as runs of T complex
// values.  One workgroup barrier per tile on each side of that crossing.
//
// Forward: rows packed as complex c[j] = x[2j] + i x[2j+1] (length
// L = nx / 2), FFT of length L, then the r2c split
//   X[k] = e + W^k o,  e = (Z[k] + conj Z[L-k]) / 2,  o = -i (Z[k] - conj Z[L-k]) / 2,
// W = exp(-2 pi i / nx), with the Nyquist value packed into column 0 as
// (Re Z0 + Im Z0) + i (Re Z0 - Im Z0).  Inverse: the adjoint pre-step, then
// the inverse FFT (no 1/N: the update carries it) and the rows unpacked.
#include <hip/hip_runtime.h>

#include "wave2d.hpp"
#include "wfft.hpp"

namespace psatd {
namespace wave2d {

namespace {

__device__ __forceinline__ double2 f2d(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ float2 d2f(double2 v) {
  return make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
}

// Rows per tile and the FP32 staging layout of a wave's rows inside its
// region: row g, column k at g (L + 1) + k (float2 units; the odd row stride
// keeps the column-wise reads of the crossing free of bank conflicts).
template <int L>
struct XTile {
  static constexpr int G = wfft::Line<L>::G;
  static constexpr int T = kWavesPerBlock * G;
  static constexpr int ROW = L + 1;
  static_assert(G * ROW <= 2 * wfft::Line<L>::REGION, "staging fits the region");
  static_assert((T & (T - 1)) == 0, "rows per tile a power of two");
};

// Partner index L - k of the r2c split (k = 0 pairs with itself).
template <int L>
__device__ __forceinline__ int partner(int k) {
  return k == 0 ? 0 : L - k;
}

template <int L>
__device__ void x_fwd_tile(const PatchDev* __restrict__ P, const WorkItem& wi,
                           const FieldPtrs& fields, float* __restrict__ ws, double2* lds) {
  using LN = wfft::Line<L>;
  using XT = XTile<L>;
  constexpr int NP = LN::P;
  constexpr int S = LN::S;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int g = lane / S;
  const int s = lane % S;
  double2* const region = lds + wave * LN::REGION;
  const int row = wave * XT::G + g;
  const bool active = row < wi.count;
  const int z = wi.first + (active ? row : 0);  // idle rows read a valid row

  // rows: point j of row z is the complex pair (x[2j], x[2j+1])
  const float2* src = reinterpret_cast<const float2*>(
                          static_cast<const float*>(field_ptr(fields, wi.comp)) + P->off_real) +
                      static_cast<long long>(z) * L;
  wfft::Twiddles<L> tws;
  tws.load(P->fx.tw, s);
  double2 v[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) v[m] = f2d(src[s + S * m]);
  wfft::fft<L, -1>(v, region, g, s, tws);

  // r2c split: every lane needs Z[L - k] of its own k, held by another lane
  double2* const line = region + g * LN::STRIDE;
#pragma unroll
  for (int m = 0; m < NP; ++m) line[wfft::pa(s + S * m)] = v[m];
  wfft::wave_sync();
  float2 out[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int k = s + S * m;
    const double2 a = v[m];
    if (k == 0) {
      out[m] = d2f(make_double2(a.x + a.y, a.x - a.y));
    } else {
      const double2 b = line[wfft::pa(partner<L>(k))];
      const double2 e = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      const double2 d = make_double2(a.x - b.x, a.y + b.y);
      const double2 o = make_double2(0.5 * d.y, -0.5 * d.x);
      out[m] = d2f(cadd(e, cmul(gload(P->post, k), o)));
    }
  }
  wfft::wave_sync();  // every partner read is done before the staging overwrites the region
  float2* const stg = reinterpret_cast<float2*>(region);
#pragma unroll
  for (int m = 0; m < NP; ++m) stg[g * XT::ROW + s + S * m] = out[m];
  __syncthreads();

  // the crossing: T consecutive z of each kx, as runs of T complex values
  float2* const spec = reinterpret_cast<float2*>(ws) + P->off_spec +
                       static_cast<long long>(wi.comp) * P->comp_stride;
  const int nz = P->nz;
  constexpr int total = XT::T * L;
#pragma unroll 4
  for (int idx = tid; idx < total; idx += kBlock) {
    const int zl = idx & (XT::T - 1);
    const int kx = idx / XT::T;
    if (zl < wi.count) {
      const float2* w = reinterpret_cast<const float2*>(lds + (zl / XT::G) * LN::REGION);
      spec[static_cast<long long>(kx) * nz + wi.first + zl] = w[(zl % XT::G) * XT::ROW + kx];
    }
  }
  __syncthreads();  // the regions are reused by the next tile
}

template <int L>
__device__ void x_inv_tile(const PatchDev* __restrict__ P, const WorkItem& wi,
                           const FieldPtrs& fields, float* __restrict__ ws, double2* lds) {
  using LN = wfft::Line<L>;
  using XT = XTile<L>;
  constexpr int NP = LN::P;
  constexpr int S = LN::S;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int g = lane / S;
  const int s = lane % S;
  double2* const region = lds + wave * LN::REGION;
  const int row = wave * XT::G + g;
  const bool active = row < wi.count;

  // the crossing: runs of T consecutive z of each kx into the rows' staging
  const float2* const spec = reinterpret_cast<const float2*>(ws) + P->off_spec +
                             static_cast<long long>(wi.comp) * P->comp_stride;
  const int nz = P->nz;
  constexpr int total = XT::T * L;
#pragma unroll 4
  for (int idx = tid; idx < total; idx += kBlock) {
    const int zl = idx & (XT::T - 1);
    const int kx = idx / XT::T;
    if (zl < wi.count) {
      float2* w = reinterpret_cast<float2*>(lds + (zl / XT::G) * LN::REGION);
      w[(zl % XT::G) * XT::ROW + kx] = spec[static_cast<long long>(kx) * nz + wi.first + zl];
    }
  }
  __syncthreads();

  wfft::Twiddles<L> tws;
  tws.load(P->fx.tw, s);
  // c2r pre-step from the staged row (both k and L - k are there)
  const float2* const stg = reinterpret_cast<const float2*>(region) + g * XT::ROW;
  double2 v[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int k = s + S * m;
    const double2 a = f2d(stg[k]);
    if (k == 0) {
      v[m] = make_double2(a.x + a.y, a.x - a.y);
    } else {
      const double2 b = f2d(stg[partner<L>(k)]);
      const double2 p = make_double2(a.x + b.x, a.y - b.y);
      const double2 d = make_double2(a.x - b.x, a.y + b.y);
      const double2 t1 = cmul(cconj(gload(P->post, k)), d);
      v[m] = make_double2(p.x - t1.y, p.y + t1.x);
    }
  }
  wfft::wave_sync();  // staged values read before the transform reuses the region
  wfft::fft<L, 1>(v, region, g, s, tws);
  if (active) {
    float2* dst = reinterpret_cast<float2*>(static_cast<float*>(field_ptr(fields, wi.comp)) +
                                            P->off_real) +
                  static_cast<long long>(wi.first + row) * L;
#pragma unroll
    for (int m = 0; m < NP; ++m) dst[s + S * m] = d2f(v[m]);
  }
  __syncthreads();  // the regions are reused by the next tile
}

// One kernel per row length and direction; a pass launches one per length.
template <int KIND, int L>
__global__ void __launch_bounds__(kBlock)
wave_x_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items, int nitems,
              FieldPtrs fields, float* __restrict__ ws) {
  extern __shared__ double2 lds[];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[xcd_local_order(it, nitems)];
    if constexpr (KIND == kXFwd) {
      x_fwd_tile<L>(patches + wi.patch, wi, fields, ws, lds);
    } else {
      x_inv_tile<L>(patches + wi.patch, wi, fields, ws, lds);
    }
  }
}

template <int KIND>
hipError_t launch_kind(int L, const LaunchShape& sh, hipStream_t stream, const PatchDev* patches,
                       const WorkItem* items, int nitems, const FieldPtrs& f, float* w) {
#define PSATD_WX_CASE(LEN)                                                                     \
  case LEN:                                                                                    \
    hipLaunchKernelGGL((wave_x_kernel<KIND, LEN>), dim3(sh.grid), dim3(kBlock), sh.lds_bytes,  \
                       stream, patches, items, nitems, f, w);                                  \
    break;
  switch (L) {
    PSATD_WX_CASE(32) PSATD_WX_CASE(48) PSATD_WX_CASE(64) PSATD_WX_CASE(96) PSATD_WX_CASE(128)
    PSATD_WX_CASE(192) PSATD_WX_CASE(256) PSATD_WX_CASE(384) PSATD_WX_CASE(512)
    default:
      return hipErrorInvalidValue;
  }
#undef PSATD_WX_CASE
  return hipGetLastError();
}

template <int KIND, int L>
hipError_t set_x_lds_limit() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&wave_x_kernel<KIND, L>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <int KIND>
hipError_t configure_kind() {
  const hipError_t r[] = {set_x_lds_limit<KIND, 32>(),  set_x_lds_limit<KIND, 48>(),
                          set_x_lds_limit<KIND, 64>(),  set_x_lds_limit<KIND, 96>(),
                          set_x_lds_limit<KIND, 128>(), set_x_lds_limit<KIND, 192>(),
                          set_x_lds_limit<KIND, 256>(), set_x_lds_limit<KIND, 384>(),
                          set_x_lds_limit<KIND, 512>()};
  for (hipError_t e : r)
    if (e != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace

bool x_supported(int L) { return z_supported(L); }

int x_rows_per_item(int L) { return kWavesPerBlock * z_lines_per_item(L); }

hipError_t launch_x(int kind, int L, const LaunchShape& sh, hipStream_t stream,
                    const PatchDev* patches, const WorkItem* items, int nitems,
                    const FieldPtrs& fields, void* ws) {
  float* w = static_cast<float*>(ws);
  if (kind == kXFwd) return launch_kind<kXFwd>(L, sh, stream, patches, items, nitems, fields, w);
  if (kind == kXInv) return launch_kind<kXInv>(L, sh, stream, patches, items, nitems, fields, w);
  return hipErrorInvalidValue;
}

hipError_t configure_x_attributes() {
  const hipError_t e = configure_kind<kXFwd>();
  return e != hipSuccess ? e : configure_kind<kXInv>();
}

}  // namespace wave2d
}  // namespace psatd
