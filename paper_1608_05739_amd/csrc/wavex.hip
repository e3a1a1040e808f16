// Wave-resident x passes for batched 2D patches (FP32 storage, FP64
// arithmetic): the r2c transform of the field rows into the [kx][z] spectra
// and the c2r transform back.
//
// A workgroup of W wavefronts takes a tile of T = W G consecutive rows of one
// component of one patch (G rows per wave, as the wave-resident FFT lays them
// out: lane s of row g holds points s + S m; W = 8 where G <= 2, else 4, so
// that T >= 16 rows: runs of 128 bytes in the crossing, FP32).
// Row r of a patch is z in 2D and z ny + y in 3D; a tile never leaves its
// run of A = nz (2D) or ny (3D) rows, and column kx of row r = p A + a sits at
// p mx A + kx A + a of the spectra ([kx][z] in 2D, [z][kx][y] in 3D).
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
  static constexpr int W = G <= 2 ? 8 : 4;  // waves per workgroup
  static constexpr int NT = 64 * W;         // threads per workgroup
  static constexpr int T = W * G;
  static constexpr int ROW = L + 1;
  static_assert(G * ROW <= 2 * wfft::Line<L>::REGION, "staging fits the region");
  static_assert((T & (T - 1)) == 0, "rows per tile a power of two");
};

// Rows of one run of the spectra layout (see above) and the start of the
// tile's run in the spectra: p mx A + a0 for the tile's first row p A + a0.
__device__ __forceinline__ int run_rows(const PatchDev* P) { return P->ndim == 2 ? P->nz : P->ny; }
__device__ __forceinline__ long long tile_start(const PatchDev* P, int first) {
  const int A = run_rows(P);
  int p, a0;
  udivmod(first, A, p, a0);
  return static_cast<long long>(p) * P->mx * A + a0;
}

// Partner index L - k of the r2c split (k = 0 pairs with itself).
template <int L>
__device__ __forceinline__ int partner(int k) {
  return k == 0 ? 0 : L - k;
}

// cos and sin of pi m / P (m < P) for the points per lane P = 8, 12, 16,
// from first-octant constants, so that the symmetries hold exactly.
constexpr double kC12 = 0.96592582628906828675;  // cos(pi/12)
constexpr double kS12 = 0.25881904510252076235;  // sin(pi/12)
constexpr double kCa = 0.98078528040323044913;   // cos(pi/16)
constexpr double kSa = 0.19509032201612826785;   // sin(pi/16)
constexpr double kCb = 0.83146961230254523708;   // cos(3 pi/16)
constexpr double kSb = 0.55557023301960222474;   // sin(3 pi/16)
template <int P>
constexpr double cos_pm(int m) {
  if constexpr (P == 8) {
    constexpr double t[8] = {1.0, kC1, kR2, kS1, 0.0, -kS1, -kR2, -kC1};
    return t[m];
  } else if constexpr (P == 12) {
    constexpr double t[12] = {1.0, kC12, kH3, kR2, 0.5, kS12, 0.0, -kS12, -0.5, -kR2, -kH3, -kC12};
    return t[m];
  } else {
    static_assert(P == 16, "points per lane");
    constexpr double t[16] = {1.0, kCa, kC1, kCb, kR2, kSb, kS1, kSa,
                              0.0, -kSa, -kS1, -kSb, -kR2, -kCb, -kC1, -kCa};
    return t[m];
  }
}
template <int P>
constexpr double sin_pm(int m) {
  if constexpr (P == 8) {
    constexpr double t[8] = {0.0, kS1, kR2, kC1, 1.0, kC1, kR2, kS1};
    return t[m];
  } else if constexpr (P == 12) {
    constexpr double t[12] = {0.0, kS12, 0.5, kR2, kH3, kC12, 1.0, kC12, kH3, kR2, 0.5, kS12};
    return t[m];
  } else {
    constexpr double t[16] = {0.0, kSa, kS1, kSb, kR2, kCb, kC1, kCa,
                              1.0, kCa, kC1, kCb, kR2, kSb, kS1, kSa};
    return t[m];
  }
}

// Every entry lies on the unit circle, and the angle doubles where the
// tables overlap (pi m / 8 = pi 2m / 16, pi m / 6 = pi 2m / 12).
template <int P>
constexpr bool half_turn_tables_ok() {
  for (int m = 0; m < P; ++m) {
    const double r = cos_pm<P>(m) * cos_pm<P>(m) + sin_pm<P>(m) * sin_pm<P>(m) - 1.0;
    if (r > 4e-16 || r < -4e-16) return false;
  }
  return true;
}
static_assert(half_turn_tables_ok<8>() && half_turn_tables_ok<12>() && half_turn_tables_ok<16>(),
              "cos / sin of pi m / P");
static_assert(cos_pm<8>(3) == cos_pm<16>(6) && sin_pm<8>(5) == sin_pm<16>(10) &&
                  cos_pm<12>(4) == 0.5 && sin_pm<12>(2) == 0.5,
              "cos / sin of pi m / P");

// The r2c post-twiddle W^k = exp(-i pi k / L) of the lane's point m
// (k = s + S m): W^s, one read of the plan's table, times exp(-i pi m / P),
// a constant (S P = L).
template <int P>
__device__ __forceinline__ double2 post_twiddle(double2 ws, int m) {
  return m == 0 ? ws : cmul(ws, make_double2(cos_pm<P>(m), -sin_pm<P>(m)));
}

template <int L>
__device__ void x_fwd_tile(const PatchDev* __restrict__ P, const WorkItem& wi,
                           const FieldPtrs& fields, float* __restrict__ ws, double2* lds,
                           const wfft::Twiddles<L>& tws) {
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
  double2 v[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) v[m] = f2d(src[s + S * m]);
  wfft::fft<L, -1>(v, region, g, s, tws);

  // r2c split: every lane needs Z[L - k] of its own k, held by another lane
  double2* const line = region + g * LN::STRIDE;
#pragma unroll
  for (int m = 0; m < NP; ++m) line[wfft::pa(s + S * m)] = v[m];
  wfft::wave_sync();
  const double2 wpost = gload(P->post, s);
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
      out[m] = d2f(cadd(e, cmul(post_twiddle<NP>(wpost, m), o)));
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
  const int A = run_rows(P);
  float2* const dst = spec + tile_start(P, wi.first);
  constexpr int total = XT::T * L;
#pragma unroll 4
  for (int idx = tid; idx < total; idx += XT::NT) {
    const int zl = idx & (XT::T - 1);
    const int kx = idx / XT::T;
    if (zl < wi.count) {
      const float2* w = reinterpret_cast<const float2*>(lds + (zl / XT::G) * LN::REGION);
      dst[static_cast<long long>(kx) * A + zl] = w[(zl % XT::G) * XT::ROW + kx];
    }
  }
  __syncthreads();  // the regions are reused by the next tile
}

template <int L>
__device__ void x_inv_tile(const PatchDev* __restrict__ P, const WorkItem& wi,
                           const FieldPtrs& fields, float* __restrict__ ws, double2* lds,
                           const wfft::Twiddles<L>& tws) {
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
  const int A = run_rows(P);
  const float2* const in = spec + tile_start(P, wi.first);
  constexpr int total = XT::T * L;
#pragma unroll 4
  for (int idx = tid; idx < total; idx += XT::NT) {
    const int zl = idx & (XT::T - 1);
    const int kx = idx / XT::T;
    if (zl < wi.count) {
      float2* w = reinterpret_cast<float2*>(lds + (zl / XT::G) * LN::REGION);
      w[(zl % XT::G) * XT::ROW + kx] = in[static_cast<long long>(kx) * A + zl];
    }
  }
  __syncthreads();

  // c2r pre-step from the staged row (both k and L - k are there)
  const float2* const stg = reinterpret_cast<const float2*>(region) + g * XT::ROW;
  const double2 wpost = gload(P->post, s);
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
      const double2 t1 = cmul(cconj(post_twiddle<NP>(wpost, m)), d);
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

// y passes (3D): lines along y, length L = ny.  A tile is T consecutive z
// of one kx (line l = kx nz + z); the forward pass reads each line from the
// x pass's [z][kx][y] block and writes runs of T consecutive z per (kx, y)
// into the [kx][y][z] block of the z passes; the inverse pass the reverse.
template <int L, int SIGN>
__device__ void y_tile(const PatchDev* __restrict__ P, const WorkItem& wi, float* __restrict__ ws,
                       double2* lds, const wfft::Twiddles<L>& tws) {
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
  const int nz = P->nz;
  int kx, z0;
  udivmod(wi.first, nz, kx, z0);
  const int z = z0 + (active ? row : 0);  // idle rows read a valid line
  float2* const blk_x = reinterpret_cast<float2*>(ws) + P->off_spec +
                        static_cast<long long>(wi.comp) * P->comp_stride;
  float2* const blk_z = reinterpret_cast<float2*>(ws) + P->off_z +
                        static_cast<long long>(wi.comp) * P->comp_stride;
  // [z][kx][y]: line (kx, z) at (z mx + kx) L;  [kx][y][z]: (kx, y, z) at (kx L + y) nz + z
  float2* const yline = blk_x + (static_cast<long long>(z) * P->mx + kx) * L;
  float2* const zrun = blk_z + static_cast<long long>(kx) * L * nz + z0;
  constexpr int total = XT::T * L;
  double2 v[NP];
  if constexpr (SIGN < 0) {
#pragma unroll
    for (int m = 0; m < NP; ++m) v[m] = f2d(yline[s + S * m]);
    wfft::fft<L, -1>(v, region, g, s, tws);
    wfft::wave_sync();  // the transform's last reads are done before the staging
    float2* const stg = reinterpret_cast<float2*>(region);
#pragma unroll
    for (int m = 0; m < NP; ++m) stg[g * XT::ROW + s + S * m] = d2f(v[m]);
    __syncthreads();
#pragma unroll 4
    for (int idx = tid; idx < total; idx += XT::NT) {
      const int zl = idx & (XT::T - 1);
      const int y = idx / XT::T;
      if (zl < wi.count) {
        const float2* w = reinterpret_cast<const float2*>(lds + (zl / XT::G) * LN::REGION);
        zrun[static_cast<long long>(y) * nz + zl] = w[(zl % XT::G) * XT::ROW + y];
      }
    }
  } else {
#pragma unroll 4
    for (int idx = tid; idx < total; idx += XT::NT) {
      const int zl = idx & (XT::T - 1);
      const int y = idx / XT::T;
      if (zl < wi.count) {
        float2* w = reinterpret_cast<float2*>(lds + (zl / XT::G) * LN::REGION);
        w[(zl % XT::G) * XT::ROW + y] = zrun[static_cast<long long>(y) * nz + zl];
      }
    }
    __syncthreads();
    const float2* const stg = reinterpret_cast<const float2*>(region) + g * XT::ROW;
#pragma unroll
    for (int m = 0; m < NP; ++m) v[m] = f2d(stg[s + S * m]);
    wfft::wave_sync();  // staged values read before the transform reuses the region
    wfft::fft<L, 1>(v, region, g, s, tws);
    if (active) {
#pragma unroll
      for (int m = 0; m < NP; ++m) yline[s + S * m] = d2f(v[m]);
    }
  }
  __syncthreads();  // the regions are reused by the next tile
}

// One kernel per line length and pass kind; a pass launches one per length.
template <int KIND, int L>
__global__ void __launch_bounds__(512)
wave_x_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items, int nitems,
              FieldPtrs fields, float* __restrict__ ws) {
  extern __shared__ double2 lds[];
  if (static_cast<int>(blockIdx.x) >= nitems) return;
  // The twiddle bases depend only on the length and the lane's position, and
  // every item of this launch has length L.  The forward passes up to 512
  // points keep one set for the whole launch (measured faster); the others
  // request them per tile (holding them cost the inverse passes time, and the
  // 1024-point kernels a wave per SIMD).
  constexpr bool kHold = (KIND == kXFwd || KIND == kYFwd) && L <= 512;
  const int s = (threadIdx.x & 63) % wfft::Line<L>::S;
  wfft::Twiddles<L> tws;
  if constexpr (kHold) {
    const PatchDev* P0 = patches + items[0].patch;
    tws.load(KIND == kYFwd ? P0->fy.tw : P0->fx.tw, s);
  }
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[xcd_local_order(it, nitems)];
    if constexpr (!kHold) {
      const PatchDev* Pi = patches + wi.patch;
      tws.load(KIND == kYFwd || KIND == kYInv ? Pi->fy.tw : Pi->fx.tw, s);
    }
    if constexpr (KIND == kXFwd) {
      x_fwd_tile<L>(patches + wi.patch, wi, fields, ws, lds, tws);
    } else if constexpr (KIND == kXInv) {
      x_inv_tile<L>(patches + wi.patch, wi, fields, ws, lds, tws);
    } else {
      y_tile<L, KIND == kYFwd ? -1 : 1>(patches + wi.patch, wi, ws, lds, tws);
    }
  }
}

template <int KIND>
hipError_t launch_kind(int L, const LaunchShape& sh, hipStream_t stream, const PatchDev* patches,
                       const WorkItem* items, int nitems, const FieldPtrs& f, float* w) {
#define PSATD_WX_CASE(LEN)                                                                     \
  case LEN:                                                                                    \
    hipLaunchKernelGGL((wave_x_kernel<KIND, LEN>), dim3(sh.grid), dim3(XTile<LEN>::NT),        \
                       sh.lds_bytes,                                                           \
                       stream, patches, items, nitems, f, w);                                  \
    break;
  switch (L) {
    PSATD_WX_CASE(32) PSATD_WX_CASE(48) PSATD_WX_CASE(64) PSATD_WX_CASE(96) PSATD_WX_CASE(128)
    PSATD_WX_CASE(192) PSATD_WX_CASE(256) PSATD_WX_CASE(384) PSATD_WX_CASE(512)
    PSATD_WX_CASE(1024)
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
                          set_x_lds_limit<KIND, 512>(), set_x_lds_limit<KIND, 1024>()};
  for (hipError_t e : r)
    if (e != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace

bool x_supported(int L) { return z_supported(L) || L == 1024; }

int x_waves(int L) { return z_lines_per_item(L) <= 2 ? 8 : 4; }

int x_rows_per_item(int L) { return x_waves(L) * z_lines_per_item(L); }

int x_block(int L) { return 64 * x_waves(L); }

size_t x_lds(int L) {
  return static_cast<size_t>(x_waves(L)) * z_lines_per_item(L) * wfft::stride_of(L) *
         sizeof(double2);
}

hipError_t launch_x(int kind, int L, const LaunchShape& sh, hipStream_t stream,
                    const PatchDev* patches, const WorkItem* items, int nitems,
                    const FieldPtrs& fields, void* ws) {
  float* w = static_cast<float*>(ws);
  switch (kind) {
    case kXFwd: return launch_kind<kXFwd>(L, sh, stream, patches, items, nitems, fields, w);
    case kXInv: return launch_kind<kXInv>(L, sh, stream, patches, items, nitems, fields, w);
    case kYFwd: return launch_kind<kYFwd>(L, sh, stream, patches, items, nitems, fields, w);
    case kYInv: return launch_kind<kYInv>(L, sh, stream, patches, items, nitems, fields, w);
    default: return hipErrorInvalidValue;
  }
}

hipError_t configure_x_attributes() {
  const hipError_t r[] = {configure_kind<kXFwd>(), configure_kind<kXInv>(), configure_kind<kYFwd>(),
                          configure_kind<kYInv>()};
  for (hipError_t e : r)
    if (e != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace wave2d
}  // namespace psatd
