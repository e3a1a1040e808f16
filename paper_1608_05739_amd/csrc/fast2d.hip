// Specialized 2D kernels for nx = nz = 4096 (FP32 storage, FP64 arithmetic).
//
// The z transform of length 4096 is split as 4096 = 512 x 8 (Cooley-Tukey):
// with z = z1 + 512 z2 and k = k2 + 8 k1,
//   X[k2 + 8 k1] = sum_z1 W512^(z1 k1) [ W4096^(z1 k2) sum_z2 x[z1 + 512 z2] W8^(z2 k2) ].
// The 8-point sums over z2 (and the W4096 twiddles) are done by the x passes,
// which therefore work on the eight rows z1 + 512 z2 of one tile; the fused z
// pass only runs the eight 512-point transforms of each column.  The inverse
// mirrors this.  Intermediate spectra live in the workspace as
//   [kx][8 z1 + k2]   (lines along z contiguous, one column per kx).
//
// x pass: one wavefront per row; the 2048-point complex FFT of the packed row
// z[m] = x[2m] + i x[2m+1] (radices 16, 16, 8) stays in registers, with
// wave-private LDS exchanges in FP64 (real and imaginary halves in turn).
#include <hip/hip_runtime.h>

#include "fast2d.hpp"
#include "fft.hpp"
#include "groups.hpp"
#include "update.hpp"

namespace psatd {
namespace fast2d {

constexpr int kMX = 2048;    // complex points per x line (nx = 4096)
constexpr int kNZ = 4096;    // z line length
constexpr int kN1 = 512;     // z1 range
constexpr int kWaves = 8;    // one wave per row of a tile
constexpr int kRegion = kMX + kMX / 16;  // doubles per wave region (padded)

// Wave regions are padded: logical index i sits at padx(i) = i + (i >> 4).

// After the wave regions, the inverse x pass keeps the per-lane twiddles of
// every tile in LDS, read from the FP64 tables once per workgroup (a global
// load inside a tile would hold up the LDS waits that follow it):
constexpr int kXtB = 0;       // W2048^(8 k), k < 16: stage-B bases (k = l mod 16)
constexpr int kXtC = 16;      // W2048^m, m < 256: stage-C bases (m = l + 64 b)
constexpr int kXtPost = 272;  // W4096^m, m <= 512: r2c post-twiddles and their step
constexpr int kXtCount = 785;


// One twiddle from an LDS table at an index the optimizer cannot see through,
// so that it is read again where it is used (reuse across tiles or
// transforms would keep the bases and their powers live through the whole
// kernel).
__device__ __forceinline__ double2 lds_twiddle(const double2* t, int idx) {
  asm volatile("" : "+v"(idx));
  return t[idx];
}

// Fill the x-pass table from the plan's FP64 tables (every patch of these
// passes has nx = 4096 and shares them).
__device__ __forceinline__ void fill_x_table(double2* xt, const PatchDev* P) {
  for (int e = threadIdx.x; e < kXtCount; e += blockDim.x) {
    double2 v;
    if (e < kXtC) v = P->fx.tw[8 * (e - kXtB)];
    else if (e < kXtPost) v = P->fx.tw[e - kXtC];
    else v = P->post[e - kXtPost];
    xt[e] = v;
  }
  __syncthreads();
}

// Order LDS traffic within one wavefront (no other wave touches the region).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 4 x 4 transpose of 16-byte chunks across the lanes l, l + 16, l + 32,
// l + 48 of a wave (l < 16): on return, chunk j of lane l + 16 a holds what
// chunk a of lane l + 16 j held.  Two register-only lane swaps per dword
// (v_permlane32_swap exchanges the lane bit of weight 32 with the chunk bit
// of weight 2, v_permlane16_swap the lane bit 16 with the chunk bit 1).
// The workspace columns lie 32 KB apart, so a wave whose 64 lanes each
// touch a different column translates 64 addresses per instruction; after
// the transpose four lanes share a column and an instruction touches 16.
__device__ __forceinline__ void quad_transpose(float4 (&c)[4]) {
  auto swap32 = [](float& x, float& y) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y),
                                                    false, false);
    x = __uint_as_float(r[0]);
    y = __uint_as_float(r[1]);
  };
  auto swap16 = [](float& x, float& y) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y),
                                                    false, false);
    x = __uint_as_float(r[0]);
    y = __uint_as_float(r[1]);
  };
#pragma unroll
  for (int j0 = 0; j0 < 2; ++j0) {
    swap32(c[j0].x, c[2 + j0].x);
    swap32(c[j0].y, c[2 + j0].y);
    swap32(c[j0].z, c[2 + j0].z);
    swap32(c[j0].w, c[2 + j0].w);
  }
#pragma unroll
  for (int j1 = 0; j1 < 4; j1 += 2) {
    swap16(c[j1].x, c[j1 + 1].x);
    swap16(c[j1].y, c[j1 + 1].y);
    swap16(c[j1].z, c[j1 + 1].z);
    swap16(c[j1].w, c[j1 + 1].w);
  }
}

// Exchange 32 complex values through a wave region: value (b, q) is written at
// padded index widx(b, q) and value (b', q') is read back from ridx(b', q').
// The index functions return padx() of the logical index written as a per-lane
// base plus a compile-time constant, so the constants fold into the LDS
// instruction offsets instead of each index taking registers of its own.
template <int NB_W, int NQ_W, int NB_R, int NQ_R, typename WF, typename RF>
__device__ __forceinline__ void wave_exchange(double* region, double2 (&v)[NB_W][NQ_W],
                                              double2 (&out)[NB_R][NQ_R], WF widx, RF ridx) {
#pragma unroll
  for (int b = 0; b < NB_W; ++b)
#pragma unroll
    for (int q = 0; q < NQ_W; ++q) region[widx(b, q)] = v[b][q].x;
  wave_lds_sync();
#pragma unroll
  for (int b = 0; b < NB_R; ++b)
#pragma unroll
    for (int q = 0; q < NQ_R; ++q) out[b][q].x = region[ridx(b, q)];
  wave_lds_sync();
#pragma unroll
  for (int b = 0; b < NB_W; ++b)
#pragma unroll
    for (int q = 0; q < NQ_W; ++q) region[widx(b, q)] = v[b][q].y;
  wave_lds_sync();
#pragma unroll
  for (int b = 0; b < NB_R; ++b)
#pragma unroll
    for (int q = 0; q < NQ_R; ++q) out[b][q].y = region[ridx(b, q)];
  wave_lds_sync();
}

// 2048-point FFT of one row held by one wave.  On entry lane l holds
// a[b][q] = z[l + 64 b + 128 q] (b < 2, q < 16); on exit c[b][q] = Z[l + 64 b + 256 q]
// (b < 4, q < 8), natural order.  twB = exp(SIGN 2 pi i (l mod 16)/256),
// twC[b] = exp(SIGN 2 pi i (l + 64 b)/2048).
template <int SIGN>
__device__ __forceinline__ void wave_fft2048(double* region, double2 (&a)[2][16],
                                             double2 (&c)[4][8], const double2 twB,
                                             const double2 (&twC)[4]) {
  const int l = threadIdx.x & 63;
  // stage A: radix 16, Ns = 1
#pragma unroll
  for (int b = 0; b < 2; ++b) DFT<16, SIGN>::run(a[b]);
  double2 s[2][16];
  // padx(16 (l + 64 b) + q) = 17 l + 1088 b + q            (q < 16)
  // padx(l + 64 b + 128 q)   = l + (l >> 4) + 68 b + 136 q
  const int wA = 17 * l;
  const int rA = l + (l >> 4);
  wave_exchange(region, a, s, [&](int b, int q) { return wA + 1088 * b + q; },
                [&](int b, int q) { return rA + 68 * b + 136 * q; });
  // stage B: radix 16, Ns = 16, k = j mod 16 = l mod 16
  {
    double2 wq = twB;
#pragma unroll
    for (int q = 1; q < 16; ++q) {
      s[0][q] = cmul(s[0][q], wq);
      s[1][q] = cmul(s[1][q], wq);
      if (q < 15) wq = cmul(wq, twB);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) DFT<16, SIGN>::run(s[b]);
  }
  // padx((l + 64 b - kB) 16 + kB + 16 q) = 272 (l >> 4) + kB + 1088 b + 17 q   (kB = l mod 16)
  // padx(l + 64 b + 256 q)                = l + (l >> 4) + 68 b + 272 q
  const int wB = 272 * (l >> 4) + (l & 15);
  wave_exchange(region, s, c, [&](int b, int q) { return wB + 1088 * b + 17 * q; },
                [&](int b, int q) { return rA + 68 * b + 272 * q; });
  // stage C: radix 8, Ns = 256, k = j
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double2 wq = twC[b];
#pragma unroll
    for (int q = 1; q < 8; ++q) {
      c[b][q] = cmul(c[b][q], wq);
      if (q < 7) wq = cmul(wq, twC[b]);
    }
    DFT<8, SIGN>::run(c[b]);
  }
}

__device__ __forceinline__ double2 ld_f2(const float2* p) {
  const float2 v = *p;
  return make_double2(v.x, v.y);
}

// ------------------------------------------------------------------ P1
// Forward: rows z1 + 512 z2 (z2 = wave) of component `comp` -> r2c along x ->
// 8-point DFT over z2 and twiddle W4096^(z1 k2) -> spectra [kx][8 z1 + k2].
//
// A workgroup loops over tiles when the grid is smaller than the tile count.
// The FFT state is dead during a tile's output phase, so the wave then loads
// its next tile's row (FP32) into registers there: the HBM latency of that load
// overlaps the output phase instead of stalling the next tile's FFT.

__device__ __forceinline__ const float2* x_row(const PatchDev* P, const FieldPtrs& fields,
                                               const WorkItem& wi, int w) {
  return reinterpret_cast<const float2*>(static_cast<const float*>(field_ptr(fields, wi.comp)) +
                                         P->off_real + (long long)(wi.first + kN1 * w) * (2 * kMX));
}

// lane l loads z[l + 64 b + 128 q] of the packed row (z[m] = x[2m] + i x[2m+1])
__device__ __forceinline__ void x_load_row(const float2* row, float2 (&raw)[2][16], int l) {
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int q = 0; q < 16; ++q) raw[b][q] = row[l + 64 * b + 128 * q];
}

__global__ void __launch_bounds__(512)
x_fwd_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
             int nitems, FieldPtrs fields, float* __restrict__ ws) {
  extern __shared__ double lds_d[];
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  double* region = lds_d + w * kRegion;
  int it = blockIdx.x;
  if (it >= nitems) return;
  float2 raw[2][16];
  {
    const WorkItem wi = items[xcd_local_order(it, nitems)];
    x_load_row(x_row(patches + wi.patch, fields, wi, w), raw, l);
  }
  for (; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[xcd_local_order(it, nitems)];
    const PatchDev* P = patches + wi.patch;
    const int z1 = wi.first;
    const double2* tw2048 = P->fx.tw;
    const double2* tw4096 = P->fz.tw;
    double2 twB = gload(tw2048, 8 * (l & 15));
    double2 twC[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) twC[b] = gload(tw2048, l + 64 * b);

    double2 a[2][16];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 16; ++q) a[b][q] = make_double2(raw[b][q].x, raw[b][q].y);
    double2 c[4][8];
    wave_fft2048<-1>(region, a, c, twB, twC);
    // stage Z (FP32) into this wave's region: Z[m] at float2 index m
    float2* zrow = reinterpret_cast<float2*>(region);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        zrow[l + 64 * b + 256 * q] = make_float2(static_cast<float>(c[b][q].x),
                                                 static_cast<float>(c[b][q].y));
    __syncthreads();

    // Output-phase constants, loaded before the next row: loads complete in
    // order, so waiting for a load issued after the prefetch would wait for
    // the whole prefetch.  post[t + 512 i] = post[t] post[512]^i and
    // W4096^(z1 k2) = (W4096^z1)^k2 follow by multiplication.
    const double2 wk0 = gload(P->post, static_cast<int>(threadIdx.x));
    const double2 wstep = gload(P->post, 512);
    const double2 wz1 = gload(tw4096, z1);
    __builtin_amdgcn_sched_barrier(0);
    // next tile's row (the same workgroup's next item), in flight during the output phase
    const int nit = it + gridDim.x;
    if (nit < nitems) {
      const WorkItem wn = items[xcd_local_order(nit, nitems)];
      x_load_row(x_row(patches + wn.patch, fields, wn, w), raw, l);
    }

    // output phase: kx = t + 512 i
    double2 tz[8];
    tz[0] = make_double2(1.0, 0.0);
    tz[1] = wz1;
#pragma unroll
    for (int k2 = 2; k2 < 8; ++k2) tz[k2] = cmul(tz[k2 - 1], wz1);
    double2 wk = wk0;
    float2* out = reinterpret_cast<float2*>(ws) + P->off_spec + (long long)wi.comp * P->comp_stride;
    // The r2c split X = (Z[k] + conj Z[N-k]) / 2 - (i/2) W^k (Z[k] - conj Z[N-k]) is
    // computed without the halving: this pass delivers 2X, and the z pass
    // folds the 1/2 into its coefficients (exactly: a power of two).
#pragma unroll 1
    for (int i = 0; i < 4; ++i) {
      const int kx = threadIdx.x + 512 * i;
      const int km = (kMX - kx) & (kMX - 1);
      double2 X[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const float2* zr = reinterpret_cast<const float2*>(lds_d + r * kRegion);
        const double2 za = ld_f2(zr + kx);
        const double2 zb = ld_f2(zr + km);  // km = 0 for kx = 0: in bounds, result replaced
        const double2 wd = cmul(wk, make_double2(za.x - zb.x, za.y + zb.y));
        X[r] = make_double2((za.x + zb.x) + wd.y, (za.y - zb.y) - wd.x);
      }
      // kx = 0 holds DC and Nyquist packed (2 Re Z[0] +- 2 Im Z[0]): only the
      // first thread of the first wave in the first iteration (a uniform branch)
      if (i == 0 && w == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const double2 za = ld_f2(reinterpret_cast<const float2*>(lds_d + r * kRegion) + kx);
          if (kx == 0) X[r] = make_double2(2.0 * (za.x + za.y), 2.0 * (za.x - za.y));
        }
      }
      DFT<8, -1>::run(X);
      float4 ch[4];
#pragma unroll
      for (int k2 = 0; k2 < 8; k2 += 2) {
        const double2 u = cmul(X[k2], tz[k2]);
        const double2 v = cmul(X[k2 + 1], tz[k2 + 1]);
        ch[k2 / 2] = make_float4(static_cast<float>(u.x), static_cast<float>(u.y),
                                 static_cast<float>(v.x), static_cast<float>(v.y));
      }
      // lane l + 16 a now stores chunk a (k2 = 2a, 2a + 1) of the columns of
      // lanes l + 16 j, j = 0..3: 16 columns per store instead of 64
      quad_transpose(ch);
      const int lq = l & 15, aq = l >> 4;
      const long long kx0 = kx - l + lq;  // the column of lane lq (j = 0)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float4* dst = reinterpret_cast<float4*>(out + (kx0 + 16 * j) * kNZ + 8 * z1) + aq;
        *dst = ch[j];
      }
      wk = cmul(wk, wstep);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ P3
// Inverse: spectra [kx][8 z1 + k2] -> inverse 8-point DFT over k2 -> rows
// z1 + 512 z2 -> c2r along x -> real rows of E, B.
__global__ void __launch_bounds__(512)
x_inv_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
             int nitems, FieldPtrs fields, float* __restrict__ ws) {
  extern __shared__ double lds_d[];
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  double* region = lds_d + w * kRegion;
  const double2* xt = reinterpret_cast<const double2*>(lds_d + kRegion * kWaves);
  if (static_cast<int>(blockIdx.x) >= nitems) return;
  fill_x_table(reinterpret_cast<double2*>(lds_d + kRegion * kWaves),
               patches + items[xcd_local_order(blockIdx.x, nitems)].patch);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[xcd_local_order(it, nitems)];
    const PatchDev* P = patches + wi.patch;
    const int z1 = wi.first;
    const float2* in = reinterpret_cast<const float2*>(ws) + P->off_spec +
                       (long long)wi.comp * P->comp_stride;
    // phase 1: inverse DFT over k2 for each kx, into the FP32 staging rows
#pragma unroll 1
    for (int i = 0; i < 4; ++i) {
      const int kx = threadIdx.x + 512 * i;
      // lane l + 16 a loads chunk a of the columns of lanes l + 16 j (16
      // columns per load instead of 64); the transpose then hands every lane
      // the four chunks of its own column
      const int lq = l & 15, aq = l >> 4;
      const long long kx0 = kx - l + lq;
      float4 ch[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        ch[j] = *(reinterpret_cast<const float4*>(in + (kx0 + 16 * j) * kNZ + 8 * z1) + aq);
      quad_transpose(ch);
      double2 X[8];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        X[2 * h] = make_double2(ch[h].x, ch[h].y);
        X[2 * h + 1] = make_double2(ch[h].z, ch[h].w);
      }
      DFT<8, 1>::run(X);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        float2* zr = reinterpret_cast<float2*>(lds_d + r * kRegion);
        zr[kx] = make_float2(static_cast<float>(X[r].x), static_cast<float>(X[r].y));
      }
    }
    __syncthreads();
    // phase 2: wave w owns row z = z1 + 512 w: c2r pre-twiddle, inverse FFT
    double2 twB = cconj(lds_twiddle(xt, kXtB + (l & 15)));
    double2 twC[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) twC[b] = cconj(lds_twiddle(xt, kXtC + l + 64 * b));
    const float2* zrow = reinterpret_cast<const float2*>(region);
    const float2* zmir = zrow + (64 - l);
    // pre-twiddles W^k, k = l + 64 b + 128 q: start at W^(l + 64 b), step W^128
    double2 wk[2];
    wk[0] = lds_twiddle(xt, kXtPost + l);
    wk[1] = lds_twiddle(xt, kXtPost + l + 64);
    const double2 wstep = lds_twiddle(xt, kXtPost + 128);
    double2 a[2][16];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        __builtin_amdgcn_sched_barrier(0);
        const int k = l + 64 * b + 128 * q;
        const double2 xa = ld_f2(zrow + k);
        // mirror index kMX - k = (64 - l) + 64 (1 - b) + 128 (15 - q), a lane base
        // plus a constant; for k = 0 it is kMX, inside the wave's padded region,
        // and the k = 0 entry (DC and Nyquist packed together) is selected below
        const double2 xb = ld_f2(zmir + 64 * (1 - b) + 128 * (15 - q));
        const double2 p = make_double2(xa.x + xb.x, xa.y - xb.y);
        const double2 m = make_double2(xa.x - xb.x, xa.y + xb.y);
        const double2 t1 = cmul(cconj(wk[b]), m);
        a[b][q] = make_double2(p.x - t1.y, p.y + t1.x);
        if (b == 0 && q == 0 && l == 0) a[b][q] = make_double2(xa.x + xa.y, xa.x - xa.y);
        if (q < 15) wk[b] = cmul(wk[b], wstep);
      }
    wave_lds_sync();
    double2 c[4][8];
    wave_fft2048<1>(region, a, c, twB, twC);
    float2* row = reinterpret_cast<float2*>(static_cast<float*>(field_ptr(fields, wi.comp)) + P->off_real +
                                            (long long)(z1 + kN1 * w) * (2 * kMX));
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        row[l + 64 * b + 256 * q] =
            make_float2(static_cast<float>(c[b][q].x), static_cast<float>(c[b][q].y));
    __syncthreads();
  }
}

// ------------------------------------------------------------------ P2
// Fused z pass on one column kx (4096 modes) per workgroup of 512 threads,
// run as eight 512-point transforms (group k2 over z1 or k1), each with three
// radix-8 stages.  Two thread mappings:
//   A (global memory): thread t = 8 j + k2 holds elements j + 64 q of group k2,
//     i.e. column positions t + 512 q: coalesced loads and stores;
//   B (transform and update): wave w = k2 holds group k2, lane j its elements
//     j + 64 q; the mode index of element j + 64 q of group k2 is
//     8 (j + 64 q) + k2.
// A forward transform runs stage 1 in A, hands over to B through LDS (the one
// workgroup barrier) and runs stages 2 and 3 in B with a wave-private
// exchange.  The inverse is the adjoint of the forward (stages in reverse
// order, exchanges transposed, butterflies and twiddles conjugated): stages 3
// and 2 in B, hand-over, stage 1 in A.  Waves meet once per transform.
// LDS: two transition buffers used alternately, so that the writes of one
// hand-over never meet the reads of the previous one (a barrier always lies
// between two uses of the same buffer); a wave's private exchange uses its own
// group's region of the current buffer.  Element e of group k2 lives at
// 513 k2 + e: the eight lanes that the LDS serves together then hit
// consecutive slots in every access below, and every address is a per-thread
// base plus a compile-time offset.
constexpr int kGroupStride = 513;
constexpr int kZBuf = kGroupStride * 7 + 512;  // double2 per transition buffer

// After the transition buffers and the coefficient slots, LDS holds the
// twiddles every thread uses in every transform, read from the FP64 table
// once per workgroup: a global load inside a transform would be issued after
// the prefetch of the next input, and since loads complete in order, waiting
// for it would wait for the prefetch.
constexpr int kZtS2 = 0;      // W4096^(64 k), k < 8: stage-2 bases (k = jB mod 8)
constexpr int kZtS3 = 8;      // W4096^(8 j), j < 64: stage-3 bases (j = jB)
constexpr int kZtOut = 72;    // W4096^(jA k2A) of thread tA: first output twiddle of an inverse
constexpr int kZtStep = 584;  // W4096^(64 k2), k2 < 8: its step over q
constexpr int kZtCount = 592;


template <int SIGN>
__device__ __forceinline__ void twiddle8(double2 (&v)[8], double2 w) {
  if constexpr (SIGN > 0) w.y = -w.y;
  double2 wq = w;
  v[1] = cmul(v[1], w);
#pragma unroll
  for (int q = 2; q < 8; ++q) {
    wq = cmul(wq, w);
    v[q] = cmul(v[q], wq);
  }
}

// Thread indices of both mappings and the LDS bases of the exchanges.
struct ZIdx {
  int tA, jA, k2A;  // mapping A
  int tB, jB, k2B;  // mapping B (tB = 64 k2B + jB = threadIdx.x)
  int baseA;        // element 8 jA of group k2A       (+ q)
  int baseB1;       // element jB of group k2B         (+ 64 q)
  int baseB2;       // element 8 (jB - k) + k, k = jB mod 8, of group k2B (+ 8 q)
};

__device__ __forceinline__ ZIdx make_zidx() {
  ZIdx x;
  x.tA = threadIdx.x;
  x.jA = x.tA >> 3;
  x.k2A = x.tA & 7;
  x.tB = threadIdx.x;
  x.jB = x.tB & 63;
  x.k2B = x.tB >> 6;
  const int k = x.jB & 7;
  x.baseA = kGroupStride * x.k2A + 8 * x.jA;
  x.baseB1 = kGroupStride * x.k2B + x.jB;
  x.baseB2 = kGroupStride * x.k2B + 8 * (x.jB - k) + k;
  return x;
}

// Forward: v holds elements jA + 64 q of group k2A (mapping A) on entry and
// transform outputs jB + 64 q of group k2B (mapping B) on exit.  The twiddle
// bases are read from LDS inside each call, after a barrier: otherwise the
// compiler would keep the powers of the (identical) bases of every call live
// across the whole kernel.
__device__ __forceinline__ void fwd512(double2 (&v)[8], double2* buf, const ZIdx& x,
                                       const double2* zt) {
  DFT<8, -1>::run(v);  // stage 1 (Ns = 1), mapping A; outputs 8 j + q
  double2* wa = buf + x.baseA;
#pragma unroll
  for (int q = 0; q < 8; ++q) wa[q] = v[q];
  __syncthreads();
  double2* b1 = buf + x.baseB1;
  double2* b2 = buf + x.baseB2;
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = b1[64 * q];
  // stage 2: Ns = 8, k = j mod 8, w = exp(-2 pi i k / 64); outputs 8 (j - k) + k + 8 q
  twiddle8<-1>(v, lds_twiddle(zt, kZtS2 + (x.jB & 7)));
  DFT<8, -1>::run(v);
#pragma unroll
  for (int q = 0; q < 8; ++q) b2[8 * q] = v[q];
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = b1[64 * q];
  // stage 3: Ns = 64, k = j, w = exp(-2 pi i j / 512); outputs j + 64 q
  twiddle8<-1>(v, lds_twiddle(zt, kZtS3 + x.jB));
  DFT<8, -1>::run(v);
}

// Inverse (unnormalized, the adjoint of fwd512): v holds elements jB + 64 q of
// group k2B (mapping B) on entry and elements jA + 64 q of group k2A
// (mapping A) on exit.
__device__ __forceinline__ void inv512(double2 (&v)[8], double2* buf, const ZIdx& x,
                                       const double2* zt) {
  double2* b1 = buf + x.baseB1;
  double2* b2 = buf + x.baseB2;
  // adjoint of stage 3
  DFT<8, 1>::run(v);
  twiddle8<1>(v, lds_twiddle(zt, kZtS3 + x.jB));  // conjugate twiddles after the butterflies
#pragma unroll
  for (int q = 0; q < 8; ++q) b1[64 * q] = v[q];
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = b2[8 * q];
  // adjoint of stage 2
  DFT<8, 1>::run(v);
  twiddle8<1>(v, lds_twiddle(zt, kZtS2 + (x.jB & 7)));
#pragma unroll
  for (int q = 0; q < 8; ++q) b1[64 * q] = v[q];
  __syncthreads();
  const double2* ra = buf + x.baseA;
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = ra[q];
  // adjoint of stage 1, mapping A
  DFT<8, 1>::run(v);
}

// Loads of one component column into FP32 registers (mapping A, positions
// t + 512 q): a uniform base per q plus one 32-bit lane offset.
__device__ __forceinline__ void z_load(const float2* src, float2 (&raw)[8], int t) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float2* __restrict__ bq = src + 512 * q;
    raw[q] = bq[t];
  }
}

// Per-column state of the z pass.  The transforms alternate between the two
// transition buffers: `tr` counts them (uniform across the workgroup).
// EXACT: the k tables hold the exact wavenumbers, so kz follows from the mode
// index; otherwise (order p) kz is read from the table.
template <bool EXACT>
struct ZCol {
  float2* col;       // workspace spectrum of column kx, component 0
  long long cs;      // component stride (complex elements)
  double kx, dt, c, c2, eps0, ie, scale;
  double dkz;        // 2 pi / (nz dz) for the exact wavenumbers, else 0
  const double* kzb; // kz in mapping-B order (order-p tables)
  const double2* zt; // the twiddles in LDS (kZt*)
  ZIdx x;
  double2* lds;      // two transition buffers of kZBuf double2
  int tr;

  __device__ __forceinline__ double2* next_buf() {
    double2* b = lds + (tr & 1) * kZBuf;
    ++tr;
    return b;
  }
  // kz of mode 8 jB + k2B + 512 q.  Exact wavenumbers come from the index, as
  // the k table computes them (a global load here would wait for the
  // prefetch, see kZt*); order-p tables are read.  The empty asm makes every
  // kz opaque to the optimizer: the s and p groups evaluate the same
  // coefficients, and merging the two evaluations would keep them live
  // across the s group's inverse transforms.
  __device__ __forceinline__ double kz_of(int q) const {
    int o = 512 * q;
    asm volatile("" : "+v"(o));
    double v;
    if constexpr (EXACT) {
      const int idx = 8 * x.jB + x.k2B + o;
      const int m = idx < kNZ / 2 ? idx : (idx == kNZ / 2 ? 0 : idx - kNZ);
      v = static_cast<double>(m) * dkz;
    } else {
      v = gload(kzb, x.tB + o);
    }
    asm volatile("" : "+v"(v));
    return v;
  }
  __device__ __forceinline__ Coef coef(double kzv) const {
    return psatd_coef(sqrt(kx * kx + kzv * kzv), dt, c, eps0, scale);
  }
  __device__ __forceinline__ const float2* src(int comp) const { return col + comp * cs; }
  // Software pipeline: `pre` holds the loads issued one phase earlier.  Issue
  // the loads of `next` into `pre`, then transform the previous contents into
  // `dst` (mapping B), so that the HBM latency of the next input overlaps this
  // transform and the update that follows it.
  __device__ __forceinline__ void fwd(float2 (&pre)[8], const float2* next, float2 (&dst)[8]) {
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = ld2(pre[q]);
    z_load(next, pre, x.tA);
    fwd512(v, next_buf(), x, zt);
#pragma unroll
    for (int q = 0; q < 8; ++q) dst[q] = st2(v[q]);
    // keep the transform's temporaries apart from the update that follows
    __builtin_amdgcn_sched_barrier(0);
  }
  // Inverse transform of one accumulator (mapping B), twiddle W4096^(-z1 k2)
  // with z1 = jA + 64 q, store (mapping A).
  __device__ __forceinline__ void inv(int comp, const float2 (&src_b)[8]) {
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = ld2(src_b[q]);
    inv512(v, next_buf(), x, zt);
    double2 tq = cconj(lds_twiddle(zt, kZtOut + x.tA));
    const double2 step = cconj(lds_twiddle(zt, kZtStep + x.k2A));
    float2* dst = col + comp * cs;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      float2* __restrict__ bq = dst + 512 * q;
      bq[x.tA] = st2(cmul(v[q], tq));
      if (q < 7) tq = cmul(tq, step);
    }
  }
};

template <bool EXACT>
__device__ __forceinline__ ZCol<EXACT> make_zcol(const PatchDev* P, int kxcol, float* ws,
                                          const Physics& ph, double2* lds, int tr) {
  ZCol<EXACT> z;
  z.col = reinterpret_cast<float2*>(ws) + P->off_spec + (long long)kxcol * kNZ;
  z.cs = P->comp_stride;
  z.kx = P->kx[kxcol];
  z.dt = P->dt;
  z.c = ph.c;
  z.c2 = ph.c * ph.c;
  z.eps0 = ph.eps0;
  z.ie = 1.0 / ph.eps0;
  z.scale = 0.5 * P->inv_n;  // the forward x pass delivers twice the spectrum
  z.dkz = P->dkz;
  z.kzb = P->kz_b;
  z.zt = lds + 2 * kZBuf + kNZ / 4;
  z.x = make_zidx();
  z.lds = lds;
  z.tr = tr;
  return z;
}

// The update is linear in every input, so each group accumulates its three
// outputs while its inputs are transformed one at a time: only the FP32
// accumulators, the per-mode coefficients that later phases need and the
// transform in flight are live.  The arithmetic of every term is FP64.
//
// s-pol (Ey, Bx, Bz), any source form:
//   sources Jy: Ey' = -(S/eps0) Jy, Bx' = -i X1 kz Jy, Bz' = i X1 kx Jy
//   Bx: Ey' += i c^2 S kz Bx,  Bx' += C Bx
//   Bz: Ey' -= i c^2 S kx Bz,  Bz' += C Bz
//   Ey: Ey' += C Ey,  Bx' += i S kz Ey,  Bz' -= i S kx Ey
// p-pol (Ex, Ez, By) in vacuum:
//   By: Ex' -= i c^2 S kz By,  Ez' += i c^2 S kx By,  By' += C By
//   Ex: Ex' += C Ex,  By' -= i S kz Ex
//   Ez: Ez' += C Ez,  By' += i S kx Ez
// (p-pol with sources: z_ppol_sources.)
template <int G, int SRC, typename Z>
__device__ __forceinline__ void z_group(Z& z, float2 (&pre)[8], const float2* next) {
  static_assert(G == 0 || SRC == kVacuum, "p-pol with sources has its own schedule");
  constexpr bool kSrc = SRC != kVacuum;
  constexpr int kO0 = G == 0 ? kEy : kEx;
  constexpr int kO1 = G == 0 ? kBx : kEz;
  constexpr int kO2 = G == 0 ? kBz : kBy;
  const double kx = z.kx, c2 = z.c2;

  float2 acc[3][8];
  double cC[8], cS[8];

  if constexpr (kSrc) {
    float2 jy[8];
    z.fwd(pre, z.src(kBx), jy);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double kz = z.kz_of(q);
      const Coef cf = z.coef(kz);
      cC[q] = cf.C;
      cS[q] = cf.S;
      double2 a, b, c;
      src_2d_s(kx, kz, cf, ld2(jy[q]), a, b, c);
      acc[0][q] = st2(a);
      acc[1][q] = st2(b);
      acc[2][q] = st2(c);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // ---- field 1: s-pol Bx, p-pol By
  {
    float2 f[8];
    z.fwd(pre, z.src(G == 0 ? kBz : kEx), f);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double kz = z.kz_of(q);
      if constexpr (!kSrc) {
        const Coef cf = z.coef(kz);
        cC[q] = cf.C;
        cS[q] = cf.S;
      }
      const double C = cC[q], cS2 = c2 * cS[q];
      const double2 v = ld2(f[q]);
      double2 a0 = kSrc ? ld2(acc[0][q]) : make_double2(0.0, 0.0);
      double2 a1 = kSrc ? ld2(acc[1][q]) : make_double2(0.0, 0.0);
      double2 a2 = kSrc ? ld2(acc[2][q]) : make_double2(0.0, 0.0);
      if constexpr (G == 0) {
        a0.x -= cS2 * kz * v.y;
        a0.y += cS2 * kz * v.x;
        a1.x += C * v.x;
        a1.y += C * v.y;
      } else {
        a0.x += cS2 * kz * v.y;
        a0.y -= cS2 * kz * v.x;
        a1.x -= cS2 * kx * v.y;
        a1.y += cS2 * kx * v.x;
        a2.x += C * v.x;
        a2.y += C * v.y;
      }
      acc[0][q] = st2(a0);
      acc[1][q] = st2(a1);
      acc[2][q] = st2(a2);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // ---- field 2: s-pol Bz, p-pol Ex
  {
    float2 f[8];
    z.fwd(pre, z.src(G == 0 ? kEy : kEz), f);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double kz = z.kz_of(q);
      const double C = cC[q], S = cS[q], cS2 = c2 * cS[q];
      const double2 v = ld2(f[q]);
      double2 a0 = ld2(acc[0][q]), a2 = ld2(acc[2][q]);
      if constexpr (G == 0) {
        a0.x += cS2 * kx * v.y;
        a0.y -= cS2 * kx * v.x;
        a2.x += C * v.x;
        a2.y += C * v.y;
      } else {
        a0.x += C * v.x;
        a0.y += C * v.y;
        a2.x += S * kz * v.y;
        a2.y -= S * kz * v.x;
      }
      acc[0][q] = st2(a0);
      acc[2][q] = st2(a2);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // ---- field 3: s-pol Ey, p-pol Ez
  {
    float2 f[8];
    z.fwd(pre, next, f);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double kz = z.kz_of(q);
      const double C = cC[q], S = cS[q];
      const double2 v = ld2(f[q]);
      double2 a0 = ld2(acc[0][q]), a1 = ld2(acc[1][q]), a2 = ld2(acc[2][q]);
      if constexpr (G == 0) {
        a0.x += C * v.x;
        a0.y += C * v.y;
        a1.x -= S * kz * v.y;
        a1.y += S * kz * v.x;
        a2.x += S * kx * v.y;
        a2.y -= S * kx * v.x;
      } else {
        a1.x += C * v.x;
        a1.y += C * v.y;
        a2.x -= S * kx * v.y;
        a2.y += S * kx * v.x;
      }
      acc[0][q] = st2(a0);
      acc[1][q] = st2(a1);
      acc[2][q] = st2(a2);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  z.inv(kO0, acc[0]);
  z.inv(kO1, acc[1]);
  z.inv(kO2, acc[2]);
}

// p-pol (Ex, Ez, By) with sources.  The coefficients are evaluated once, in
// the first phase; C and S stay in registers and the third coefficient that a
// later phase needs goes to the thread's own LDS slots (cx[t + 512 q], written
// and read by the same thread only, so no barrier is involved).  The slots are
// FP32: the two transition buffers leave 16 KB of LDS, and a coefficient
// rounded to FP32 adds an error of the same size as the FP32 rounding of the
// result it multiplies into (the arithmetic stays FP64).
//   rho form:  rho_old, rho_new: Ex' = i kx R, Ez' = i kz R, R = X3 rho_old - X2 rho_new
//                                (cx = X1)
//              Jx: Ex' -= (S/eps0) Jx, By' = i X1 kz Jx
//              Jz: Ez' -= (S/eps0) Jz, By' -= i X1 kx Jz
//              By, Ex, Ez: field terms as in vacuum
//   J form:    Jx, Jz: Ex' = -(S/eps0) Jx - dt X2 kx (k.J), Ez' = -(S/eps0) Jz - dt X2 kz (k.J),
//                      By' = i X1 (kz Jx - kx Jz)      (cx = L1 = eps0 c^2 X1)
//              By: field terms as in vacuum
//              Ex: Ex' += C Ex + L1 kx kx Ex, Ez' += L1 kz kx Ex, By' -= i S kz Ex
//              Ez: Ez' += C Ez + L1 kz kz Ez, Ex' += L1 kx kz Ez, By' += i S kx Ez
template <int SRC, typename Z>
__device__ __forceinline__ void z_ppol_sources(Z& z, float* cx, float2 (&pre)[8],
                                               const float2* next) {
  static_assert(SRC == kRho || SRC == kJForm, "source forms only");
  const double kx = z.kx, c2 = z.c2;
  const int t = z.x.tB;
  float2 acc[3][8];
  double cC[8], cS[8];
  if constexpr (SRC == kRho) {
    {
      float2 ro[8], rn[8];
      z.fwd(pre, z.src(kRhoNew), ro);
      z.fwd(pre, z.src(kJx), rn);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double kz = z.kz_of(q);
        const Coef cf = z.coef(kz);
        cC[q] = cf.C;
        cS[q] = cf.S;
        cx[t + 512 * q] = static_cast<float>(cf.X1);
        const double2 o = ld2(ro[q]), n = ld2(rn[q]);
        const double2 R = make_double2(cf.X3 * o.x - cf.X2 * n.x, cf.X3 * o.y - cf.X2 * n.y);
        acc[0][q] = st2(make_double2(-kx * R.y, kx * R.x));
        acc[1][q] = st2(make_double2(-kz * R.y, kz * R.x));
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    {
      float2 f[8];
      z.fwd(pre, z.src(kJz), f);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double kz = z.kz_of(q);
        const double Se = cS[q] * z.ie, X1 = cx[t + 512 * q];
        const double2 v = ld2(f[q]);
        double2 a0 = ld2(acc[0][q]);
        a0.x -= Se * v.x;
        a0.y -= Se * v.y;
        acc[0][q] = st2(a0);
        acc[2][q] = st2(make_double2(-X1 * kz * v.y, X1 * kz * v.x));
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    {
      float2 f[8];
      z.fwd(pre, z.src(kBy), f);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double Se = cS[q] * z.ie, X1 = cx[t + 512 * q];
        const double2 v = ld2(f[q]);
        double2 a1 = ld2(acc[1][q]), a2 = ld2(acc[2][q]);
        a1.x -= Se * v.x;
        a1.y -= Se * v.y;
        a2.x += X1 * kx * v.y;
        a2.y -= X1 * kx * v.x;
        acc[1][q] = st2(a1);
        acc[2][q] = st2(a2);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  } else {
    float2 jx[8], jz[8];
    z.fwd(pre, z.src(kJz), jx);
    z.fwd(pre, z.src(kBy), jz);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double kz = z.kz_of(q);
      const Coef cf = z.coef(kz);
      cC[q] = cf.C;
      cS[q] = cf.S;
      cx[t + 512 * q] = static_cast<float>(z.eps0 * c2 * cf.X1);
      double2 a, b, c;
      const double2 zero = make_double2(0.0, 0.0);
      src_2d_p<kJForm>(kx, kz, cf, z.dt, ld2(jx[q]), ld2(jz[q]), zero, zero, a, b, c);
      acc[0][q] = st2(a);
      acc[1][q] = st2(b);
      acc[2][q] = st2(c);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // By: Ex' -= i c^2 S kz By, Ez' += i c^2 S kx By, By' += C By
  {
    float2 f[8];
    z.fwd(pre, z.src(kEx), f);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double kz = z.kz_of(q);
      const double C = cC[q], cS2 = c2 * cS[q];
      const double2 v = ld2(f[q]);
      double2 a0 = ld2(acc[0][q]), a1 = ld2(acc[1][q]), a2 = ld2(acc[2][q]);
      a0.x += cS2 * kz * v.y;
      a0.y -= cS2 * kz * v.x;
      a1.x -= cS2 * kx * v.y;
      a1.y += cS2 * kx * v.x;
      a2.x += C * v.x;
      a2.y += C * v.y;
      acc[0][q] = st2(a0);
      acc[1][q] = st2(a1);
      acc[2][q] = st2(a2);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // Ex: Ex' += C Ex, By' -= i S kz Ex  (J form: Ex' += L1 kx kx Ex, Ez' += L1 kz kx Ex)
  {
    float2 f[8];
    z.fwd(pre, z.src(kEz), f);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double kz = z.kz_of(q);
      const double C = cC[q], S = cS[q];
      const double2 v = ld2(f[q]);
      double2 a0 = ld2(acc[0][q]), a2 = ld2(acc[2][q]);
      a0.x += C * v.x;
      a0.y += C * v.y;
      a2.x += S * kz * v.y;
      a2.y -= S * kz * v.x;
      if constexpr (SRC == kJForm) {
        const double L = cx[t + 512 * q];
        double2 a1 = ld2(acc[1][q]);
        a0.x += L * kx * kx * v.x;
        a0.y += L * kx * kx * v.y;
        a1.x += L * kz * kx * v.x;
        a1.y += L * kz * kx * v.y;
        acc[1][q] = st2(a1);
      }
      acc[0][q] = st2(a0);
      acc[2][q] = st2(a2);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // Ez: Ez' += C Ez, By' += i S kx Ez  (J form: Ex' += L1 kx kz Ez, Ez' += L1 kz kz Ez)
  {
    float2 f[8];
    z.fwd(pre, next, f);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double kz = z.kz_of(q);
      const double C = cC[q], S = cS[q];
      const double2 v = ld2(f[q]);
      double2 a1 = ld2(acc[1][q]), a2 = ld2(acc[2][q]);
      a1.x += C * v.x;
      a1.y += C * v.y;
      a2.x -= S * kx * v.y;
      a2.y += S * kx * v.x;
      if constexpr (SRC == kJForm) {
        const double L = cx[t + 512 * q];
        double2 a0 = ld2(acc[0][q]);
        a0.x += L * kx * kz * v.x;
        a0.y += L * kx * kz * v.y;
        a1.x += L * kz * kz * v.x;
        a1.y += L * kz * kz * v.y;
        acc[0][q] = st2(a0);
      }
      acc[1][q] = st2(a1);
      acc[2][q] = st2(a2);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  z.inv(kEx, acc[0]);
  z.inv(kEz, acc[1]);
  z.inv(kBy, acc[2]);
}

// First input of the s group and of the p group, in processing order.
template <int SRC>
struct ZOrder {
  static constexpr int kFirstS = SRC == kVacuum ? kBx : kJy;
  static constexpr int kFirstP = SRC == kVacuum ? kBy : (SRC == kRho ? kRhoOld : kJx);
};

template <int SRC, bool EXACT>
__global__ void __launch_bounds__(512)
z_fused_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
               int nitems, float* __restrict__ ws, Physics ph) {
  extern __shared__ double2 lds2[];
  // two transition buffers, then one coefficient per mode (FP32, see z_ppol_sources)
  float* cx = reinterpret_cast<float*>(lds2 + 2 * kZBuf);
  int it = blockIdx.x;
  if (it >= nitems) return;
  int patch = items[it].patch, kxcol = items[it].first;
  {
    // every patch of this pass has nz = 4096 and shares the FP64 table
    const double2* __restrict__ tw = patches[patch].fz.tw;
    double2* zt = lds2 + 2 * kZBuf + kNZ / 4;
    for (int e = threadIdx.x; e < kZtCount; e += blockDim.x) {
      int m;
      if (e < kZtS3) m = 64 * (e - kZtS2);
      else if (e < kZtOut) m = 8 * (e - kZtS3);
      else if (e < kZtStep) m = (((e - kZtOut) >> 3) * ((e - kZtOut) & 7)) & (kNZ - 1);
      else m = (64 * (e - kZtStep)) & (kNZ - 1);
      zt[e] = tw[m];
    }
    __syncthreads();
  }
  float2 pre[8];
  z_load(make_zcol<EXACT>(patches + patch, kxcol, ws, ph, lds2, 0).src(ZOrder<SRC>::kFirstS), pre,
         threadIdx.x);
  int tr = 0;  // transforms done so far: selects the transition buffer
  for (; it < nitems; it += gridDim.x) {
    ZCol<EXACT> z = make_zcol<EXACT>(patches + patch, kxcol, ws, ph, lds2, tr);
    // The p group's last phase prefetches the next column's first input; after
    // the last column it re-reads this column's (never used).
    const int nit = it + gridDim.x;
    const bool more = nit < nitems;
    const int npatch = more ? items[nit].patch : patch;
    const int nkx = more ? items[nit].first : kxcol;
    const PatchDev* Pn = patches + npatch;
    const float2* next = reinterpret_cast<const float2*>(ws) + Pn->off_spec +
                         (long long)nkx * kNZ + ZOrder<SRC>::kFirstS * Pn->comp_stride;
    z_group<0, SRC>(z, pre, z.src(ZOrder<SRC>::kFirstP));
    if constexpr (SRC == kVacuum)
      z_group<1, kVacuum>(z, pre, next);
    else
      z_ppol_sources<SRC>(z, cx, pre, next);
    tr = z.tr;
    patch = npatch;
    kxcol = nkx;
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_x_fwd(const LaunchShape& sh, hipStream_t s, const PatchDev* p,
                        const WorkItem* it, int n, const FieldPtrs& f, void* ws) {
  hipLaunchKernelGGL(x_fwd_kernel, dim3(sh.grid), dim3(sh.block), sh.lds_bytes, s, p, it, n, f,
                     static_cast<float*>(ws));
  return hipGetLastError();
}

hipError_t launch_x_inv(const LaunchShape& sh, hipStream_t s, const PatchDev* p,
                        const WorkItem* it, int n, const FieldPtrs& f, void* ws) {
  hipLaunchKernelGGL(x_inv_kernel, dim3(sh.grid), dim3(sh.block), sh.lds_bytes, s, p, it, n, f,
                     static_cast<float*>(ws));
  return hipGetLastError();
}

template <bool EXACT>
static void launch_z(int src, const LaunchShape& sh, hipStream_t s, const PatchDev* p,
                     const WorkItem* it, int n, float* w, Physics ph) {
  switch (src) {
    case kVacuum:
      hipLaunchKernelGGL((z_fused_kernel<kVacuum, EXACT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, s, p, it, n, w, ph);
      break;
    case kRho:
      hipLaunchKernelGGL((z_fused_kernel<kRho, EXACT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, s, p, it, n, w, ph);
      break;
    default:
      hipLaunchKernelGGL((z_fused_kernel<kJForm, EXACT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, s, p, it, n, w, ph);
      break;
  }
}

hipError_t launch_z_fused(int src, bool exact_k, const LaunchShape& sh, hipStream_t s,
                          const PatchDev* p, const WorkItem* it, int n, void* ws, Physics ph) {
  float* w = static_cast<float*>(ws);
  if (exact_k) launch_z<true>(src, sh, s, p, it, n, w, ph);
  else launch_z<false>(src, sh, s, p, it, n, w, ph);
  return hipGetLastError();
}

hipError_t configure_attributes() {
  const int lim = 160 * 1024;
  hipError_t e = hipSuccess, r;
  const void* fns[] = {reinterpret_cast<const void*>(&x_fwd_kernel),
                       reinterpret_cast<const void*>(&x_inv_kernel),
                       reinterpret_cast<const void*>(&z_fused_kernel<kVacuum, true>),
                       reinterpret_cast<const void*>(&z_fused_kernel<kRho, true>),
                       reinterpret_cast<const void*>(&z_fused_kernel<kJForm, true>),
                       reinterpret_cast<const void*>(&z_fused_kernel<kVacuum, false>),
                       reinterpret_cast<const void*>(&z_fused_kernel<kRho, false>),
                       reinterpret_cast<const void*>(&z_fused_kernel<kJForm, false>)};
  for (const void* f : fns)
    if ((r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim)) != hipSuccess)
      e = r;
  return e;
}

size_t x_fwd_lds_bytes() { return sizeof(double) * kRegion * kWaves; }
size_t x_inv_lds_bytes() { return sizeof(double) * kRegion * kWaves + sizeof(double2) * kXtCount; }
size_t z_lds_bytes() {
  return sizeof(double2) * 2 * kZBuf + sizeof(float) * kNZ + sizeof(double2) * kZtCount;
}

}  // namespace fast2d
}  // namespace psatd
