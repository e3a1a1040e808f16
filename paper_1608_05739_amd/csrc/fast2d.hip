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
constexpr int kN2 = 8;       // z2 range (rows per tile)
constexpr int kWaves = 8;    // one wave per row of a tile
constexpr int kRegion = kMX + kMX / 16;  // doubles per wave region (padded)

__device__ __forceinline__ int padx(int i) { return i + (i >> 4); }

// Order LDS traffic within one wavefront (no other wave touches the region).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N>
__device__ __forceinline__ void powers(double2 w, double2* wp) {
  // wp[q] = w^q, q = 0..N-1
  wp[0] = make_double2(1.0, 0.0);
  wp[1] = w;
#pragma unroll
  for (int q = 2; q < N; ++q) wp[q] = cmul(wp[q - 1], w);
}

// Exchange 32 complex values through a wave region: value (b, q) is written at
// logical index widx(b, q) and value (b', q') is read back from ridx(b', q').
template <int NB_W, int NQ_W, int NB_R, int NQ_R, typename WF, typename RF>
__device__ __forceinline__ void wave_exchange(double* region, double2 (&v)[NB_W][NQ_W],
                                              double2 (&out)[NB_R][NQ_R], WF widx, RF ridx) {
#pragma unroll
  for (int b = 0; b < NB_W; ++b)
#pragma unroll
    for (int q = 0; q < NQ_W; ++q) region[padx(widx(b, q))] = v[b][q].x;
  wave_lds_sync();
#pragma unroll
  for (int b = 0; b < NB_R; ++b)
#pragma unroll
    for (int q = 0; q < NQ_R; ++q) out[b][q].x = region[padx(ridx(b, q))];
  wave_lds_sync();
#pragma unroll
  for (int b = 0; b < NB_W; ++b)
#pragma unroll
    for (int q = 0; q < NQ_W; ++q) region[padx(widx(b, q))] = v[b][q].y;
  wave_lds_sync();
#pragma unroll
  for (int b = 0; b < NB_R; ++b)
#pragma unroll
    for (int q = 0; q < NQ_R; ++q) out[b][q].y = region[padx(ridx(b, q))];
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
  wave_exchange(region, a, s, [&](int b, int q) { return 16 * (l + 64 * b) + q; },
                [&](int b, int q) { return l + 64 * b + 128 * q; });
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
  const int kB = l & 15;
  wave_exchange(region, s, c,
                [&](int b, int q) { return (l + 64 * b - kB) * 16 + kB + 16 * q; },
                [&](int b, int q) { return l + 64 * b + 256 * q; });
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
__global__ void __launch_bounds__(512)
x_fwd_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
             int nitems, FieldPtrs fields, float* __restrict__ ws) {
  extern __shared__ double lds_d[];
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  double* region = lds_d + w * kRegion;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const PatchDev* P = patches + wi.patch;
    const int z1 = wi.first;
    const double2* tw2048 = P->fx.tw;
    const double2* tw4096 = P->fz.tw;
    double2 twB = tw2048[8 * (l & 15)];
    double2 twC[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) twC[b] = tw2048[l + 64 * b];

    // load row z = z1 + 512 w as complex pairs
    const float2* row = reinterpret_cast<const float2*>(
        static_cast<const float*>(fields.f[wi.comp]) + P->off_real +
        (long long)(z1 + kN1 * w) * (2 * kMX));
    double2 a[2][16];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 16; ++q) a[b][q] = ld_f2(row + l + 64 * b + 128 * q);
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

    // output phase: kx = t + 512 i
    double2 tz[8];
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) tz[k2] = tw4096[(z1 * k2) & (kNZ - 1)];
    float2* out = reinterpret_cast<float2*>(ws) + P->off_spec + (long long)wi.comp * P->comp_stride;
#pragma unroll 1
    for (int i = 0; i < 4; ++i) {
      const int kx = threadIdx.x + 512 * i;
      const int km = (kMX - kx) & (kMX - 1);
      const double2 wk = P->post[kx];
      double2 X[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const float2* zr = reinterpret_cast<const float2*>(lds_d + r * kRegion);
        const double2 za = ld_f2(zr + kx);
        if (kx == 0) {
          X[r] = make_double2(za.x + za.y, za.x - za.y);
        } else {
          const double2 zb = ld_f2(zr + km);
          const double2 e = make_double2(0.5 * (za.x + zb.x), 0.5 * (za.y - zb.y));
          const double2 d = make_double2(za.x - zb.x, za.y + zb.y);
          const double2 o = make_double2(0.5 * d.y, -0.5 * d.x);
          X[r] = cadd(e, cmul(wk, o));
        }
      }
      DFT<8, -1>::run(X);
      float4* dst = reinterpret_cast<float4*>(out + (long long)kx * kNZ + 8 * z1);
#pragma unroll
      for (int k2 = 0; k2 < 8; k2 += 2) {
        const double2 u = cmul(X[k2], tz[k2]);
        const double2 v = cmul(X[k2 + 1], tz[k2 + 1]);
        dst[k2 / 2] = make_float4(static_cast<float>(u.x), static_cast<float>(u.y),
                                  static_cast<float>(v.x), static_cast<float>(v.y));
      }
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
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const PatchDev* P = patches + wi.patch;
    const int z1 = wi.first;
    const double2* tw2048 = P->fx.tw;
    const float2* in = reinterpret_cast<const float2*>(ws) + P->off_spec +
                       (long long)wi.comp * P->comp_stride;
    // phase 1: inverse DFT over k2 for each kx, into the FP32 staging rows
#pragma unroll 1
    for (int i = 0; i < 4; ++i) {
      const int kx = threadIdx.x + 512 * i;
      const float4* src = reinterpret_cast<const float4*>(in + (long long)kx * kNZ + 8 * z1);
      double2 X[8];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const float4 v = src[h];
        X[2 * h] = make_double2(v.x, v.y);
        X[2 * h + 1] = make_double2(v.z, v.w);
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
    double2 twB = cconj(tw2048[8 * (l & 15)]);
    double2 twC[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) twC[b] = cconj(tw2048[l + 64 * b]);
    const float2* zrow = reinterpret_cast<const float2*>(region);
    double2 a[2][16];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        __builtin_amdgcn_sched_barrier(0);
        const int k = l + 64 * b + 128 * q;
        const double2 xa = ld_f2(zrow + k);
        if (k == 0) {
          a[b][q] = make_double2(xa.x + xa.y, xa.x - xa.y);
        } else {
          const double2 xb = ld_f2(zrow + (kMX - k));
          const double2 p = make_double2(xa.x + xb.x, xa.y - xb.y);
          const double2 m = make_double2(xa.x - xb.x, xa.y + xb.y);
          const double2 t1 = cmul(cconj(P->post[k & (kMX - 1)]), m);
          a[b][q] = make_double2(p.x - t1.y, p.y + t1.x);
        }
      }
    wave_lds_sync();
    double2 c[4][8];
    wave_fft2048<1>(region, a, c, twB, twC);
    float2* row = reinterpret_cast<float2*>(static_cast<float*>(fields.f[wi.comp]) + P->off_real +
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
// Fused z pass on one column kx (4096 modes) per workgroup of 512 threads.
// Thread t = 8 j + k2 works on the 512-point transform of group k2 over
// z1 (or k1) and holds entries j + 64 q, q < 8.  LDS exchanges use two FP64
// buffers laid out [e][k2] (element e of group k2 at 8 e + k2): the eight
// lanes that the LDS serves together share j and differ in k2, so every
// exchange is bank-conflict free.
template <int SIGN>
__device__ __forceinline__ void fft512_group(double2 (&v)[8], double2* bufA, double2* bufB, int j,
                                             int k2, double2 w2, double2 w3) {
  // stage 1: radix 8, Ns = 1
  DFT<8, SIGN>::run(v);
#pragma unroll
  for (int q = 0; q < 8; ++q) bufA[(8 * j + q) * 8 + k2] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = bufA[(j + 64 * q) * 8 + k2];
  // stage 2: radix 8, Ns = 8, k = j mod 8
  {
    double2 wq = w2;
    v[1] = cmul(v[1], w2);
#pragma unroll
    for (int q = 2; q < 8; ++q) {
      wq = cmul(wq, w2);
      v[q] = cmul(v[q], wq);
    }
  }
  DFT<8, SIGN>::run(v);
  const int k = j & 7;
#pragma unroll
  for (int q = 0; q < 8; ++q) bufB[((j - k) * 8 + k + 8 * q) * 8 + k2] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = bufB[(j + 64 * q) * 8 + k2];
  // stage 3: radix 8, Ns = 64, k = j
  {
    double2 wq = w3;
    v[1] = cmul(v[1], w3);
#pragma unroll
    for (int q = 2; q < 8; ++q) {
      wq = cmul(wq, w3);
      v[q] = cmul(v[q], wq);
    }
  }
  DFT<8, SIGN>::run(v);
}

// Forward transform of one component column into FP32 registers (modes t + 512 q).
__device__ __forceinline__ void z_forward(const float2* src, float2 (&dst)[8], double2* bufA,
                                          double2* bufB, int t, int j, int k2, double2 w2,
                                          double2 w3) {
  double2 v[8];
  // uniform base per q plus one 32-bit lane offset (SGPR-base addressing)
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float2* __restrict__ bq = src + 512 * q;
    v[q] = ld_f2(bq + t);
  }
  fft512_group<-1>(v, bufA, bufB, j, k2, w2, w3);
#pragma unroll
  for (int q = 0; q < 8; ++q) dst[q] = st2(v[q]);
}

// Inverse transform of one component held in registers, twiddle W4096^(-z1 k2), store.
__device__ __forceinline__ void z_inverse(const float2 (&src)[8], float2* dst, double2* bufA,
                                          double2* bufB, int t, int j, int k2, double2 w2i,
                                          double2 w3i, const double2* __restrict__ tw4096) {
  double2 v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = ld2(src[q]);
  fft512_group<1>(v, bufA, bufB, j, k2, w2i, w3i);
  // W4096^(-z1 k2) for z1 = j + 64 q: start at W^(-j k2), step W^(-64 k2)
  double2 tq = cconj(tw4096[(j * k2) & (kNZ - 1)]);
  const double2 step = cconj(tw4096[(64 * k2) & (kNZ - 1)]);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    float2* __restrict__ bq = dst + 512 * q;
    bq[t] = st2(cmul(v[q], tq));
    if (q < 7) tq = cmul(tq, step);
  }
}

// One polarization group of one column (G = 0: s-pol, G = 1: p-pol), in three
// phases so that at most three transformed fields, three source contributions
// and the per-mode C and S are live at once:
//   sources: transform J (and rho), evaluate the coefficients, fold the
//            sources into three contributions per mode;
//   fields:  transform E and B, apply C, S and the contributions;
//   inverse: transform the three updated components back.
template <int G, int SRC>
__device__ __forceinline__ void z_group(const PatchDev* P, int kxcol, float* ws, const Physics& ph,
                                        double2* bufA, double2* bufB, const double2& w2,
                                        const double2& w3) {
  constexpr bool kSrc = SRC != kVacuum;
  constexpr int kF0 = G == 0 ? kEy : kEx;
  constexpr int kF1 = G == 0 ? kBx : kEz;
  constexpr int kF2 = G == 0 ? kBz : kBy;
  const int t = threadIdx.x;
  const int k2 = t & 7;
  const int j = t >> 3;
  float2* col = reinterpret_cast<float2*>(ws) + P->off_spec + (long long)kxcol * kNZ;
  const long long cs = P->comp_stride;
  const double kx = P->kx[kxcol];
  const double dt = P->dt;

  float2 sc[3][8];  // source contributions
  double cC[8], cS[8], cL[8];
  if constexpr (kSrc) {
    if constexpr (G == 0) {
      float2 jy[8];
      z_forward(col + kJy * cs, jy, bufA, bufB, t, j, k2, w2, w3);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double* __restrict__ kzq = P->kz + 512 * q;
        const double kz = kzq[t];
        const Coef cf = psatd_coef(sqrt(kx * kx + kz * kz), dt, ph.c, ph.eps0, P->inv_n);
        cC[q] = cf.C;
        cS[q] = cf.S;
        double2 a, b, c;
        src_2d_s(kx, kz, cf, ld2(jy[q]), a, b, c);
        sc[0][q] = st2(a);
        sc[1][q] = st2(b);
        sc[2][q] = st2(c);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      float2 jx[8], jz[8], ro[8], rn[8];
      z_forward(col + kJx * cs, jx, bufA, bufB, t, j, k2, w2, w3);
      z_forward(col + kJz * cs, jz, bufA, bufB, t, j, k2, w2, w3);
      if constexpr (SRC == kRho) {
        z_forward(col + kRhoOld * cs, ro, bufA, bufB, t, j, k2, w2, w3);
        z_forward(col + kRhoNew * cs, rn, bufA, bufB, t, j, k2, w2, w3);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double* __restrict__ kzq = P->kz + 512 * q;
        const double kz = kzq[t];
        const Coef cf = psatd_coef(sqrt(kx * kx + kz * kz), dt, ph.c, ph.eps0, P->inv_n);
        cC[q] = cf.C;
        cS[q] = cf.S;
        cL[q] = ph.eps0 * ph.c * ph.c * cf.X1;
        double2 a, b, c;
        const double2 zero = make_double2(0.0, 0.0);
        src_2d_p<SRC>(kx, kz, cf, dt, ld2(jx[q]), ld2(jz[q]),
                      SRC == kRho ? ld2(ro[q]) : zero, SRC == kRho ? ld2(rn[q]) : zero, a, b, c);
        sc[0][q] = st2(a);
        sc[1][q] = st2(b);
        sc[2][q] = st2(c);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  float2 f[3][8];
  z_forward(col + kF0 * cs, f[0], bufA, bufB, t, j, k2, w2, w3);
  z_forward(col + kF1 * cs, f[1], bufA, bufB, t, j, k2, w2, w3);
  z_forward(col + kF2 * cs, f[2], bufA, bufB, t, j, k2, w2, w3);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double* __restrict__ kzq = P->kz + 512 * q;
        const double kz = kzq[t];
    double C, S, L1 = 0.0;
    double2 s0 = make_double2(0.0, 0.0), s1 = s0, s2 = s0;
    if constexpr (kSrc) {
      C = cC[q];
      S = cS[q];
      L1 = cL[q];
      s0 = ld2(sc[0][q]);
      s1 = ld2(sc[1][q]);
      s2 = ld2(sc[2][q]);
    } else {
      const Coef cf = psatd_coef(sqrt(kx * kx + kz * kz), dt, ph.c, ph.eps0, P->inv_n);
      C = cf.C;
      S = cf.S;
    }
    double2 a = ld2(f[0][q]), b = ld2(f[1][q]), c = ld2(f[2][q]);
    if constexpr (G == 0) fld_2d_s(kx, kz, C, S, ph.c, a, b, c, s0, s1, s2);
    else fld_2d_p<SRC>(kx, kz, C, S, L1, ph.c, a, b, c, s0, s1, s2);
    f[0][q] = st2(a);
    f[1][q] = st2(b);
    f[2][q] = st2(c);
    __builtin_amdgcn_sched_barrier(0);
  }
  const double2 w2i = cconj(w2), w3i = cconj(w3);
  const double2* tw4096 = P->fz.tw;
  z_inverse(f[0], col + kF0 * cs, bufA, bufB, t, j, k2, w2i, w3i, tw4096);
  z_inverse(f[1], col + kF1 * cs, bufA, bufB, t, j, k2, w2i, w3i, tw4096);
  z_inverse(f[2], col + kF2 * cs, bufA, bufB, t, j, k2, w2i, w3i, tw4096);
}

template <int SRC>
__global__ void __launch_bounds__(512)
z_fused_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
               int nitems, float* __restrict__ ws, Physics ph) {
  extern __shared__ double2 lds2[];
  double2* bufA = lds2;
  double2* bufB = lds2 + kNZ;
  const int j = threadIdx.x >> 3;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const PatchDev* P = patches + wi.patch;
    const double2* tw4096 = P->fz.tw;
    const double2 w2 = tw4096[64 * (j & 7)];  // exp(-2 pi i (j mod 8) / 64)
    const double2 w3 = tw4096[8 * j];         // exp(-2 pi i j / 512)
    z_group<0, SRC>(P, wi.first, ws, ph, bufA, bufB, w2, w3);
    z_group<1, SRC>(P, wi.first, ws, ph, bufA, bufB, w2, w3);
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

hipError_t launch_z_fused(int src, const LaunchShape& sh, hipStream_t s, const PatchDev* p,
                          const WorkItem* it, int n, void* ws, Physics ph) {
  float* w = static_cast<float*>(ws);
  switch (src) {
    case kVacuum:
      hipLaunchKernelGGL(z_fused_kernel<kVacuum>, dim3(sh.grid), dim3(sh.block), sh.lds_bytes, s,
                         p, it, n, w, ph);
      break;
    case kRho:
      hipLaunchKernelGGL(z_fused_kernel<kRho>, dim3(sh.grid), dim3(sh.block), sh.lds_bytes, s, p,
                         it, n, w, ph);
      break;
    default:
      hipLaunchKernelGGL(z_fused_kernel<kJForm>, dim3(sh.grid), dim3(sh.block), sh.lds_bytes, s,
                         p, it, n, w, ph);
      break;
  }
  return hipGetLastError();
}

hipError_t configure_attributes() {
  const int lim = 160 * 1024;
  hipError_t e = hipSuccess, r;
  const void* fns[] = {reinterpret_cast<const void*>(&x_fwd_kernel),
                       reinterpret_cast<const void*>(&x_inv_kernel),
                       reinterpret_cast<const void*>(&z_fused_kernel<kVacuum>),
                       reinterpret_cast<const void*>(&z_fused_kernel<kRho>),
                       reinterpret_cast<const void*>(&z_fused_kernel<kJForm>)};
  for (const void* f : fns)
    if ((r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim)) != hipSuccess)
      e = r;
  return e;
}

size_t x_lds_bytes() { return sizeof(double) * kRegion * kWaves; }
size_t z_lds_bytes() { return sizeof(double2) * 2 * kNZ; }

}  // namespace fast2d
}  // namespace psatd
