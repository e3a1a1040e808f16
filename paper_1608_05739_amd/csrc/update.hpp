// Per-mode PSATD update (Sec. III.B, item 2; Table 1, PSATD row), FP64.
//
// With theta = c|k|dt:
//   C  = cos theta
//   S  = sin theta / (c|k|)              = dt sinc(theta)
//   X1 = (1 - C) / (eps0 c^2 |k|^2)      = dt^2 sinc(theta/2)^2 / (2 eps0)
//   X2 = (1 - sinc theta) / (eps0 |k|^2) = c^2 dt^2 g(theta) / eps0
//   X3 = (C - sinc theta) / (eps0 |k|^2) = c^2 dt^2 (g - sinc(theta/2)^2 / 2) / eps0
// where g(theta) = (1 - sinc theta) / theta^2 uses its Taylor series below
// theta = 0.25, so no coefficient is formed by cancelling subtraction and all
// are finite at k = 0.  One sincos of theta/2 gives every trigonometric value.
//
//   rho form: E' = C E + i c^2 S (k x B) - (S/eps0) J + i k (X3 rho_old - X2 rho_new)
//   J form:   E' = C E + i c^2 S (k x B) - (S/eps0) J + eps0 c^2 X1 k (k.E) - dt X2 k (k.J)
//             B' = C B - i S (k x E) + i X1 (k x J)
// Every coefficient is multiplied by `scale` (the 1/N of the inverse FFTs).
#pragma once

#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "internal.hpp"

namespace psatd {

struct Coef {
  double C, S, X1, X2, X3;
  double Se;  // S / eps0
};

// sin and cos of a bounded argument, |h| <= kSincosMax.  Cody-Waite reduction
// h = n pi/2 + r with pi/2 split into three parts (the first two with 33
// significant bits, so n * part is exact for |n| < 2^20), then the Taylor
// series of sin to r^17 and of cos to r^18 on |r| <= pi/4 (truncation below
// 1e-18 relative).  Written with explicit fma so host and device round alike.
constexpr double kSincosMax = 1.0e5;

// Polynomial constants live in a constant-memory table so that, inside
// persistent loops, they stay in scalar registers instead of being hoisted
// into vector registers.
struct TrigConsts {
  double two_over_pi, p1, p2, p3;
  double s[8];  // 1/17!, -1/15!, ..., -1/3!   (Horner order)
  double c[9];  // -1/18!, 1/16!, ..., -1/2!
  double g[6];  // 1/6, 1/120, 1/5040, 1/362880, 1/39916800, 1/6227020800
};

#define PSATD_TRIG_CONSTS                                                                      \
  {0.63661977236758138, 1.5707963267341256, 6.077100506303966e-11, 2.0222662487959506e-21,     \
   {2.8114572543455206e-15, -7.647163731819816e-13, 1.6059043836821613e-10,                    \
    -2.505210838544172e-08, 2.7557319223985893e-06, -1.984126984126984e-04,                    \
    8.333333333333333e-03, -1.6666666666666666e-01},                                           \
   {-1.5619206968586225e-16, 4.779477332387385e-14, -1.1470745597729725e-11,                   \
    2.08767569878681e-09, -2.755731922398589e-07, 2.48015873015873e-05, -1.388888888888889e-03, \
    4.1666666666666664e-02, -0.5},                                                             \
   {1.0 / 6.0, 1.0 / 120.0, 1.0 / 5040.0, 1.0 / 362880.0, 1.0 / 39916800.0, 1.0 / 6227020800.0}}

__constant__ static const TrigConsts kTrigDev = PSATD_TRIG_CONSTS;
static const TrigConsts kTrigHost = PSATD_TRIG_CONSTS;

__host__ __device__ inline const TrigConsts& trig_consts() {
#if defined(__HIP_DEVICE_COMPILE__)
  return kTrigDev;
#else
  return kTrigHost;
#endif
}

__host__ __device__ inline void psatd_sincos(double h, double* s_out, double* c_out) {
  const TrigConsts& T = trig_consts();
  const double n = rint(h * T.two_over_pi);
  double r = fma(-n, T.p1, h);
  r = fma(-n, T.p2, r);
  r = fma(-n, T.p3, r);
  const double r2 = r * r;
  double ps = T.s[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) ps = fma(ps, r2, T.s[i]);
  const double sr = fma(r * r2, ps, r);
  double pc = T.c[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) pc = fma(pc, r2, T.c[i]);
  const double cr = fma(r2, pc, 1.0);
  const int quad = static_cast<int>(n) & 3;
  const double sv = (quad & 1) ? cr : sr;
  const double cv = (quad & 1) ? sr : cr;
  *s_out = (quad & 2) ? -sv : sv;
  *c_out = ((quad + 1) & 2) ? -cv : cv;
}

__host__ __device__ inline Coef psatd_coef(double K, double dt, double c, double eps0,
                                           double scale) {
  const double th = c * K * dt;
  const double h = 0.5 * th;
  double sh, ch;
  psatd_sincos(h, &sh, &ch);
  const double ih = (h > 0.0) ? 1.0 / h : 0.0;
  const double sinc_h = (h > 0.0) ? sh * ih : 1.0;
  const double sinc_th = sinc_h * ch;  // sin(th)/th = (2 sh ch)/(2 h)
  // Both forms are evaluated and one is selected: no divergent branch.
  const TrigConsts& T = trig_consts();
  const double t2 = th * th;
  const double g_series =
      T.g[0] - t2 * (T.g[1] - t2 * (T.g[2] - t2 * (T.g[3] - t2 * (T.g[4] - t2 * T.g[5]))));
  const double g_direct = (1.0 - sinc_th) * (0.25 * ih * ih);  // (1 - sinc th) / th^2
  const double g = (th < 0.25) ? g_series : g_direct;
  const double ie = scale / eps0;
  Coef k;
  k.C = (ch - sh) * (ch + sh) * scale;
  k.S = dt * sinc_th * scale;
  k.Se = dt * sinc_th * ie;
  k.X1 = dt * dt * sinc_h * sinc_h * 0.5 * ie;
  k.X2 = c * c * dt * dt * g * ie;
  k.X3 = c * c * dt * dt * (g - 0.5 * sinc_h * sinc_h) * ie;
  return k;
}

// i * a * s  for real s
__device__ __forceinline__ double2 i_times(double2 a, double s) {
  return make_double2(-a.y * s, a.x * s);
}

// Advance one mode.  in: E[3], B[3], J[3], rho_old, rho_new (unused slots
// ignored according to SRC).  out: E'[3], B'[3].
template <int SRC>
__device__ __forceinline__ void update_mode(const double kx, const double ky, const double kz,
                                            const Coef& q, double c, double eps0, double dt,
                                            const double2* E, const double2* B, const double2* J,
                                            double2 ro, double2 rn, double2* Eo, double2* Bo) {
  const double kv[3] = {kx, ky, kz};
  // k x B, k x E
  const double2 kxB[3] = {
      csub(cscale(B[2], ky), cscale(B[1], kz)),
      csub(cscale(B[0], kz), cscale(B[2], kx)),
      csub(cscale(B[1], kx), cscale(B[0], ky))};
  const double2 kxE[3] = {
      csub(cscale(E[2], ky), cscale(E[1], kz)),
      csub(cscale(E[0], kz), cscale(E[2], kx)),
      csub(cscale(E[1], kx), cscale(E[0], ky))};
  const double cS = c * c * q.S;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Eo[i] = cadd(cscale(E[i], q.C), i_times(kxB[i], cS));
    Bo[i] = csub(cscale(B[i], q.C), i_times(kxE[i], q.S));
  }
  if constexpr (SRC == kJForm) {
    const double2 kdE = cadd(cadd(cscale(E[0], kx), cscale(E[1], ky)), cscale(E[2], kz));
    const double a = eps0 * c * c * q.X1;
#pragma unroll
    for (int i = 0; i < 3; ++i) Eo[i] = cadd(Eo[i], cscale(kdE, a * kv[i]));
  }
  if constexpr (SRC != kVacuum) {
    const double2 kxJ[3] = {
        csub(cscale(J[2], ky), cscale(J[1], kz)),
        csub(cscale(J[0], kz), cscale(J[2], kx)),
        csub(cscale(J[1], kx), cscale(J[0], ky))};
    const double sj = q.S / eps0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Eo[i] = csub(Eo[i], cscale(J[i], sj));
      Bo[i] = cadd(Bo[i], i_times(kxJ[i], q.X1));
    }
    if constexpr (SRC == kJForm) {
      const double2 kdJ = cadd(cadd(cscale(J[0], kx), cscale(J[1], ky)), cscale(J[2], kz));
      const double b = dt * q.X2;
#pragma unroll
      for (int i = 0; i < 3; ++i) Eo[i] = csub(Eo[i], cscale(kdJ, b * kv[i]));
    } else {
      const double2 lam = csub(cscale(ro, q.X3), cscale(rn, q.X2));
#pragma unroll
      for (int i = 0; i < 3; ++i) Eo[i] = cadd(Eo[i], i_times(lam, kv[i]));
    }
  }
}

// PSTD leapfrog step of one mode (Table 1, PSTD row: spectral derivatives,
// finite differences in time), the contrast solver.  B is at half-integer
// times:
//   B' = B - i dt (k x E),   E' = E + i c^2 dt (k x B') - (dt/eps0) J
// and both results are multiplied by `scale`.
template <int SRC>
__device__ __forceinline__ void pstd_update_mode(const double kx, const double ky,
                                                 const double kz, double dt, double c,
                                                 double eps0, double scale, const double2* E,
                                                 const double2* B, const double2* J, double2* Eo,
                                                 double2* Bo) {
  const double2 kxE[3] = {
      csub(cscale(E[2], ky), cscale(E[1], kz)),
      csub(cscale(E[0], kz), cscale(E[2], kx)),
      csub(cscale(E[1], kx), cscale(E[0], ky))};
  double2 Bn[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Bn[i] = csub(B[i], i_times(kxE[i], dt));
  const double2 kxB[3] = {
      csub(cscale(Bn[2], ky), cscale(Bn[1], kz)),
      csub(cscale(Bn[0], kz), cscale(Bn[2], kx)),
      csub(cscale(Bn[1], kx), cscale(Bn[0], ky))};
  const double cdt = c * c * dt;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double2 e = cadd(E[i], i_times(kxB[i], cdt));
    if constexpr (SRC == kPstdJ) e = csub(e, cscale(J[i], dt / eps0));
    Eo[i] = cscale(e, scale);
    Bo[i] = cscale(Bn[i], scale);
  }
}

// ------------------------------------------------------------------ 2D forms
// In 2D (k_y = 0) the update splits into two independent sets:
//   s-polarization (Ey, Bx, Bz; Jy):
//     Ey' = C Ey + i c^2 S (kz Bx - kx Bz) - (S/eps0) Jy
//     Bx' = C Bx + i S kz Ey - i X1 kz Jy
//     Bz' = C Bz - i S kx Ey + i X1 kx Jy
//   p-polarization (Ex, Ez, By; Jx, Jz, rho):
//     Ex' = C Ex - i c^2 S kz By - (S/eps0) Jx + [longitudinal]_x
//     Ez' = C Ez + i c^2 S kx By - (S/eps0) Jz + [longitudinal]_z
//     By' = C By - i S (kz Ex - kx Ez) + i X1 (kz Jx - kx Jz)
//   [longitudinal] = i k (X3 rho_old - X2 rho_new)                       (rho form)
//                  = eps0 c^2 X1 k (k.E) - dt X2 k (k.J)                 (J form)
// These are the general update with k_y = 0 written out, so that no term is
// multiplied by an explicit zero.

// FP32 storage <-> FP64 arithmetic.
__device__ __forceinline__ double2 ld2(const float2& v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ float2 st2(double2 v) {
  return make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
}

// ------------------------------------------------------------------ 2D, sources
// The source part of the 2D update, evaluated once the sources are
// transformed (the field part is accumulated term by term by the z pass).
// It returns the contributions
//   s-pol: sEy = -(S/eps0) Jy,  sBx = -i X1 kz Jy,  sBz = i X1 kx Jy
//   p-pol: sEx = -(S/eps0) Jx + Lx,  sEz = -(S/eps0) Jz + Lz,  sBy = i X1 (kz Jx - kx Jz)
//          L = i k (X3 rho_old - X2 rho_new)      (rho form)
//          L = -dt X2 k (k.J)                      (J form)
// to which the field part adds C E + i c^2 S (k x B) [+ eps0 c^2 X1 k (k.E),
// J form] and C B - i S (k x E).
__device__ __forceinline__ void src_2d_s(double kx, double kz, const Coef& q, double2 jy,
                                         double2& sEy, double2& sBx, double2& sBz) {
  sEy = make_double2(-q.Se * jy.x, -q.Se * jy.y);
  sBx = make_double2(q.X1 * kz * jy.y, -q.X1 * kz * jy.x);
  sBz = make_double2(-q.X1 * kx * jy.y, q.X1 * kx * jy.x);
}

template <int SRC>
__device__ __forceinline__ void src_2d_p(double kx, double kz, const Coef& q, double dt,
                                         double2 jx, double2 jz, double2 ro, double2 rn,
                                         double2& sEx, double2& sEz, double2& sBy) {
  sEx = make_double2(-q.Se * jx.x, -q.Se * jx.y);
  sEz = make_double2(-q.Se * jz.x, -q.Se * jz.y);
  const double2 kj = make_double2(kz * jx.x - kx * jz.x, kz * jx.y - kx * jz.y);
  sBy = make_double2(-q.X1 * kj.y, q.X1 * kj.x);
  if constexpr (SRC == kJForm) {
    const double b = dt * q.X2;
    const double2 kdJ = make_double2(kx * jx.x + kz * jz.x, kx * jx.y + kz * jz.y);
    sEx.x -= b * kx * kdJ.x;
    sEx.y -= b * kx * kdJ.y;
    sEz.x -= b * kz * kdJ.x;
    sEz.y -= b * kz * kdJ.y;
  } else if constexpr (SRC == kRho) {
    const double2 lam = make_double2(q.X3 * ro.x - q.X2 * rn.x, q.X3 * ro.y - q.X2 * rn.y);
    sEx.x -= kx * lam.y;
    sEx.y += kx * lam.x;
    sEz.x -= kz * lam.y;
    sEz.y += kz * lam.x;
  }
}

}  // namespace psatd
