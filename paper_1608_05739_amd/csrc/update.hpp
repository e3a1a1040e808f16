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
};

__device__ __forceinline__ double g_of_theta(double th, double sinc_th) {
  if (th < 0.25) {
    const double t2 = th * th;
    return 1.0 / 6.0 -
           t2 * (1.0 / 120.0 -
                 t2 * (1.0 / 5040.0 -
                       t2 * (1.0 / 362880.0 - t2 * (1.0 / 39916800.0 - t2 / 6227020800.0))));
  }
  return (1.0 - sinc_th) / (th * th);
}

__device__ __forceinline__ Coef psatd_coef(double K, double dt, double c, double eps0,
                                           double scale) {
  const double th = c * K * dt;
  const double h = 0.5 * th;
  double sh, ch;
  sincos(h, &sh, &ch);
  const double sinc_h = (h > 0.0) ? sh / h : 1.0;
  const double sinc_th = sinc_h * ch;  // sin(th)/th = (2 sh ch)/(2 h)
  const double g = g_of_theta(th, sinc_th);
  Coef k;
  k.C = (ch - sh) * (ch + sh) * scale;
  k.S = dt * sinc_th * scale;
  k.X1 = dt * dt * sinc_h * sinc_h / (2.0 * eps0) * scale;
  k.X2 = c * c * dt * dt * g / eps0 * scale;
  k.X3 = c * c * dt * dt * (g - 0.5 * sinc_h * sinc_h) / eps0 * scale;
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

}  // namespace psatd
