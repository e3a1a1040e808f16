// Device FFT building blocks for gfx950: FP64 complex arithmetic, small DFTs
// with compile-time twiddles, and a Stockham autosort stage over lines held
// in LDS.  Storage precision is chosen by the callers; arithmetic here is FP64
// (full rate on CDNA4, the same as unpacked FP32).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"

namespace psatd {

// ------------------------------------------------------------------ complex
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) {
  return make_double2(a.x * s, a.y * s);
}
// a * (SIGN * i)
template <int SIGN>
__device__ __forceinline__ double2 mul_si(double2 a) {
  if constexpr (SIGN > 0) return make_double2(-a.y, a.x);
  else return make_double2(a.y, -a.x);
}

// Element i of a plan table (device memory), read through a global-address-
// space pointer: a global load, counted by vmcnt only, instead of a flat load,
// which every LDS wait (lgkmcnt) would also wait for.  (The host pass of the
// compiler, which never runs this, reads through the plain pointer.)
template <typename T>
__device__ __forceinline__ T gload(const T* p, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
  const __attribute__((address_space(1))) T* g = (const __attribute__((address_space(1))) T*)p;
  return g[i];
#else
  return p[i];
#endif
}

// ------------------------------------------------------------------ static_for
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// exp(2 pi i m / 16) for m in [0, 16), built from three constants so that
// the table is exactly symmetric.
constexpr double kC1 = 0.92387953251128674;  // cos(pi/8)
constexpr double kS1 = 0.38268343236508978;  // sin(pi/8)
constexpr double kR2 = 0.70710678118654752;  // sqrt(1/2)

constexpr double cos16(int m) {
  constexpr double t[16] = {1.0, kC1, kR2, kS1, 0.0, -kS1, -kR2, -kC1,
                            -1.0, -kC1, -kR2, -kS1, 0.0, kS1, kR2, kC1};
  return t[m];
}
constexpr double sin16(int m) {
  constexpr double t[16] = {0.0, kS1, kR2, kC1, 1.0, kC1, kR2, kS1,
                            0.0, -kS1, -kR2, -kC1, -1.0, -kC1, -kR2, -kS1};
  return t[m];
}

// a * exp(SIGN * 2 pi i M / N) for N dividing 16.
template <int N, int M, int SIGN>
__device__ __forceinline__ double2 twc(double2 a) {
  constexpr int m = ((M % N) + N) % N;
  constexpr int q = m * (16 / N);
  if constexpr (q == 0) return a;
  else if constexpr (q == 4) return mul_si<SIGN>(a);
  else if constexpr (q == 8) return make_double2(-a.x, -a.y);
  else if constexpr (q == 12) return mul_si<-SIGN>(a);
  else return cmul(a, make_double2(cos16(q), SIGN * sin16(q)));
}

// exp(2 pi i m / 12) from two constants (multiples of 30 degrees).
constexpr double kH3 = 0.86602540378443865;  // sqrt(3)/2
constexpr double cos12(int m) {
  constexpr double t[12] = {1.0, kH3, 0.5, 0.0, -0.5, -kH3, -1.0, -kH3, -0.5, 0.0, 0.5, kH3};
  return t[m];
}
constexpr double sin12(int m) {
  constexpr double t[12] = {0.0, 0.5, kH3, 1.0, kH3, 0.5, 0.0, -0.5, -kH3, -1.0, -kH3, -0.5};
  return t[m];
}

// a * exp(SIGN * 2 pi i M / N) for N dividing 16 or N = 12.
template <int N, int M, int SIGN>
__device__ __forceinline__ double2 twn(double2 a) {
  if constexpr (16 % N == 0) {
    return twc<N, M, SIGN>(a);
  } else {
    static_assert(N == 12, "compile-time twiddles for N dividing 16, or 12");
    constexpr int m = ((M % 12) + 12) % 12;
    if constexpr (m == 0) return a;
    else if constexpr (m == 3) return mul_si<SIGN>(a);
    else if constexpr (m == 6) return make_double2(-a.x, -a.y);
    else if constexpr (m == 9) return mul_si<-SIGN>(a);
    else return cmul(a, make_double2(cos12(m), SIGN * sin12(m)));
  }
}

// ------------------------------------------------------------------ small DFTs
// In-place DFT of length R: v[k] <- sum_n v[n] exp(SIGN 2 pi i n k / R).
template <int R, int SIGN>
struct DFT;

template <int SIGN>
struct DFT<2, SIGN> {
  static __device__ __forceinline__ void run(double2* v) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int SIGN>
struct DFT<3, SIGN> {
  static __device__ __forceinline__ void run(double2* v) {
    constexpr double kH = 0.86602540378443865;  // sqrt(3)/2
    const double2 t = cadd(v[1], v[2]);
    const double2 u = make_double2(v[0].x - 0.5 * t.x, v[0].y - 0.5 * t.y);
    const double2 w = mul_si<SIGN>(cscale(csub(v[1], v[2]), kH));
    v[0] = cadd(v[0], t);
    v[1] = cadd(u, w);
    v[2] = csub(u, w);
  }
};

template <int SIGN>
struct DFT<4, SIGN> {
  static __device__ __forceinline__ void run(double2* v) {
    const double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const double2 c = cadd(v[1], v[3]), d = mul_si<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

// N = R1 R2 with n = R2 n1 + n2 and k = k1 + R1 k2:
//   X[k1 + R1 k2] = sum_n2 W_N^{n2 k1} W_R2^{n2 k2} sum_n1 x[R2 n1 + n2] W_R1^{n1 k1}.
template <int R1, int R2, int SIGN>
__device__ __forceinline__ void dft_split(double2* x) {
  constexpr int N = R1 * R2;
  double2 a[R2][R1];
  static_for<0, R2>([&](auto n2c) __attribute__((always_inline)) {
    constexpr int n2 = decltype(n2c)::value;
    double2 t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = x[R2 * n1 + n2];
    DFT<R1, SIGN>::run(t);
    static_for<0, R1>([&](auto k1c) __attribute__((always_inline)) {
      constexpr int k1 = decltype(k1c)::value;
      a[n2][k1] = twn<N, n2 * k1, SIGN>(t[k1]);
    });
  });
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    double2 t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = a[n2][k1];
    DFT<R2, SIGN>::run(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) x[k1 + R1 * k2] = t[k2];
  }
}

template <int SIGN>
struct DFT<8, SIGN> {
  static __device__ __forceinline__ void run(double2* v) { dft_split<2, 4, SIGN>(v); }
};

template <int SIGN>
struct DFT<16, SIGN> {
  static __device__ __forceinline__ void run(double2* v) { dft_split<4, 4, SIGN>(v); }
};

template <int SIGN>
struct DFT<12, SIGN> {
  static __device__ __forceinline__ void run(double2* v) { dft_split<4, 3, SIGN>(v); }
};

// ------------------------------------------------------------------ LDS layout and indices
// Lines in LDS are padded by one element every 16: logical element i sits at
// lpad(i) = i + floor(i / 16).  A radix-R stage writes element (j R + q) from
// lane j; without the padding the lanes of a wave would all hit the same LDS
// banks when R is 8 or 16.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// Elements of LDS holding n logical elements.
__host__ __device__ constexpr int lpad_size(int n) { return n + (n >> 4) + 1; }

// q = x / d, r = x mod d for a divisor that every lane shares (a power of two
// takes a shift and a mask).
__device__ __forceinline__ void udivmod(int x, int d, int& q, int& r) {
  if ((d & (d - 1)) == 0) {
    const int s = __builtin_ctz(d);
    q = x >> s;
    r = x & (d - 1);
  } else {
    q = x / d;
    r = x - q * d;
  }
}

// Walks idx = threadIdx.x + t blockDim.x as (hi, lo) = (idx / n, idx mod n):
// one division per thread, then every step adds blockDim.x with a carry.
struct Walk2 {
  int hi, lo, dhi, dlo, n;
  __device__ __forceinline__ explicit Walk2(int n_) : n(n_) {
    udivmod(static_cast<int>(threadIdx.x), n, hi, lo);
    udivmod(static_cast<int>(blockDim.x), n, dhi, dlo);
  }
  __device__ __forceinline__ void next() {
    hi += dhi;
    lo += dlo;
    if (lo >= n) {
      lo -= n;
      ++hi;
    }
  }
};

// ------------------------------------------------------------------ Stockham stage
// One radix-R stage over nl lines of length L stored in LDS (line stride LS
// in logical elements, padded by lpad; in place).  Ns is the product of the radices already applied.  Butterfly
// j of a line reads x[j + q L/R], multiplies by w^q with
// w = exp(SIGN 2 pi i (j mod Ns) / (Ns R)), applies DFT<R> and writes
// y[(j - j mod Ns) R + j mod Ns + q Ns].  Each thread handles at most
// MAXPTS / R butterflies (the planner guarantees that).
template <int R, int SIGN, int MAXPTS>
__device__ __forceinline__ void lds_stage(double2* lds, int L, int nl, int LS, int Ns,
                                          const double2* __restrict__ tw) {
  constexpr int BPT = MAXPTS / R;
  const int nb = L / R;
  const int twstride = L / (Ns * R);
  // butterfly b = threadIdx.x + t blockDim.x is index j of line `line`, and
  // k = j mod Ns; Ns divides nb, so a carry out of j leaves k unchanged
  Walk2 w(nb);
  int k, dk, unused;
  udivmod(w.lo, Ns, unused, k);
  udivmod(w.dlo, Ns, unused, dk);
  // Twiddles first, for every butterfly slot (k < Ns keeps the index inside
  // the table even for slots past the tile), so that they are in flight
  // during the LDS reads; k = 0 takes tw[0] = 1, which multiplies exactly.
  // The first stage (Ns = 1) has k = 0 throughout and needs none.
  const bool twiddled = Ns > 1;
  double2 wt[BPT];
  if (twiddled) {
    int kk = k;
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      wt[t] = gload(tw, kk * twstride);
      kk += dk;
      if (kk >= Ns) kk -= Ns;
    }
  }
  double2 v[BPT][R];
  int obase[BPT];
#pragma unroll
  for (int t = 0; t < BPT; ++t) {
    obase[t] = -1;
    if (w.hi < nl) {
      const int src = w.hi * LS + w.lo;
#pragma unroll
      for (int q = 0; q < R; ++q) v[t][q] = lds[lpad(src + q * nb)];
      obase[t] = w.hi * LS + (w.lo - k) * R + k;
    }
    w.next();
    k += dk;
    if (k >= Ns) k -= Ns;
  }
#pragma unroll
  for (int t = 0; t < BPT; ++t) {
    if (twiddled && obase[t] >= 0) {
      double2 u = wt[t];
      if constexpr (SIGN > 0) u.y = -u.y;
      double2 uq = u;
      v[t][1] = cmul(v[t][1], u);
#pragma unroll
      for (int q = 2; q < R; ++q) {
        uq = cmul(uq, u);
        v[t][q] = cmul(v[t][q], uq);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < BPT; ++t) {
    if (obase[t] >= 0) {
      DFT<R, SIGN>::run(v[t]);
#pragma unroll
      for (int q = 0; q < R; ++q) lds[lpad(obase[t] + q * Ns)] = v[t][q];
    }
  }
  __syncthreads();
}

// Full complex FFT (unnormalized) of nl lines in LDS, radices from a plan in
// global memory.  SIGN = -1 forward, +1 inverse.  Ends with a barrier.
template <int SIGN, int MAXPTS>
__device__ __forceinline__ void fft_lds(double2* lds, int nl, int LS, const FFTPlanDev* __restrict__ f) {
  const int L = f->n;
  const int ns = f->nstages;
  const double2* tw = f->tw;
  int Ns = 1;
  for (int s = 0; s < ns; ++s) {
    const int R = f->radix[s];
    if (MAXPTS >= 16 && R == 16) {
      if constexpr (MAXPTS >= 16) lds_stage<16, SIGN, MAXPTS>(lds, L, nl, LS, Ns, tw);
    } else if (R == 8) {
      lds_stage<8, SIGN, MAXPTS>(lds, L, nl, LS, Ns, tw);
    } else if (R == 4) {
      lds_stage<4, SIGN, MAXPTS>(lds, L, nl, LS, Ns, tw);
    } else if (R == 3) {
      lds_stage<3, SIGN, MAXPTS>(lds, L, nl, LS, Ns, tw);
    } else {
      lds_stage<2, SIGN, MAXPTS>(lds, L, nl, LS, Ns, tw);
    }
    Ns *= R;
  }
}

}  // namespace psatd
