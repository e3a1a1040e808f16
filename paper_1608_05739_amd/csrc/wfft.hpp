// Wave-resident Stockham FFT for compile-time line lengths (gfx950).
//
// A wavefront owns whole lines: lane l = g S + s holds points s + S m
// (m < P) of line g, so a line spans S = L / P lanes and a wave holds
// G = 64 / S lines.  Each radix-R stage runs P / R butterflies per lane in
// registers: butterfly t is j = s + S t, it reads x[j + q L/R] -- register
// t + q P/R of the lane -- multiplies by w^(q k) with k = j mod Ns,
// w = exp(SIGN 2 pi i / (Ns R)), applies DFT<R> and produces
// y[(j - k) R + k + q Ns] (Stockham autosort; Ns = product of the radices
// before the stage).  Between stages the wave exchanges y through its own LDS
// region (padded, see kPadShift) and reads back y[s + S m]; no other
// wave touches that region, so no workgroup barrier is needed.  The last
// stage's outputs already sit in the input layout (natural order, point
// s + S m in register m), so input and output are both natural order.
//
// Radix schedules (every radix divides P):
//   P = 8:  32 = 8.4   64 = 8.8   128 = 8.4.4   256 = 8.8.4   512 = 8.8.8
//   P = 12: 48 = 4.12  96 = 4.2.12  192 = 4.4.12  384 = 4.4.2.12  768 = 4.4.4.12
//   P = 16: 1024 = 16.16.4
// The radix-12 stage of the 3 * 2^k lengths comes last, where Ns = S, so that
// k = s and every LDS address is a per-lane base plus a compile-time offset
// (checked for every length and stage, lane by lane, by a NumPy emulation of
// this index logic against numpy.fft before the first GPU run).
#pragma once

#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace psatd {
namespace wfft {

// ------------------------------------------------------------------ schedules
template <int L>
struct Sched;
template <> struct Sched<32>   { static constexpr int P = 8,  N = 2; static constexpr int R[4] = {8, 4}; };
template <> struct Sched<64>   { static constexpr int P = 8,  N = 2; static constexpr int R[4] = {8, 8}; };
template <> struct Sched<128>  { static constexpr int P = 8,  N = 3; static constexpr int R[4] = {8, 4, 4}; };
template <> struct Sched<256>  { static constexpr int P = 8,  N = 3; static constexpr int R[4] = {8, 8, 4}; };
template <> struct Sched<512>  { static constexpr int P = 8,  N = 3; static constexpr int R[4] = {8, 8, 8}; };
template <> struct Sched<48>   { static constexpr int P = 12, N = 2; static constexpr int R[4] = {4, 12}; };
template <> struct Sched<96>   { static constexpr int P = 12, N = 3; static constexpr int R[4] = {4, 2, 12}; };
template <> struct Sched<192>  { static constexpr int P = 12, N = 3; static constexpr int R[4] = {4, 4, 12}; };
template <> struct Sched<384>  { static constexpr int P = 12, N = 4; static constexpr int R[4] = {4, 4, 2, 12}; };
template <> struct Sched<768>  { static constexpr int P = 12, N = 4; static constexpr int R[4] = {4, 4, 4, 12}; };
template <> struct Sched<1024> { static constexpr int P = 16, N = 3; static constexpr int R[4] = {16, 16, 4}; };

// Is L one of the lengths above?  (host and device)
__host__ __device__ constexpr bool supported(int L) {
  return L == 32 || L == 64 || L == 128 || L == 256 || L == 512 || L == 48 || L == 96 ||
         L == 192 || L == 384 || L == 768 || L == 1024;
}
__host__ __device__ constexpr int points(int L) {
  return (L % 3 == 0) ? 12 : (L == 1024 ? 16 : 8);
}

// LDS padding: one element every 2^kPadShift (e -> e + (e >> kPadShift)).
constexpr int kPadShift = 4;
// Padded LDS elements of one line of length L.
__host__ __device__ constexpr int stride_of(int L) { return L + (L >> kPadShift); }

template <int L>
struct Line {
  static constexpr int P = Sched<L>::P;
  static constexpr int S = L / P;                // lanes per line
  static constexpr int G = 64 / S;               // lines per wave
  static constexpr int STRIDE = stride_of(L);    // padded LDS elements per line
  static constexpr int REGION = G * STRIDE;      // double2 elements per wave region
  static_assert(L % P == 0 && 64 % S == 0 && L % 8 == 0, "wave layout");
};

// Padded LDS index of logical element e.
__host__ __device__ constexpr int pa(int e) { return e + (e >> kPadShift); }

// Product of the radices before stage i.
template <int L>
__host__ __device__ constexpr int ns_before(int i) {
  int n = 1;
  for (int j = 0; j < i; ++j) n *= Sched<L>::R[j];
  return n;
}

// Stockham output index of butterfly t, output q, lane s, at stage i.
template <int L, int I>
__host__ __device__ constexpr int out_index(int s, int t, int q) {
  constexpr int R = Sched<L>::R[I];
  constexpr int Ns = ns_before<L>(I);
  const int j = s + Line<L>::S * t;
  const int k = j % Ns;
  return (j - k) * R + k + q * Ns;
}

// Wave-level ordering of LDS traffic inside one wavefront's region.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ twiddles
// Distinct twiddle bases a lane uses in stage I: butterfly t has
// k_t = (s + S t) mod Ns, which is s mod Ns for every t when Ns <= S and
// repeats with period Ns / S in t otherwise.
template <int L>
__host__ __device__ constexpr int nbases(int i) {
  const int Ns = ns_before<L>(i);
  const int bpt = Sched<L>::P / Sched<L>::R[i];
  if (Ns == 1) return 0;
  if (Ns <= Line<L>::S) return 1;
  return (Ns / Line<L>::S) < bpt ? (Ns / Line<L>::S) : bpt;
}

// Where a transform takes its twiddle bases exp(-2 pi i k / (Ns R)) from.
//
// Twiddles<L>: the lane's bases of every stage, loaded once and kept in
// registers.  They depend only on the lane's position s, so every transform
// of the length (forward, and conjugated for the inverse) uses the same ones.
// For kernels that run one transform per tile.
template <int L>
struct Twiddles {
  double2 w[4][4];

  template <int I>
  __device__ __forceinline__ double2 base(int t, int /*s*/) const {
    // a copy the optimizer cannot see through: the powers of the base are
    // formed in each transform, not kept live from one transform to the next
    double2 u = w[I][t];
    asm volatile("" : "+v"(u.x), "+v"(u.y));
    return u;
  }

  // tw[m] = exp(-2 pi i m / L) in FP64 (the plan's table for this length)
  __device__ __forceinline__ void load(const double2* __restrict__ tw, int s) {
    static_for<0, Sched<L>::N>([&](auto ic) __attribute__((always_inline)) {
      constexpr int I = decltype(ic)::value;
      constexpr int Ns = ns_before<L>(I);
      constexpr int step = L / (Ns * Sched<L>::R[I]);
#pragma unroll
      for (int t = 0; t < nbases<L>(I); ++t) {
        const int k = (Ns <= Line<L>::S) ? (s % Ns) : (s + Line<L>::S * t);
        w[I][t] = gload(tw, k * step);
      }
    });
  }
};

// TableTwiddles<L>: each transform loads its bases from the plan's table
// again, through an index the optimizer cannot see through, instead of
// keeping them (and their powers) live from one transform to the next.  For
// kernels that hold other state across many transforms.
template <int L>
struct TableTwiddles {
  const double2* tw;  // tw[m] = exp(-2 pi i m / L), FP64

  template <int I>
  __device__ __forceinline__ double2 base(int t, int s) const {
    constexpr int Ns = ns_before<L>(I);
    constexpr int step = L / (Ns * Sched<L>::R[I]);
    int k = (Ns <= Line<L>::S) ? (s % Ns) : (s + Line<L>::S * t);
    asm volatile("" : "+v"(k));
    return gload(tw, k * step);
  }
};

// ------------------------------------------------------------------ the transform
// In-place FFT (unnormalized) of the G lines a wave holds.  v[m] = point
// s + S m of the lane's line on entry and on exit.  region: this wave's LDS
// region (Line<L>::REGION elements); g, s: the lane's line and position;
// tws: the lane's twiddle bases (Twiddles<L> or TableTwiddles<L>).
template <int L, int SIGN, typename TW>
__device__ __forceinline__ void fft(double2 (&v)[Sched<L>::P], double2* region, int g_in, int s_in,
                                    const TW& tws) {
  using LN = Line<L>;
  constexpr int P = LN::P;
  constexpr int S = LN::S;
  static_for<0, Sched<L>::N>([&](auto ic) __attribute__((always_inline)) {
    constexpr int I = decltype(ic)::value;
    // the lane coordinates through opaque copies: each stage computes its own
    // addresses and twiddle indices where it uses them, instead of all of them
    // being computed once and held in registers across every transform
    int s = s_in, g = g_in;
    asm volatile("" : "+v"(s), "+v"(g));
    double2* const line = region + g * LN::STRIDE;
    constexpr int R = Sched<L>::R[I];
    constexpr int Ns = ns_before<L>(I);
    constexpr int BPT = P / R;
    constexpr bool last = I == Sched<L>::N - 1;
    // twiddle bases w_t = exp(SIGN 2 pi i k_t / (Ns R)), k_t = (s + S t) mod Ns
    double2 wb[BPT];
    if constexpr (Ns > 1) {
#pragma unroll
      for (int t = 0; t < BPT; ++t) {
        if (t >= nbases<L>(I)) {
          wb[t] = wb[t % nbases<L>(I)];
        } else {
          double2 w = tws.template base<I>(t, s);
          if constexpr (SIGN > 0) w.y = -w.y;
          wb[t] = w;
        }
      }
    }
    // lane part of this stage's output addresses (the rest is compile-time)
    const int wbase = pa(out_index<L, I>(s, 0, 0));
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      double2 a[R];
#pragma unroll
      for (int q = 0; q < R; ++q) a[q] = v[t + q * BPT];
      if constexpr (Ns > 1) {
        const double2 u = wb[t];
        double2 uq = u;
        a[1] = cmul(a[1], u);
#pragma unroll
        for (int q = 2; q < R; ++q) {
          uq = cmul(uq, u);
          a[q] = cmul(a[q], uq);
        }
      }
      DFT<R, SIGN>::run(a);
      if constexpr (last) {
#pragma unroll
        for (int q = 0; q < R; ++q) v[t + q * BPT] = a[q];
      } else {
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int off = pa(out_index<L, I>(0, t, q)) - pa(out_index<L, I>(0, 0, 0));
          line[wbase + off] = a[q];
        }
      }
    }
    if constexpr (!last) {
      wave_sync();
      const int rbase = pa(s);
#pragma unroll
      for (int m = 0; m < P; ++m) v[m] = line[rbase + pa(S * m)];
      wave_sync();
    }
  });
}

}  // namespace wfft
}  // namespace psatd
