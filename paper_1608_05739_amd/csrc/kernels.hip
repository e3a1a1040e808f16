// PSATD kernels for gfx950.
//
// Data path of one step (2D; 3D adds the y passes):
//   x pass   real rows -> r2c FFT along x (half-length complex FFT + post
//            twiddle) -> spectra with the lines of the next axis contiguous
//   z pass   fused: forward FFT of every input along z, per-mode analytic
//            update, inverse FFT of E' and B' along z, all in one launch
//   x pass   inverse: pre-twiddle + inverse complex FFT -> real rows of E, B
// Storage is FP32 or FP64 (template S); FFT and update arithmetic is FP64.
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "kernels.hpp"
#include "groups.hpp"
#include "update.hpp"

namespace psatd {

template <typename S>
struct Vec2;
template <>
struct Vec2<float> {
  using type = float2;
};
template <>
struct Vec2<double> {
  using type = double2;
};

__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
template <typename V>
__device__ __forceinline__ V from_d2(double2 v);
template <>
__device__ __forceinline__ float2 from_d2<float2>(double2 v) {
  return make_float2(static_cast<float>(v.x), static_cast<float>(v.y));
}
template <>
__device__ __forceinline__ double2 from_d2<double2>(double2 v) {
  return v;
}

// ------------------------------------------------------------------ addressing
// Strided ("tile") side of a line pass: element n of line l sits at
// (l % A) + (l / A) * B + n * C (complex elements), so R consecutive lines are
// R consecutive addresses whenever they share l / A.
struct TileMap {
  long long A, B, C;
};

__device__ __forceinline__ TileMap tile_map(int kind, const PatchDev* P) {
  TileMap t;
  if (kind == kXFwd || kind == kXInv) {
    if (P->ndim == 2) {  // lines l = z ; spectra [kx][z]
      t.A = P->nz; t.B = 0; t.C = P->nz;
    } else {             // lines l = z*ny + y ; spectra [z][kx][y]
      t.A = P->ny; t.B = (long long)P->mx * P->ny; t.C = P->ny;
    }
  } else {               // y passes: lines l = kx*nz + z ; spectra [kx][y][z]
    t.A = P->nz; t.B = (long long)P->ny * P->nz; t.C = P->nz;
  }
  return t;
}

// Element n of line l in the tile layout: (l mod A) + (l / A) B + n C.
__device__ __forceinline__ long long tile_offset(const TileMap& t, int l, int n) {
  int q, r;
  udivmod(l, static_cast<int>(t.A), q, r);
  return r + q * t.B + n * t.C;
}

// Start of contiguous line l for the y passes ([z][kx][y]: l = kx*nz + z).
__device__ __forceinline__ long long yline_start(const PatchDev* P, int l) {
  int kx, z;
  udivmod(l, P->nz, kx, z);
  return ((long long)z * P->mx + kx) * P->ny;
}

// ------------------------------------------------------------------ r2c / c2r
// Runs op(row, k, W^k) for every pair (k, M - k), k = 0..M/2, of each of the
// nl lines (row: the line's first logical LDS element).  A thread takes its
// pairs kPairGroup at a time and requests their post-twiddles before their
// LDS work, so the loads are in flight together; distinct pairs touch
// distinct elements.
constexpr int kPairGroup = 4;

template <typename Op>
__device__ __forceinline__ void for_each_pair(int nl, int LS, int M, const double2* __restrict__ post,
                                              Op&& op) {
  Walk2 w(M / 2 + 1);
  while (w.hi < nl) {
    int row[kPairGroup], kk[kPairGroup];
    double2 wk[kPairGroup];
#pragma unroll
    for (int g = 0; g < kPairGroup; ++g) {
      row[g] = -1;
      if (w.hi < nl) {
        row[g] = w.hi * LS;
        kk[g] = w.lo;
        wk[g] = gload(post, w.lo);
      }
      w.next();
    }
#pragma unroll
    for (int g = 0; g < kPairGroup; ++g)
      if (row[g] >= 0) op(row[g], kk[g], wk[g]);
  }
}

// After the forward complex FFT of z[m] = x[2m] + i x[2m+1] (length M):
//   F[k] = E[k] + W^k O[k],  E = (Z[k] + conj Z[M-k])/2,  O = -i (Z[k] - conj Z[M-k])/2,
//   F[M-k] = conj(E[k] - W^k O[k]),  W = exp(-2 pi i / (2M)).
// Column 0 is packed as F[0] + i F[M] (both real).
__device__ __forceinline__ void r2c_post(double2* lds, int nl, int LS, int M, const double2* __restrict__ post) {
  for_each_pair(nl, LS, M, post, [&](int row, int k, double2 wk) __attribute__((always_inline)) {
    if (k == 0) {
      const double2 z = lds[lpad(row)];
      lds[lpad(row)] = make_double2(z.x + z.y, z.x - z.y);
      return;
    }
    const int km = M - k;
    const double2 a = lds[lpad(row + k)];
    const double2 b = lds[lpad(row + km)];
    const double2 e = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    const double2 d = make_double2(a.x - b.x, a.y + b.y);  // a - conj(b)
    const double2 o = make_double2(0.5 * d.y, -0.5 * d.x);  // -i d / 2
    const double2 wo = cmul(wk, o);
    lds[lpad(row + k)] = cadd(e, wo);
    if (km != k) lds[lpad(row + km)] = cconj(csub(e, wo));
  });
  __syncthreads();
}

// Inverse of r2c_post up to a factor 2:  Z'[k] = p + i conj(W^k) m,
// Z'[M-k] = conj(p) + i W^k conj(m) with p = F[k] + conj F[M-k], m = F[k] - conj F[M-k];
// column 0: Z'[0] = (F0 + FM) + i (F0 - FM).
__device__ __forceinline__ void c2r_pre(double2* lds, int nl, int LS, int M, const double2* __restrict__ post) {
  for_each_pair(nl, LS, M, post, [&](int row, int k, double2 wk) __attribute__((always_inline)) {
    if (k == 0) {
      const double2 x = lds[lpad(row)];
      lds[lpad(row)] = make_double2(x.x + x.y, x.x - x.y);
      return;
    }
    const int km = M - k;
    const double2 a = lds[lpad(row + k)];
    const double2 b = lds[lpad(row + km)];
    const double2 p = make_double2(a.x + b.x, a.y - b.y);
    const double2 m = make_double2(a.x - b.x, a.y + b.y);
    const double2 t1 = cmul(cconj(wk), m);
    const double2 t2 = cmul(wk, cconj(m));
    lds[lpad(row + k)] = make_double2(p.x - t1.y, p.y + t1.x);
    if (km != k) lds[lpad(row + km)] = make_double2(p.x - t2.y, -p.y + t2.x);
  });
  __syncthreads();
}

// ------------------------------------------------------------------ line pass
// The line passes at PPT = 4 points per thread run radix-4 stages (then one
// radix-2 and the radix-3 stages), derived from the line length in the same
// order as the planner's radix_plan(L, 4); at PPT = 8 they run the plan's
// stored radices (at most 8).
template <int SIGN>
__device__ __forceinline__ void fft_lds_r4(double2* lds, int nl, int LS, const FFTPlanDev* __restrict__ f) {
  const int L = f->n;
  int n = L, b = 0;
  while (n % 3 == 0) {
    n /= 3;
    ++b;
  }
  int a = __builtin_ctz(n);
  int Ns = 1;
  for (; a >= 2; a -= 2, Ns *= 4) lds_stage<4, SIGN, 4>(lds, L, nl, LS, Ns, f->tw);
  if (a == 1) {
    lds_stage<2, SIGN, 4>(lds, L, nl, LS, Ns, f->tw);
    Ns *= 2;
  }
  for (; b > 0; --b, Ns *= 3) lds_stage<3, SIGN, 4>(lds, L, nl, LS, Ns, f->tw);
}

// Pair j of local row r of a mapped patch (GlobalMap) in the global grid,
// in complex-pair units; `interior` tells whether the cell belongs to the
// patch's interior.
__device__ __forceinline__ long long mapped_pair(const PatchDev* P, int r, int j, bool* interior) {
  const GlobalMap& m = P->map;
  int lz, ly;
  udivmod(r, P->ny, lz, ly);
  const int gz = (m.oz + lz) % m.gnz;
  const int gy = (m.oy + ly) % m.gny;
  const int gx2 = (m.ox / 2 + j) % (m.gnx / 2);
  if (interior)
    *interior = lz >= m.iz0 && lz < m.iz1 && ly >= m.iy0 && ly < m.iy1 && 2 * j >= m.ix0 &&
                2 * j < m.ix1;
  return (static_cast<long long>(gz) * m.gny + gy) * (m.gnx / 2) + gx2;
}

template <typename S, int KIND, int PPT>
__global__ void __launch_bounds__(kLineBlockMax)
line_pass_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
                 int nitems, FieldPtrs fields, S* __restrict__ ws) {
  using V = typename Vec2<S>::type;
  extern __shared__ double2 lds[];
  constexpr int SIGN = (KIND == kXFwd || KIND == kYFwd || KIND == kZFwd) ? -1 : 1;
  const int T = blockDim.x;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[xcd_local_order(it, nitems)];
    const PatchDev* P = patches + wi.patch;
    const FFTPlanDev* F = (KIND == kXFwd || KIND == kXInv)   ? &P->fx
                          : (KIND == kYFwd || KIND == kYInv) ? &P->fy
                                                             : &P->fz;
    const int L = F->n;
    const int nl = wi.count;
    const int l0 = wi.first;
    const int LS = L;
    const int total = nl * L;
    // x passes use block off_spec, z passes block off_z; the y passes read one
    // and write the other (forward: off_spec -> off_z; inverse: off_z -> off_spec)
    V* const blk_x = reinterpret_cast<V*>(ws) + P->off_spec + (long long)wi.comp * P->comp_stride;
    V* const blk_z = reinterpret_cast<V*>(ws) + P->off_z + (long long)wi.comp * P->comp_stride;
    V* spec = (KIND == kXFwd || KIND == kXInv || KIND == kYFwd) ? blk_x : blk_z;  // loads
    V* spec_out = (KIND == kXFwd || KIND == kXInv || KIND == kYInv) ? blk_x : blk_z;  // stores

    // ---------------- load
    // Every element a thread owns (at most PPT) is requested before the
    // first one is written to LDS, so a thread's loads are in flight together.
    V r[PPT];
    if constexpr (KIND == kXInv || KIND == kYInv) {
      // strided side: element n of tile line r goes to LDS element r LS + n
      const TileMap tm = tile_map(KIND, P);
      int dst[PPT];
      Walk2 w(nl);
#pragma unroll
      for (int t = 0; t < PPT; ++t) {
        dst[t] = -1;
        if (w.hi < L) {
          r[t] = spec[tile_offset(tm, l0 + w.lo, w.hi)];
          dst[t] = w.lo * LS + w.hi;
        }
        w.next();
      }
#pragma unroll
      for (int t = 0; t < PPT; ++t)
        if (dst[t] >= 0) lds[lpad(dst[t])] = to_d2(r[t]);
    } else {
      // lines of the tile in LDS order: element idx = (line, n) sits at idx
      if constexpr (KIND == kYFwd) {
        Walk2 w(L);
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
          if (w.hi < nl) r[t] = spec[yline_start(P, l0 + w.hi) + w.lo];
          w.next();
        }
      } else if (KIND == kXFwd && P->map.on) {
        // a patch of a decomposition: its rows straight from the global grid
        const V* src = reinterpret_cast<const V*>(field_ptr(fields, wi.comp));
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
          const int idx = threadIdx.x + t * T;
          if (idx < total) {
            const int line = idx / L;
            r[t] = src[mapped_pair(P, l0 + line, idx - line * L, nullptr)];
          }
        }
      } else {
        // x rows (real pairs) or z lines: the tile is contiguous
        const V* src = KIND == kXFwd
                           ? reinterpret_cast<const V*>(static_cast<const S*>(field_ptr(fields, wi.comp)) +
                                                        P->off_real)
                           : spec;
        src += (long long)l0 * L;
#pragma unroll
        for (int t = 0; t < PPT; ++t) {
          const int idx = threadIdx.x + t * T;
          if (idx < total) r[t] = src[idx];
        }
      }
#pragma unroll
      for (int t = 0; t < PPT; ++t) {
        const int idx = threadIdx.x + t * T;
        if (idx < total) lds[lpad(idx)] = to_d2(r[t]);
      }
    }
    __syncthreads();

    if constexpr (KIND == kXInv) c2r_pre(lds, nl, LS, L, P->post);
    if constexpr (PPT == 4) fft_lds_r4<SIGN>(lds, nl, LS, F);
    else fft_lds<SIGN, PPT>(lds, nl, LS, F);
    if constexpr (KIND == kXFwd) r2c_post(lds, nl, LS, L, P->post);

    // ---------------- store
    if constexpr (KIND == kXFwd || KIND == kYFwd) {
      const TileMap tm = tile_map(KIND, P);
      for (Walk2 w(nl); w.hi < L; w.next()) {
        const int n = w.hi, r = w.lo;
        spec_out[tile_offset(tm, l0 + r, n)] = from_d2<V>(lds[lpad(r * LS + n)]);
      }
    } else if constexpr (KIND == kXInv) {
      if (P->map.on) {
        // a patch of a decomposition: its interior straight into the global grid
        V* dst = reinterpret_cast<V*>(field_ptr(fields, wi.comp));
        for (Walk2 w(L); w.hi < nl; w.next()) {
          bool inside;
          const long long gi = mapped_pair(P, l0 + w.hi, w.lo, &inside);
          if (inside) dst[gi] = from_d2<V>(lds[lpad(w.hi * LS + w.lo)]);
        }
      } else {
        V* dst = reinterpret_cast<V*>(static_cast<S*>(field_ptr(fields, wi.comp)) + P->off_real);
        for (Walk2 w(L); w.hi < nl; w.next())
          dst[(long long)(l0 + w.hi) * L + w.lo] = from_d2<V>(lds[lpad(w.hi * LS + w.lo)]);
      }
    } else if constexpr (KIND == kYInv) {
      for (Walk2 w(L); w.hi < nl; w.next())
        spec_out[yline_start(P, l0 + w.hi) + w.lo] = from_d2<V>(lds[lpad(w.hi * LS + w.lo)]);
    } else {
      V* dst = spec_out + (long long)l0 * L;
      for (int idx = threadIdx.x; idx < total; idx += T) dst[idx] = from_d2<V>(lds[lpad(idx)]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ compile-time line passes
// The same passes as line_pass_kernel for the line lengths the workloads use,
// with the length, the tile (lines per workgroup), the block size and the
// radix schedule fixed at compile time, so that every index of the loads,
// the Stockham stages, the r2c/c2r pairs and the stores folds to shifts,
// multiplications by constants and immediate offsets.  One kernel per pass
// kind; each work item dispatches on its line length.  A tile never straddles
// the A of the tile map (the planner checks it), so one division per tile
// places its strided side.
namespace ct {

constexpr int kT = 512;  // threads per workgroup

__host__ __device__ constexpr bool supported(int L) {
  return L == 32 || L == 48 || L == 64 || L == 96 || L == 128 || L == 192 || L == 256 ||
         L == 384 || L == 512 || L == 1024;
}
// points per thread per stage and lines per tile
__host__ __device__ constexpr int ppt(int L) { return (L % 3 == 0) ? 6 : 8; }
__host__ __device__ constexpr int tile_lines(int L) { return kT * ppt(L) / L; }

// Radix schedule of radix_plan(L, 8): radix 8 while possible, then 4 or 2,
// then the radix-3 stages.
__host__ __device__ constexpr int nstages(int L) {
  int a = 0, b = 0;
  while (L % 2 == 0) { L /= 2; ++a; }
  while (L % 3 == 0) { L /= 3; ++b; }
  return a / 3 + (a % 3 != 0) + b;
}
__host__ __device__ constexpr int radix_at(int L, int i) {
  int a = 0, b = 0;
  while (L % 2 == 0) { L /= 2; ++a; }
  while (L % 3 == 0) { L /= 3; ++b; }
  const int n8 = a / 3;
  if (i < n8) return 8;
  if (a % 3 != 0) {
    if (i == n8) return 1 << (a % 3);
    return 3;
  }
  return 3;
}
__host__ __device__ constexpr int ns_at(int L, int i) {
  int n = 1;
  for (int j = 0; j < i; ++j) n *= radix_at(L, j);
  return n;
}

template <int L, int I, int SIGN>
__device__ __forceinline__ void stage(double2* lds, const double2* __restrict__ tw) {
  constexpr int NL = tile_lines(L);
  constexpr int R = radix_at(L, I);
  constexpr int Ns = ns_at(L, I);
  constexpr int nb = L / R;
  constexpr int NB = NL * nb;
  constexpr int BPT = (NB + kT - 1) / kT;
  constexpr int step = L / (Ns * R);
  static_assert(BPT * R <= 8, "points per thread");
  // the thread index through an opaque copy: each stage computes its own
  // addresses where it uses them, instead of every stage's addresses being
  // computed up front and held in registers across the whole transform
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  double2 v[BPT][R];
  double2 wt[BPT];
  int ob[BPT];
#pragma unroll
  for (int t = 0; t < BPT; ++t) {
    const int b0 = tid + t * kT;
    const int b = (NB % kT == 0 || b0 < NB) ? b0 : 0;  // idle slots read a valid butterfly
    const int line = b / nb;
    const int j = b - line * nb;
    const int k = j % Ns;
    if constexpr (Ns > 1) wt[t] = gload(tw, k * step);
    const int src = line * L + j;
#pragma unroll
    for (int q = 0; q < R; ++q) v[t][q] = lds[lpad(src + q * nb)];
    ob[t] = (NB % kT == 0 || b0 < NB) ? line * L + (j - k) * R + k : -1;
  }
  if constexpr (Ns > 1) {
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
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
    DFT<R, SIGN>::run(v[t]);
    if (ob[t] >= 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) lds[lpad(ob[t] + q * Ns)] = v[t][q];
    }
  }
  __syncthreads();
}

template <int L, int SIGN>
__device__ __forceinline__ void fft(double2* lds, const double2* __restrict__ tw) {
  static_for<0, nstages(L)>([&](auto ic) __attribute__((always_inline)) {
    stage<L, decltype(ic)::value, SIGN>(lds, tw);
  });
}

// op(row, k, W^k) for the pairs (k, L - k), k = 0..L/2, of the tile's lines
template <int L, typename Op>
__device__ __forceinline__ void for_pairs(const double2* __restrict__ post, Op&& op) {
  constexpr int NL = tile_lines(L);
  constexpr int NP = L / 2 + 1;
  constexpr int total = NL * NP;
  constexpr int rounds = (total + kT - 1) / kT;
  constexpr int G = 4;  // pairs whose twiddles are requested together
#pragma unroll
  for (int r0 = 0; r0 < rounds; r0 += G) {
    int row[G], kk[G];
    double2 wk[G];
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int idx = tid + (r0 + g) * kT;
      row[g] = -1;
      if (r0 + g < rounds && idx < total) {
        const int line = idx / NP;
        kk[g] = idx - line * NP;
        row[g] = line * L;
        wk[g] = gload(post, kk[g]);
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (row[g] >= 0) op(row[g], kk[g], wk[g]);
  }
  __syncthreads();
}

template <int L>
__device__ __forceinline__ void r2c_post(double2* lds, const double2* __restrict__ post) {
  for_pairs<L>(post, [&](int row, int k, double2 wk) __attribute__((always_inline)) {
    if (k == 0) {
      const double2 z = lds[lpad(row)];
      lds[lpad(row)] = make_double2(z.x + z.y, z.x - z.y);
      return;
    }
    const int km = L - k;
    const double2 a = lds[lpad(row + k)];
    const double2 b = lds[lpad(row + km)];
    const double2 e = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    const double2 d = make_double2(a.x - b.x, a.y + b.y);
    const double2 o = make_double2(0.5 * d.y, -0.5 * d.x);
    const double2 wo = cmul(wk, o);
    lds[lpad(row + k)] = cadd(e, wo);
    if (km != k) lds[lpad(row + km)] = cconj(csub(e, wo));
  });
}

template <int L>
__device__ __forceinline__ void c2r_pre(double2* lds, const double2* __restrict__ post) {
  for_pairs<L>(post, [&](int row, int k, double2 wk) __attribute__((always_inline)) {
    if (k == 0) {
      const double2 x = lds[lpad(row)];
      lds[lpad(row)] = make_double2(x.x + x.y, x.x - x.y);
      return;
    }
    const int km = L - k;
    const double2 a = lds[lpad(row + k)];
    const double2 b = lds[lpad(row + km)];
    const double2 p = make_double2(a.x + b.x, a.y - b.y);
    const double2 m = make_double2(a.x - b.x, a.y + b.y);
    const double2 t1 = cmul(cconj(wk), m);
    const double2 t2 = cmul(wk, cconj(m));
    lds[lpad(row + k)] = make_double2(p.x - t1.y, p.y + t1.x);
    if (km != k) lds[lpad(row + km)] = make_double2(p.x - t2.y, -p.y + t2.x);
  });
}

template <typename S, int KIND, int L>
__device__ __forceinline__ void tile(const PatchDev* P, const WorkItem& wi, const FieldPtrs& fields,
                                     S* ws, double2* lds) {
  using V = typename Vec2<S>::type;
  constexpr int SIGN = (KIND == kXFwd || KIND == kYFwd || KIND == kZFwd) ? -1 : 1;
  constexpr int NL = tile_lines(L);
  constexpr int TOTAL = NL * L;
  constexpr int PPT = (TOTAL + kT - 1) / kT;
  const int tid = threadIdx.x;
  const int nl = wi.count;
  const int l0 = wi.first;
  const FFTPlanDev* F = (KIND == kXFwd || KIND == kXInv)   ? &P->fx
                        : (KIND == kYFwd || KIND == kYInv) ? &P->fy
                                                           : &P->fz;
  V* const blk_x = reinterpret_cast<V*>(ws) + P->off_spec + (long long)wi.comp * P->comp_stride;
  V* const blk_z = reinterpret_cast<V*>(ws) + P->off_z + (long long)wi.comp * P->comp_stride;
  V* spec = (KIND == kXFwd || KIND == kXInv || KIND == kYFwd) ? blk_x : blk_z;
  V* spec_out = (KIND == kXFwd || KIND == kXInv || KIND == kYInv) ? blk_x : blk_z;
  // strided side of the tile: element n of line r at tbase + r + n C
  long long tbase = 0, C = 0;
  if constexpr (KIND == kXFwd || KIND == kXInv || KIND == kYFwd || KIND == kYInv) {
    const TileMap tm = tile_map(KIND, P);
    tbase = tile_offset(tm, l0, 0);
    C = tm.C;
  }
  // y passes: contiguous y line r of the tile starts at ybase + r ystep
  long long ybase = 0, ystep = 0;
  if constexpr (KIND == kYFwd || KIND == kYInv) {
    ybase = yline_start(P, l0);
    ystep = static_cast<long long>(P->mx) * P->ny;
  }

  // ---------------- load (all of a thread's elements in flight together)
  V r[PPT];
  if constexpr (KIND == kXInv || KIND == kYInv) {
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      const int idx = tid + t * kT;  // line fastest: idx = n NL + line
      const int line = idx % NL, n = idx / NL;
      if ((TOTAL % kT == 0 || idx < TOTAL) && line < nl) r[t] = spec[tbase + line + n * C];
    }
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      const int idx = tid + t * kT;
      const int line = idx % NL, n = idx / NL;
      if ((TOTAL % kT == 0 || idx < TOTAL) && line < nl) lds[lpad(line * L + n)] = to_d2(r[t]);
    }
  } else {
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      const int idx = tid + t * kT;  // element fastest: idx = line L + n
      const int line = idx / L, n = idx - line * L;
      if ((TOTAL % kT == 0 || idx < TOTAL) && line < nl) {
        if constexpr (KIND == kYFwd) {
          r[t] = spec[ybase + line * ystep + n];
        } else if constexpr (KIND == kXFwd) {
          const V* src = reinterpret_cast<const V*>(static_cast<const S*>(field_ptr(fields, wi.comp)) +
                                                    P->off_real);
          r[t] = src[(long long)l0 * L + idx];
        } else {
          r[t] = spec[(long long)l0 * L + idx];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      const int idx = tid + t * kT;
      if ((TOTAL % kT == 0 || idx < TOTAL) && idx / L < nl) lds[lpad(idx)] = to_d2(r[t]);
    }
  }
  __syncthreads();

  if constexpr (KIND == kXInv) c2r_pre<L>(lds, P->post);
  fft<L, SIGN>(lds, F->tw);
  if constexpr (KIND == kXFwd) r2c_post<L>(lds, P->post);

  // ---------------- store
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const int idx = tid + t * kT;
    if (!(TOTAL % kT == 0 || idx < TOTAL)) continue;
    if constexpr (KIND == kXFwd || KIND == kYFwd) {
      const int line = idx % NL, n = idx / NL;
      if (line < nl) spec_out[tbase + line + n * C] = from_d2<V>(lds[lpad(line * L + n)]);
    } else {
      const int line = idx / L, n = idx - line * L;
      if (line >= nl) continue;
      const V val = from_d2<V>(lds[lpad(idx)]);
      if constexpr (KIND == kXInv) {
        V* dst = reinterpret_cast<V*>(static_cast<S*>(field_ptr(fields, wi.comp)) + P->off_real);
        dst[(long long)l0 * L + idx] = val;
      } else if constexpr (KIND == kYInv) {
        spec_out[ybase + line * ystep + n] = val;
      } else {
        spec_out[(long long)l0 * L + idx] = val;
      }
    }
  }
  __syncthreads();
}

// One kernel per line length (a kernel holding every length behind a switch
// would take the registers of the largest); a pass launches one per length.
template <typename S, int KIND, int L>
__global__ void __launch_bounds__(kT)
ct_line_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items, int nitems,
               FieldPtrs fields, S* __restrict__ ws) {
  extern __shared__ double2 lds[];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[xcd_local_order(it, nitems)];
    tile<S, KIND, L>(patches + wi.patch, wi, fields, ws, lds);
  }
}

}  // namespace ct

bool ct_line_supported(int L) { return ct::supported(L); }
int ct_line_tile(int L) { return ct::tile_lines(L); }

template <typename S, int KIND>
static hipError_t ct_launch_len(int L, const LaunchShape& sh, hipStream_t stream, const PatchDev* p,
                                const WorkItem* it, int n, const FieldPtrs& f, S* ws) {
#define PSATD_CT_CASE(LEN)                                                                     \
  case LEN:                                                                                    \
    hipLaunchKernelGGL((ct::ct_line_kernel<S, KIND, LEN>), dim3(sh.grid), dim3(ct::kT),        \
                       sh.lds_bytes, stream, p, it, n, f, ws);                                 \
    break;
  switch (L) {
    PSATD_CT_CASE(32) PSATD_CT_CASE(48) PSATD_CT_CASE(64) PSATD_CT_CASE(96) PSATD_CT_CASE(128)
    PSATD_CT_CASE(192) PSATD_CT_CASE(256) PSATD_CT_CASE(384) PSATD_CT_CASE(512) PSATD_CT_CASE(1024)
    default: return hipErrorInvalidValue;
  }
#undef PSATD_CT_CASE
  return hipGetLastError();
}

template <typename S>
static hipError_t ct_dispatch(int kind, int L, const LaunchShape& sh, hipStream_t stream,
                              const PatchDev* p, const WorkItem* it, int n, const FieldPtrs& f,
                              S* ws) {
  switch (kind) {
    case kXFwd: return ct_launch_len<S, kXFwd>(L, sh, stream, p, it, n, f, ws);
    case kXInv: return ct_launch_len<S, kXInv>(L, sh, stream, p, it, n, f, ws);
    case kYFwd: return ct_launch_len<S, kYFwd>(L, sh, stream, p, it, n, f, ws);
    case kYInv: return ct_launch_len<S, kYInv>(L, sh, stream, p, it, n, f, ws);
    case kZFwd: return ct_launch_len<S, kZFwd>(L, sh, stream, p, it, n, f, ws);
    default: return ct_launch_len<S, kZInv>(L, sh, stream, p, it, n, f, ws);
  }
}

hipError_t launch_ct_line(int kind, int precision, int L, const LaunchShape& sh, hipStream_t stream,
                          const PatchDev* patches, const WorkItem* items, int nitems,
                          const FieldPtrs& fields, void* ws) {
  if (precision == 0)
    return ct_dispatch<float>(kind, L, sh, stream, patches, items, nitems, fields, static_cast<float*>(ws));
  return ct_dispatch<double>(kind, L, sh, stream, patches, items, nitems, fields, static_cast<double*>(ws));
}

template <typename S, int KIND>
static void set_ct_attrs_kind(hipError_t& e) {
  const int lim = 160 * 1024;
  auto set = [&](const void* fn) {
    hipError_t r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (r != hipSuccess) e = r;
  };
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 32>));
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 48>));
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 64>));
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 96>));
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 128>));
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 192>));
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 256>));
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 384>));
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 512>));
  set(reinterpret_cast<const void*>(&ct::ct_line_kernel<S, KIND, 1024>));
}

template <typename S>
static hipError_t set_ct_attrs() {
  hipError_t e = hipSuccess;
  set_ct_attrs_kind<S, kXFwd>(e);
  set_ct_attrs_kind<S, kXInv>(e);
  set_ct_attrs_kind<S, kYFwd>(e);
  set_ct_attrs_kind<S, kYInv>(e);
  set_ct_attrs_kind<S, kZFwd>(e);
  set_ct_attrs_kind<S, kZInv>(e);
  return e;
}

// ------------------------------------------------------------------ fused z pass
// (component groups: groups.hpp)
template <typename S, int G, int SRC, int MPT>
__device__ __forceinline__ void fused_group(const PatchDev* P, const WorkItem& wi, S* ws,
                                            const Physics& ph, double2* lds) {
  using V = typename Vec2<S>::type;
  using Gr = Group<G, SRC>;
  constexpr int NIN = Gr::nin;
  const int T = blockDim.x;
  const int nz = P->nz;
  const int W = wi.count;
  const int nmodes = W * nz;
  V* base = reinterpret_cast<V*>(ws) + P->off_z + (long long)wi.first * nz;
  const long long cs = P->comp_stride;
  const FFTPlanDev* F = &P->fz;

  // SL slots are transformed together: their tiles sit one after another in
  // LDS and one FFT covers all of them, so that the stages have work for
  // every thread (SL W nz <= T kMaxPtsFused) and share their barriers.
  constexpr int SL = fused_slots(MPT);
  V reg[NIN][MPT];
  // Forward transforms of the group's inputs.  The round loop is a runtime
  // loop so that the FFT code is instantiated once; the register slot is then
  // selected by a compile-time compare chain (no dynamic register indexing).
#pragma nounroll
  for (int s0 = 0; s0 < NIN; s0 += SL) {
    const int ns = NIN - s0 < SL ? NIN - s0 : SL;
#pragma unroll
    for (int j = 0; j < SL; ++j) {
      if (j >= ns) break;
      const V* src = base + Gr::in[s0 + j] * cs;
      // a thread's loads go out in groups of PF, each group in flight
      // together before its LDS writes (small: reg holds the other slots)
      constexpr int PF = MPT < 4 ? MPT : 4;
#pragma unroll
      for (int m0 = 0; m0 < MPT; m0 += PF) {
        V pf[PF];
#pragma unroll
        for (int m = 0; m < PF; ++m) {
          const int idx = threadIdx.x + (m0 + m) * T;
          if (idx < nmodes) pf[m] = src[idx];
        }
#pragma unroll
        for (int m = 0; m < PF; ++m) {
          const int idx = threadIdx.x + (m0 + m) * T;
          if (idx < nmodes) lds[lpad(j * nmodes + idx)] = to_d2(pf[m]);
        }
      }
    }
    __syncthreads();
    fft_lds<-1, kMaxPtsFused>(lds, ns * W, nz, F);
    static_for<0, NIN>([&](auto sc) __attribute__((always_inline)) {
      constexpr int sl = decltype(sc)::value;
      const int j = sl - s0;
      if (j >= 0 && j < ns) {
#pragma unroll
        for (int m = 0; m < MPT; ++m) {
          const int idx = threadIdx.x + m * T;
          if (idx < nmodes) reg[sl][m] = from_d2<V>(lds[lpad(j * nmodes + idx)]);
        }
      }
    });
    __syncthreads();
  }

  // per-mode update
  const double dt = P->dt;
#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    const int idx = threadIdx.x + m * T;
    if (idx < nmodes) {
      int lrel, iz;
      udivmod(idx, nz, lrel, iz);
      const int line = wi.first + lrel;
      double kx, ky;
      if (P->ndim == 2) {
        kx = gload(P->kx, line);
        ky = 0.0;
      } else {
        int ix, iy;
        udivmod(line, P->ny, ix, iy);
        kx = gload(P->kx, ix);
        ky = gload(P->ky, iy);
      }
      const double kz = gload(P->kz, iz);
      double2 E[3] = {}, B[3] = {}, J[3] = {};
      double2 ro = make_double2(0.0, 0.0), rn = make_double2(0.0, 0.0);
      static_for<0, NIN>([&](auto sc) __attribute__((always_inline)) {
        constexpr int slot = decltype(sc)::value;
        constexpr int comp = Gr::in[slot];
        const double2 v = to_d2(reg[slot][m]);
        if constexpr (comp < 3) E[comp] = v;
        else if constexpr (comp < 6) B[comp - 3] = v;
        else if constexpr (comp < 9) J[comp - 6] = v;
        else if constexpr (comp == kRhoOld) ro = v;
        else rn = v;
      });
      double2 Eo[3], Bo[3];
      if constexpr (src_is_pstd(SRC)) {
        pstd_update_mode<SRC>(kx, ky, kz, dt, ph.c, ph.eps0, P->inv_n, E, B, J, Eo, Bo);
      } else {
        const double K = sqrt(kx * kx + ky * ky + kz * kz);
        const Coef q = psatd_coef(K, dt, ph.c, ph.eps0, P->inv_n);
        update_mode<SRC>(kx, ky, kz, q, ph.c, ph.eps0, dt, E, B, J, ro, rn, Eo, Bo);
      }
      static_for<0, Gr::nout>([&](auto oc) __attribute__((always_inline)) {
        constexpr int o = decltype(oc)::value;
        constexpr int comp = Gr::in[Gr::out_slot[o]];
        if constexpr (comp < 3) reg[Gr::out_slot[o]][m] = from_d2<V>(Eo[comp]);
        else reg[Gr::out_slot[o]][m] = from_d2<V>(Bo[comp - 3]);
      });
    }
    // keep the modes' updates from being interleaved (register pressure)
    __builtin_amdgcn_sched_barrier(0);
  }

  // Inverse transforms of the outputs, SL at a time, written back over the
  // input slots.
#pragma nounroll
  for (int o0 = 0; o0 < Gr::nout; o0 += SL) {
    const int no = Gr::nout - o0 < SL ? Gr::nout - o0 : SL;
    static_for<0, NIN>([&](auto sc) __attribute__((always_inline)) {
      constexpr int sl = decltype(sc)::value;
#pragma unroll
      for (int j = 0; j < SL; ++j) {
        if (j < no && Gr::out_slot[o0 + j] == sl) {
#pragma unroll
          for (int m = 0; m < MPT; ++m) {
            const int idx = threadIdx.x + m * T;
            if (idx < nmodes) lds[lpad(j * nmodes + idx)] = to_d2(reg[sl][m]);
          }
        }
      }
    });
    __syncthreads();
    fft_lds<1, kMaxPtsFused>(lds, no * W, nz, F);
    for (int j = 0; j < no; ++j) {
      V* dst = base + Gr::in[Gr::out_slot[o0 + j]] * cs;
      for (int idx = threadIdx.x; idx < nmodes; idx += T)
        dst[idx] = from_d2<V>(lds[lpad(j * nmodes + idx)]);
    }
    __syncthreads();
  }
}

template <typename S, int DIM, int SRC, int MPT>
__global__ void __launch_bounds__(kFusedBlock)
fused_z_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
               int nitems, S* __restrict__ ws, Physics ph) {
  extern __shared__ double2 lds[];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const PatchDev* P = patches + wi.patch;
    if constexpr (DIM == 2) {
      fused_group<S, 0, SRC, MPT>(P, wi, ws, ph, lds);
      fused_group<S, 1, SRC, MPT>(P, wi, ws, ph, lds);
    } else {
      fused_group<S, 2, SRC, MPT>(P, wi, ws, ph, lds);
    }
  }
}

// ------------------------------------------------------------------ plain update
template <typename S, int SRC>
__global__ void __launch_bounds__(256)
update_kernel(const PatchDev* __restrict__ patches, const WorkItem* __restrict__ items,
              int nitems, S* __restrict__ ws, Physics ph) {
  using V = typename Vec2<S>::type;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const WorkItem wi = items[it];
    const PatchDev* P = patches + wi.patch;
    V* base = reinterpret_cast<V*>(ws) + P->off_z;
    const long long cs = P->comp_stride;
    const int nz = P->nz;
    const double dt = P->dt;
    for (int j = threadIdx.x; j < wi.count; j += blockDim.x) {
      const long long idx = (long long)wi.first + j;
      const long long line = idx / nz;
      const int iz = static_cast<int>(idx - line * nz);
      double kx, ky;
      if (P->ndim == 2) {
        kx = gload(P->kx, static_cast<int>(line));
        ky = 0.0;
      } else {
        kx = gload(P->kx, static_cast<int>(line / P->ny));
        ky = gload(P->ky, static_cast<int>(line % P->ny));
      }
      const double kz = gload(P->kz, iz);
      double2 E[3], B[3], J[3] = {};
      double2 ro = make_double2(0.0, 0.0), rn = make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        E[i] = to_d2(base[(kEx + i) * cs + idx]);
        B[i] = to_d2(base[(kBx + i) * cs + idx]);
      }
      if constexpr (src_has_j(SRC)) {
#pragma unroll
        for (int i = 0; i < 3; ++i) J[i] = to_d2(base[(kJx + i) * cs + idx]);
      }
      if constexpr (SRC == kRho) {
        ro = to_d2(base[kRhoOld * cs + idx]);
        rn = to_d2(base[kRhoNew * cs + idx]);
      }
      double2 Eo[3], Bo[3];
      if constexpr (src_is_pstd(SRC)) {
        pstd_update_mode<SRC>(kx, ky, kz, dt, ph.c, ph.eps0, P->inv_n, E, B, J, Eo, Bo);
      } else {
        const double K = sqrt(kx * kx + ky * ky + kz * kz);
        const Coef q = psatd_coef(K, dt, ph.c, ph.eps0, P->inv_n);
        update_mode<SRC>(kx, ky, kz, q, ph.c, ph.eps0, dt, E, B, J, ro, rn, Eo, Bo);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        base[(kEx + i) * cs + idx] = from_d2<V>(Eo[i]);
        base[(kBx + i) * cs + idx] = from_d2<V>(Bo[i]);
      }
    }
  }
}

// ------------------------------------------------------------------ tables (FP64)
__global__ void twiddle_kernel(double2* tw, int n, int count) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < count) {
    double s, c;
    sincospi(2.0 * static_cast<double>(m) / static_cast<double>(n), &s, &c);
    tw[m] = make_double2(c, -s);
  }
}

// k_j = 2 pi m_j / (n d) in fftfreq order, the Nyquist index (even n) -> 0.
// packed_x: entries j = 0..count-1 of the halved x axis, entry 0 standing for
// both the DC and the Nyquist columns (k = 0 for both).  With stencil weights
// w_l (nf = p/2 of them) the order-p wavevector replaces k:
//   staggered  k_p = sum_l w_l (2/d) sin((2l - 1) k d / 2)
//   centered   k_p = sum_l w_l (2/d) sin(l k d)
__global__ void ktable_kernel(double* k, int n, double d, int count, int packed_x,
                              const double* __restrict__ fornberg, int nf, int centered) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  int m = (j < (n + 1) / 2) ? j : j - n;
  const bool nyquist = (n % 2 == 0) && (j == n / 2);
  if (packed_x) m = j;
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  double kv = kTwoPi * static_cast<double>(m) / (static_cast<double>(n) * d);
  if (nf > 0) {
    double acc = 0.0;
    for (int l = 1; l <= nf; ++l) {
      const double arg = centered ? l * kv * d : (2 * l - 1) * kv * d * 0.5;
      acc += fornberg[l - 1] * (2.0 / d) * sin(arg);
    }
    kv = acc;
  }
  if (nyquist || (packed_x && j == 0)) kv = 0.0;
  k[j] = kv;
}

// ------------------------------------------------------------------ field table
// Writes the caller's field pointers into the plan's device table (one
// thread; the push enqueues it ahead of a graph whose kernels read the table).
__global__ void store_fields_kernel(FieldPtrs f, FieldPtrs* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) dst->f[c] = f.f[c];
    dst->table = nullptr;
  }
}

hipError_t launch_store_fields(const FieldPtrs& f, FieldPtrs* dst, hipStream_t stream) {
  hipLaunchKernelGGL(store_fields_kernel, dim3(1), dim3(64), 0, stream, f, dst);
  return hipGetLastError();
}

// ------------------------------------------------------------------ launchers
template <typename S, int PPT>
static hipError_t line_dispatch(int kind, const LaunchShape& sh, hipStream_t stream,
                                const PatchDev* p, const WorkItem* it, int n, const FieldPtrs& f,
                                S* ws) {
  switch (kind) {
    case kXFwd:
      hipLaunchKernelGGL((line_pass_kernel<S, kXFwd, PPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, f, ws);
      break;
    case kXInv:
      hipLaunchKernelGGL((line_pass_kernel<S, kXInv, PPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, f, ws);
      break;
    case kYFwd:
      hipLaunchKernelGGL((line_pass_kernel<S, kYFwd, PPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, f, ws);
      break;
    case kYInv:
      hipLaunchKernelGGL((line_pass_kernel<S, kYInv, PPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, f, ws);
      break;
    case kZFwd:
      hipLaunchKernelGGL((line_pass_kernel<S, kZFwd, PPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, f, ws);
      break;
    default:
      hipLaunchKernelGGL((line_pass_kernel<S, kZInv, PPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, f, ws);
      break;
  }
  return hipGetLastError();
}

bool line_ppt_supported(int ppt) { return ppt == 4 || ppt == kMaxPts; }

hipError_t launch_line_pass(int kind, int precision, int ppt, const LaunchShape& sh,
                            hipStream_t stream, const PatchDev* patches, const WorkItem* items,
                            int nitems, const FieldPtrs& fields, void* ws) {
  if (!line_ppt_supported(ppt)) return hipErrorInvalidValue;
  if (precision == 0) {
    float* w = static_cast<float*>(ws);
    return ppt == 4 ? line_dispatch<float, 4>(kind, sh, stream, patches, items, nitems, fields, w)
                    : line_dispatch<float, kMaxPts>(kind, sh, stream, patches, items, nitems, fields, w);
  }
  double* w = static_cast<double*>(ws);
  return ppt == 4 ? line_dispatch<double, 4>(kind, sh, stream, patches, items, nitems, fields, w)
                  : line_dispatch<double, kMaxPts>(kind, sh, stream, patches, items, nitems, fields, w);
}

// Modes per thread compiled for each (precision, ndim): the transformed inputs
// of a group stay in registers, so MPT * inputs * sizeof(complex) is bounded.
bool fused_supported(int precision, int ndim, int mpt) {
  if (precision == 0)
    return (ndim == 2 && (mpt == 2 || mpt == 4 || mpt == 8)) || (ndim == 3 && (mpt == 2 || mpt == 4));
  return (ndim == 2 && (mpt == 2 || mpt == 4)) || (ndim == 3 && mpt == 2);
}

template <typename S, int DIM, int MPT>
static hipError_t fused_dispatch(int src, const LaunchShape& sh, hipStream_t stream,
                                 const PatchDev* p, const WorkItem* it, int n, S* ws, Physics ph) {
  switch (src) {
    case kVacuum:
      hipLaunchKernelGGL((fused_z_kernel<S, DIM, kVacuum, MPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, ws, ph);
      break;
    case kRho:
      hipLaunchKernelGGL((fused_z_kernel<S, DIM, kRho, MPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, ws, ph);
      break;
    case kPstdVacuum:
      hipLaunchKernelGGL((fused_z_kernel<S, DIM, kPstdVacuum, MPT>), dim3(sh.grid),
                         dim3(sh.block), sh.lds_bytes, stream, p, it, n, ws, ph);
      break;
    case kPstdJ:
      hipLaunchKernelGGL((fused_z_kernel<S, DIM, kPstdJ, MPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, ws, ph);
      break;
    default:
      hipLaunchKernelGGL((fused_z_kernel<S, DIM, kJForm, MPT>), dim3(sh.grid), dim3(sh.block),
                         sh.lds_bytes, stream, p, it, n, ws, ph);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_fused_z(int precision, int ndim, int src, int mpt, const LaunchShape& sh,
                          hipStream_t stream, const PatchDev* patches, const WorkItem* items,
                          int nitems, void* ws, Physics ph) {
  if (!fused_supported(precision, ndim, mpt)) return hipErrorInvalidValue;
  if (precision == 0) {
    float* w = static_cast<float*>(ws);
    if (ndim == 2)
      return mpt == 2   ? fused_dispatch<float, 2, 2>(src, sh, stream, patches, items, nitems, w, ph)
             : mpt == 4 ? fused_dispatch<float, 2, 4>(src, sh, stream, patches, items, nitems, w, ph)
                        : fused_dispatch<float, 2, 8>(src, sh, stream, patches, items, nitems, w, ph);
    return mpt == 2 ? fused_dispatch<float, 3, 2>(src, sh, stream, patches, items, nitems, w, ph)
                    : fused_dispatch<float, 3, 4>(src, sh, stream, patches, items, nitems, w, ph);
  }
  if (ndim == 2)
    return mpt == 2 ? fused_dispatch<double, 2, 2>(src, sh, stream, patches, items, nitems,
                                                   static_cast<double*>(ws), ph)
                    : fused_dispatch<double, 2, 4>(src, sh, stream, patches, items, nitems,
                                                   static_cast<double*>(ws), ph);
  return fused_dispatch<double, 3, 2>(src, sh, stream, patches, items, nitems,
                                      static_cast<double*>(ws), ph);
}

template <typename S>
static hipError_t update_dispatch(int src, const LaunchShape& sh, hipStream_t stream,
                                  const PatchDev* p, const WorkItem* it, int n, S* ws, Physics ph) {
  switch (src) {
    case kVacuum:
      hipLaunchKernelGGL((update_kernel<S, kVacuum>), dim3(sh.grid), dim3(sh.block), 0, stream, p,
                         it, n, ws, ph);
      break;
    case kRho:
      hipLaunchKernelGGL((update_kernel<S, kRho>), dim3(sh.grid), dim3(sh.block), 0, stream, p, it,
                         n, ws, ph);
      break;
    case kPstdVacuum:
      hipLaunchKernelGGL((update_kernel<S, kPstdVacuum>), dim3(sh.grid), dim3(sh.block), 0, stream,
                         p, it, n, ws, ph);
      break;
    case kPstdJ:
      hipLaunchKernelGGL((update_kernel<S, kPstdJ>), dim3(sh.grid), dim3(sh.block), 0, stream, p,
                         it, n, ws, ph);
      break;
    default:
      hipLaunchKernelGGL((update_kernel<S, kJForm>), dim3(sh.grid), dim3(sh.block), 0, stream, p,
                         it, n, ws, ph);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_update(int precision, int src, const LaunchShape& sh, hipStream_t stream,
                         const PatchDev* patches, const WorkItem* items, int nitems, void* ws,
                         Physics ph) {
  if (precision == 0)
    return update_dispatch<float>(src, sh, stream, patches, items, nitems,
                                  static_cast<float*>(ws), ph);
  return update_dispatch<double>(src, sh, stream, patches, items, nitems,
                                 static_cast<double*>(ws), ph);
}

hipError_t launch_twiddles(double2* tw, int n, int count, hipStream_t stream) {
  const int b = 256;
  hipLaunchKernelGGL(twiddle_kernel, dim3((count + b - 1) / b), dim3(b), 0, stream, tw, n, count);
  return hipGetLastError();
}

hipError_t launch_ktable(double* k, int n, double d, int count, int packed_x,
                         const double* fornberg, int nfornberg, int centered,
                         hipStream_t stream) {
  const int b = 256;
  hipLaunchKernelGGL(ktable_kernel, dim3((count + b - 1) / b), dim3(b), 0, stream, k, n, d, count,
                     packed_x, fornberg, nfornberg, centered);
  return hipGetLastError();
}

template <typename S, int PPT>
static hipError_t set_attrs_for() {
  const int lim = 160 * 1024;
  hipError_t e = hipSuccess;
  auto set = [&](const void* fn) {
    hipError_t r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (r != hipSuccess) e = r;
  };
  set(reinterpret_cast<const void*>(&line_pass_kernel<S, kXFwd, PPT>));
  set(reinterpret_cast<const void*>(&line_pass_kernel<S, kXInv, PPT>));
  set(reinterpret_cast<const void*>(&line_pass_kernel<S, kYFwd, PPT>));
  set(reinterpret_cast<const void*>(&line_pass_kernel<S, kYInv, PPT>));
  set(reinterpret_cast<const void*>(&line_pass_kernel<S, kZFwd, PPT>));
  set(reinterpret_cast<const void*>(&line_pass_kernel<S, kZInv, PPT>));
  return e;
}

template <typename S, int DIM, int MPT>
static hipError_t set_fused_attrs() {
  const int lim = 160 * 1024;
  hipError_t e = hipSuccess;
  auto set = [&](const void* fn) {
    hipError_t r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if (r != hipSuccess) e = r;
  };
  set(reinterpret_cast<const void*>(&fused_z_kernel<S, DIM, kVacuum, MPT>));
  set(reinterpret_cast<const void*>(&fused_z_kernel<S, DIM, kRho, MPT>));
  set(reinterpret_cast<const void*>(&fused_z_kernel<S, DIM, kJForm, MPT>));
  set(reinterpret_cast<const void*>(&fused_z_kernel<S, DIM, kPstdVacuum, MPT>));
  set(reinterpret_cast<const void*>(&fused_z_kernel<S, DIM, kPstdJ, MPT>));
  return e;
}

hipError_t configure_kernel_attributes() {
  hipError_t e = hipSuccess;
  hipError_t r;
  if ((r = set_attrs_for<float, 4>()) != hipSuccess) e = r;
  if ((r = set_attrs_for<float, kMaxPts>()) != hipSuccess) e = r;
  if ((r = set_attrs_for<double, 4>()) != hipSuccess) e = r;
  if ((r = set_attrs_for<double, kMaxPts>()) != hipSuccess) e = r;
  if ((r = set_fused_attrs<float, 2, 2>()) != hipSuccess) e = r;
  if ((r = set_fused_attrs<float, 2, 4>()) != hipSuccess) e = r;
  if ((r = set_fused_attrs<float, 2, 8>()) != hipSuccess) e = r;
  if ((r = set_fused_attrs<float, 3, 2>()) != hipSuccess) e = r;
  if ((r = set_fused_attrs<float, 3, 4>()) != hipSuccess) e = r;
  if ((r = set_fused_attrs<double, 2, 2>()) != hipSuccess) e = r;
  if ((r = set_fused_attrs<double, 2, 4>()) != hipSuccess) e = r;
  if ((r = set_fused_attrs<double, 3, 2>()) != hipSuccess) e = r;
  if ((r = set_ct_attrs<float>()) != hipSuccess) e = r;
  if ((r = set_ct_attrs<double>()) != hipSuccess) e = r;
  return e;
}

}  // namespace psatd
