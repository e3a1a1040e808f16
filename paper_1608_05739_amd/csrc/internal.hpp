// Device-side descriptors shared by the host planner and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace psatd {

constexpr int kMaxStages = 16;
constexpr int kMaxComp = 11;  // Ex Ey Ez Bx By Bz Jx Jy Jz rho_old rho_new

// Component slots in the workspace and in FieldPtrs.
enum Comp : int {
  kEx = 0, kEy, kEz, kBx, kBy, kBz, kJx, kJy, kJz, kRhoOld, kRhoNew
};

// Update forms: the PSATD step in vacuum, with sources in the rho form or in
// the J form, and the PSTD leapfrog contrast solver (vacuum or J).
enum SourceForm : int { kVacuum = 0, kRho = 1, kJForm = 2, kPstdVacuum = 3, kPstdJ = 4 };
constexpr bool src_is_pstd(int s) { return s == kPstdVacuum || s == kPstdJ; }
constexpr bool src_has_j(int s) { return s == kRho || s == kJForm || s == kPstdJ; }

// A complex FFT of length n factorized into radices (applied in order,
// Stockham autosort).  tw[m] = exp(-2 pi i m / n) in FP64, m in [0, n).
struct FFTPlanDev {
  int n;
  int nstages;
  int radix[kMaxStages];
  const double2* tw;
};

// A patch of a guard-cell domain decomposition (map.on != 0): the x passes
// read its cells straight from the periodic global grid, local cell
// (x, y, z) at global ((ox + x) mod gnx, (oy + y) mod gny, (oz + z) mod gnz),
// and write back only its interior [ix0, ix1) x [iy0, iy1) x [iz0, iz1)
// (local coordinates) -- the guard exchange and the gather of the
// decomposition, folded into the passes.  ox and ix0, ix1 are even, so the
// complex pairs (x[2j], x[2j + 1]) of a row never straddle the wrap.
struct GlobalMap {
  int on;
  int gnx, gny, gnz;
  int ox, oy, oz;
  int ix0, ix1, iy0, iy1, iz0, iz1;
};

// One periodic patch.  Real arrays are [nz][ny][nx] (ny = 1 in 2D).  The
// workspace holds, per patch, one block of comp_stride complex elements per
// input component; after the x pass the x axis is halved to mx = nx/2 complex
// columns, column 0 carrying the DC and Nyquist planes packed as re + i*im.
//   2D spectra  [kx][z]           (lines along z contiguous)
//   3D spectra  [z][kx][y] after the x pass (block off_spec),
//               [kx][y][z] after the y pass (block off_z).
struct PatchDev {
  int ndim;
  int nx, ny, nz, mx;
  int pad0;
  double dt;
  double inv_n;           // 1 / (nx ny nz), folded into the update
  double dkz;             // 2 pi / (nz dz) when the k tables hold the exact wavenumbers
                          // (kz of index m is m' dkz, m' = m - nz above nz/2, Nyquist 0);
                          // 0 when they hold an order-p k_p
  long long off_real;     // element offset in the caller's component buffers
  long long off_spec;     // complex-element offset of this patch's first component
  long long off_z;        // block the z passes work on: off_spec in 2D; in 3D a second
                          // block, so that the y passes, which change the layout, read
                          // one block and write the other (never lines another
                          // workgroup of the same pass has still to read)
  long long comp_stride;  // complex elements per component block (mx ny nz)
  const double* kx;       // [mx]  k_x of packed column j (column 0: k_x = 0)
  const double* ky;       // [ny]
  const double* kz;       // [nz]
  const double* kz_b;     // [nz] nz = 4096 only: kz_b[64 k2 + j + 512 q] = kz[8 j + k2 + 512 q],
                          // the order in which the 4096-point z pass updates its modes
  const double2* post;    // [mx]  exp(-2 pi i j / nx), r2c post-twiddles
  FFTPlanDev fx;          // length mx
  FFTPlanDev fy;          // length ny (3D)
  FFTPlanDev fz;          // length nz
  GlobalMap map;          // guard-cell decomposition: where the patch sits in a global grid
};

// A unit of work: `count` consecutive lines starting at `first` of component
// `comp` of patch `patch` (comp = -1 where a kernel handles all components).
struct WorkItem {
  int patch;
  int first;
  int count;
  int comp;
};

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on
// XCD b mod 8, and about 256 run at once, one per CU).  Within each run of 256
// workgroups this gives XCD x the contiguous items [32 x, 32 x + 32), so that
// neighbouring tiles, which share 128-byte lines of the [kx][8 z1 + k2]
// spectra (or, in the generic line passes, the 64-byte halves of one line of a
// tile's strided side), meet in the same L2.  A bijection on [0, n); the tail
// past the last full run of 256 keeps its order.
__device__ __forceinline__ int xcd_local_order(int b, int n) {
  const int base = b & ~255;
  if (base + 256 > n) return b;
  const int r = b & 255;
  return base + (r & 7) * 32 + (r >> 3);
}

// Caller field pointers (real arrays), indexed by Comp.  When `table` is
// set, the kernels read the pointers from that device copy instead of from
// f: a step captured once into a graph then serves any fields, the push
// writing the current pointers into the table first (see field_ptr).
struct FieldPtrs {
  void* f[kMaxComp];
  const FieldPtrs* table;
};

// Pointer of component c as a kernel sees it.
__device__ __forceinline__ void* field_ptr(const FieldPtrs& fields, int c) {
  return fields.table ? fields.table->f[c] : fields.f[c];
}

struct Physics {
  double c;
  double eps0;
};

}  // namespace psatd
