// Host-callable launchers for the PSATD kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace psatd {

// Line passes (one FFT axis per launch).
enum LineKind : int {
  kXFwd = 0,  // real rows -> r2c along x -> spectra, tile-contiguous (2D [kx][z], 3D [z][kx][y])
  kXInv = 1,  // tile-contiguous spectra -> c2r along x -> real rows (E, B in place)
  kYFwd = 2,  // 3D: [z][kx][y] lines -> forward c2c along y -> [kx][y][z]
  kYInv = 3,  // 3D: [kx][y][z] -> inverse c2c along y -> [z][kx][y]
  kZFwd = 4,  // contiguous z lines, forward c2c in place (plain path)
  kZInv = 5,  // contiguous z lines, inverse c2c in place (plain path)
};

constexpr int kMaxPts = 8;        // points per thread per FFT stage in the line passes
constexpr int kMaxPtsFused = 8;   // ... in the fused z pass, which also holds its inputs
constexpr int kMaxRadixZ = 8;     // largest radix of the z plans (fits kMaxPtsFused)
constexpr int kLineBlockMax = 512;  // launch bound of the line-pass kernels
constexpr int kFusedBlock = 512;    // launch bound (and block size) of the fused z pass

// Slots (component tiles) the fused z pass transforms in one FFT at mpt modes
// per thread: together they give each thread kMaxPtsFused points.
constexpr int fused_slots(int mpt) { return kMaxPtsFused / mpt; }

struct LaunchShape {
  int grid;
  int block;
  size_t lds_bytes;
};

// ppt: points per thread per FFT stage, 4 (radix-4 stages) or kMaxPts (the
// plan's radices); the block must give every element of a tile a thread slot.
hipError_t launch_line_pass(int kind, int precision, int ppt, const LaunchShape& sh,
                            hipStream_t stream, const PatchDev* patches, const WorkItem* items,
                            int nitems, const FieldPtrs& fields, void* ws);
bool line_ppt_supported(int ppt);

// Compile-time line passes: the line pass kinds above for the lengths
// ct_line_supported() accepts, ct_line_tile(L) lines per work item (a work
// item never crosses a multiple of the tile map's A), kCtBlock threads; one
// launch covers the work items of one line length L.
bool ct_line_supported(int L);
int ct_line_tile(int L);
hipError_t launch_ct_line(int kind, int precision, int L, const LaunchShape& sh, hipStream_t stream,
                          const PatchDev* patches, const WorkItem* items, int nitems,
                          const FieldPtrs& fields, void* ws);
constexpr int kCtBlock = 512;

// Fused z pass: forward FFT of the inputs along z, per-mode update, inverse
// FFT of E', B' along z, all in one launch.  mpt = modes per thread.
hipError_t launch_fused_z(int precision, int ndim, int src, int mpt, const LaunchShape& sh,
                          hipStream_t stream, const PatchDev* patches, const WorkItem* items,
                          int nitems, void* ws, Physics ph);
bool fused_supported(int precision, int ndim, int mpt);

// Plain per-mode update on spectra already transformed along every axis.
hipError_t launch_update(int precision, int src, const LaunchShape& sh, hipStream_t stream,
                         const PatchDev* patches, const WorkItem* items, int nitems, void* ws,
                         Physics ph);

// FP64 plan tables.
hipError_t launch_twiddles(double2* tw, int n, int count, hipStream_t stream);
hipError_t launch_ktable(double* k, int n, double d, int count, int packed_x,
                         const double* fornberg, int nfornberg, int centered,
                         hipStream_t stream);

// Copy the caller's field pointers into a device table (FieldPtrs::table).
hipError_t launch_store_fields(const FieldPtrs& f, FieldPtrs* dst, hipStream_t stream);

// Raise the dynamic-LDS limit of every kernel instantiation (once per process).
hipError_t configure_kernel_attributes();

}  // namespace psatd
