// Specialized 2D kernels for nx = nz = 4096, FP32 storage (fast2d.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "kernels.hpp"

namespace psatd {
namespace fast2d {

// Shapes the kernels are written for.
constexpr int kNX = 4096;
constexpr int kNZfast = 4096;
constexpr int kRowsPerTile = 8;   // rows z1 + 512 z2, z2 < 8
constexpr int kTilesZ = 512;      // z1 range
constexpr int kBlock = 512;

// Work items: x passes {patch, z1, 1, comp}; z pass {patch, kx column, 1, -1}.
hipError_t launch_x_fwd(const LaunchShape& sh, hipStream_t s, const PatchDev* p,
                        const WorkItem* it, int n, const FieldPtrs& f, void* ws);
hipError_t launch_x_inv(const LaunchShape& sh, hipStream_t s, const PatchDev* p,
                        const WorkItem* it, int n, const FieldPtrs& f, void* ws);
// exact_k: the plan's k tables hold the exact wavenumbers (order 0).
hipError_t launch_z_fused(int src, bool exact_k, const LaunchShape& sh, hipStream_t s,
                          const PatchDev* p, const WorkItem* it, int n, void* ws, Physics ph);
hipError_t configure_attributes();
size_t x_fwd_lds_bytes();
size_t x_inv_lds_bytes();
size_t z_lds_bytes();

}  // namespace fast2d
}  // namespace psatd
