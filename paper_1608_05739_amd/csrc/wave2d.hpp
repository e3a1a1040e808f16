// Wave-resident 2D kernels (wave2d.hip): launchers and the lengths they take.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "kernels.hpp"

namespace psatd {
namespace wave2d {

constexpr int kWavesPerBlock = 4;
constexpr int kBlock = 64 * kWavesPerBlock;

// z line lengths the fused z pass is compiled for.
bool z_supported(int nz);
// z lines of one work item (one wavefront): 64 / (lanes per line).
int z_lines_per_item(int nz);
// double2 elements of one wavefront's LDS region for z lines of length nz.
int z_region(int nz);

// Fused z pass over 2D patches stored as FP32 [kx][z] spectra: per work item
// one wavefront transforms `count` z lines of every input along z, updates
// each mode and transforms E', B' back.  region = double2 elements per wave.
hipError_t launch_z_fused(int src, const LaunchShape& sh, hipStream_t stream,
                          const PatchDev* patches, const WorkItem* items, int nitems, void* ws,
                          Physics ph, int region);

// The same pass with one polarization set per wavefront, for z lines of one
// length nz in z_set_supported (8 points per lane): the launch runs 2 nitems
// wavefronts, two per item; every item's patch must have this nz.
bool z_set_supported(int nz);
hipError_t launch_z_set(int src, int nz, const LaunchShape& sh, hipStream_t stream,
                        const PatchDev* patches, const WorkItem* items, int nitems, void* ws,
                        Physics ph, int region);

hipError_t configure_attributes();

// Fused z pass over 3D patches (wave3d.hip), PSATD forms (src kVacuum, kRho,
// kJForm), nz in z3_supported: per work item one wavefront transforms the
// z lines [first, first + count) of the [kx][y][z] spectra of every input,
// accumulates the six outputs and transforms them back over E and B.
// region = double2 elements per wave (z3_region(nz) for the plan's lengths).
bool z3_supported(int nz);
// double2 elements of one wavefront's LDS in the 3D pass: the exchange region
// and the per-mode coefficients.
int z3_region(int nz);
hipError_t launch_z3_fused(int src, const LaunchShape& sh, hipStream_t stream,
                           const PatchDev* patches, const WorkItem* items, int nitems, void* ws,
                           Physics ph, int region);
hipError_t configure_z3_attributes();

// x passes (wavex.hip): a workgroup of x_block(L) threads transforms a tile
// of up to x_rows_per_item(L) consecutive rows of one component inside one
// run of the spectra layout (L = nx / 2, the complex row length).  kind:
// kXFwd (rows -> spectra) or kXInv.  One launch covers the items of patches
// with nx / 2 = L, with x_lds(L) bytes of LDS per workgroup.
bool x_supported(int L);
int x_rows_per_item(int L);
int x_block(int L);     // threads per workgroup
size_t x_lds(int L);    // bytes of LDS per workgroup
hipError_t launch_x(int kind, int L, const LaunchShape& sh, hipStream_t stream,
                    const PatchDev* patches, const WorkItem* items, int nitems,
                    const FieldPtrs& fields, void* ws);
hipError_t configure_x_attributes();

}  // namespace wave2d
}  // namespace psatd
