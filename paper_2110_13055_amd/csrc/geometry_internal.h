// geometry_internal.h -- launcher of the straight-fibre voxelisation
// (geometry.hip; the other geometry launchers are declared in cdi_internal.h).
#pragma once

#include "cdi_internal.h"

namespace cdi {

// Electrode voxels of nfib straight fibres (8 int64 each: r, ox, oy, oz, dx,
// dy, dz, unused; 1/256 lattice units, d an integer direction) into labels
// that were cleared to 0: a voxel of the interior slab is 1 iff its centre
// lies within r of some fibre's infinite core line. One block per fibre.
hipError_t launch_voxelize_fibres(uint8_t *labels, const int64_t *fibres, int64_t nfib, int nx, int ny, int nz,
                                  int buffer_x, hipStream_t s);

}  // namespace cdi
