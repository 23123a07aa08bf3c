// diag_internal.h -- launchers of the diagnostics of Sec. 4 (diag.hip).
#pragma once

#include "cdi_internal.h"

namespace cdi {

// Per tile: sum of u_x over its fluid nodes, number of fluid-electrode faces,
// number of fluid nodes in the x = 0 plane (3 doubles per tile into part),
// then their totals into out[0..2]. ux: streamwise velocity plane (stride P);
// nbr: the face planes of the neighbour list.
hipError_t launch_diag(int dim, const Grid &g, const float *ux, const int *nbr, double *part, double *out,
                       hipStream_t s);

// Vertical averages: out[x], out[nx + x] = mean C of each species over the
// fluid voxels of plane x, out[2 nx + x] = their number. part: 3 nx zchunks
// doubles (profile_chunks chunks per plane).
int profile_chunks(const Grid &g);
hipError_t launch_profile_x(const Grid &g, const float *C, double *part, double *out, hipStream_t s);

}  // namespace cdi
