// reduce_common.h -- the persistent-workgroup machinery of the Krylov
// solvers (pot.hip, np_solve.hip): XCD-contiguous tile ranges, fixed-order
// workgroup sums and the totals of per-workgroup partial sums.
#pragma once

#include "cdi_internal.h"
#include "device_common.h"

namespace cdi {

// Contiguous tile range of this workgroup at its XCD-contiguous position:
// an XCD sweeps one contiguous eighth of the lattice.
__device__ inline void tile_range(int ntiles, int &t0, int &t1)
{
    const long long G = gridDim.x;
    const long long c = xcd_tile(blockIdx.x, gridDim.x);
    t0 = (int)(c * ntiles / G);
    t1 = (int)((c + 1) * ntiles / G);
}

// Sum of v over the workgroup in a fixed order, returned to every thread.
__device__ inline double wg_sum(double v, double *sm)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();  // sm may still be read from a previous call
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    double s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sm[w];
    return s;
}

// Whether the solve has stopped (state[slot] != 0), read once per workgroup
// so that all its waves take the same branch.
__device__ inline bool stopped_at(const double *state, int slot, int *flag)
{
    if (threadIdx.x == 0) *flag = state[slot] != 0.0;
    __syncthreads();
    return *flag != 0;
}

// Total of a partial-sum region (G values), the same in every workgroup.
__device__ inline double region_sum(const double *part, int G, double *sm)
{
    double v = 0;
    for (int k = threadIdx.x; k < G; k += blockDim.x) v += part[k];
    return wg_sum(v, sm);
}

}  // namespace cdi
