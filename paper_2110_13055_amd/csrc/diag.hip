// diag.hip -- the diagnostics of Sec. 4 on the device: the electrode's
// specific surface (for l_c = pi / s), the mean pore velocity U = sum u_i /
// (N phi), and the vertically averaged concentration along the flow axis.
// All sums are FP64 in a fixed order (per tile or per plane chunk, then one
// deterministic pass), so repeated calls give identical numbers.
#include "cdi_internal.h"
#include "device_common.h"
#include "diag_internal.h"

namespace cdi {

namespace {

constexpr int kZChunk = 8;  // z planes per workgroup of the profile

template <class L>
__global__ __launch_bounds__(kTile) void diag_kernel(Grid g, const float *ux, const int *nbr, double *part)
{
    __shared__ double sm[(kTile / 64) * 3];
    const int tile = blockIdx.x;
    const int n = tile * kTile + threadIdx.x;
    double v[3] = {0, 0, 0};
    if (n < g.n_f) {
        v[0] = ux[n];
        int faces = 0;
#pragma unroll
        for (int k = 0; k < 2 * L::D; ++k) faces += nbr[(size_t)k * g.P + n] == kElectrode;
        v[1] = faces;
        int x, y, z;
        unpack_xyz(g, g.fluid[n], x, y, z);
        v[2] = x == 0;
    }
    double out[3];
    block_sum<3>(v, sm, out);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[3 * (size_t)tile + k] = out[k];
}

// Workgroup (x, chunk): the fluid voxels of plane x with z in the chunk.
__global__ __launch_bounds__(256) void profile_part_kernel(Grid g, const float *C, double *part, int chunks)
{
    __shared__ double sm[(256 / 64) * 3];
    const int x = blockIdx.x, zc = blockIdx.y;
    const int z0 = zc * kZChunk, z1 = min(g.nz, z0 + kZChunk);
    const int64_t cells = (int64_t)g.ny * (z1 - z0);
    double v[3] = {0, 0, 0};
    for (int64_t t = threadIdx.x; t < cells; t += blockDim.x) {
        const int y = (int)(t % g.ny), z = z0 + (int)(t / g.ny);
        const int m = g.map[brick_index(g.bk, x, y, z)];
        if (m < 0) continue;
        v[0] += C[m];
        v[1] += C[(size_t)g.P + m];
        v[2] += 1.0;
    }
    double out[3];
    block_sum<3>(v, sm, out);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[((size_t)x * chunks + zc) * 3 + k] = out[k];
}

__global__ void profile_final_kernel(int nx, int chunks, const double *part, double *out)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    double s[3] = {0, 0, 0};
    for (int c = 0; c < chunks; ++c)
        for (int k = 0; k < 3; ++k) s[k] += part[((size_t)x * chunks + c) * 3 + k];
    out[x] = s[2] > 0 ? s[0] / s[2] : 0.0;
    out[nx + x] = s[2] > 0 ? s[1] / s[2] : 0.0;
    out[2 * nx + x] = s[2];
}

}  // namespace

hipError_t launch_diag(int dim, const Grid &g, const float *ux, const int *nbr, double *part, double *out,
                       hipStream_t s)
{
    const int tiles = g.P / kTile;
    if (tiles == 0) return hipSuccess;
    if (dim == 2)
        diag_kernel<D2Q9><<<tiles, kTile, 0, s>>>(g, ux, nbr, part);
    else
        diag_kernel<D3Q19><<<tiles, kTile, 0, s>>>(g, ux, nbr, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_tiles(part, tiles, 3, 3, out, s);
}

int profile_chunks(const Grid &g) { return (g.nz + kZChunk - 1) / kZChunk; }

hipError_t launch_profile_x(const Grid &g, const float *C, double *part, double *out, hipStream_t s)
{
    const int chunks = profile_chunks(g);
    profile_part_kernel<<<dim3(g.nx, chunks), 256, 0, s>>>(g, C, part, chunks);
    profile_final_kernel<<<(g.nx + 255) / 256, 256, 0, s>>>(g.nx, chunks, part, out);
    return hipGetLastError();
}

}  // namespace cdi
