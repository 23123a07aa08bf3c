// geometry.hip -- voxel labels from primitives and the compacted fluid-node
// numbering (the paper's image-voxel grid, Sec. 2), plus small fill kernels.
//
// Labels: 0 pore, 1 adsorbing electrode, 2 inert wall. A voxel (i,j,k) is
// solid iff some primitive (disk, sphere, or straight fibre of Sec. 5)
// contains its centre, tested exactly in int64 on 1/256-lattice-unit
// coordinates (centre of voxel i is 128*(2i+1)).
// Fluid voxels are numbered in lexicographic order, x fastest; the result is
// independent of scheduling (a three-pass block scan).
#include "cdi_internal.h"
#include "geometry_internal.h"

namespace cdi {

namespace {

__device__ inline int64_t fdiv256(int64_t a)
{
    // floor(a / 256) for any sign
    return a >= 0 ? a / 256 : -((-a + 255) / 256);
}

__device__ inline int wrapi(int64_t i, int n)
{
    int64_t m = i % n;
    return (int)(m < 0 ? m + n : m);
}

__global__ void init_labels_kernel(uint8_t *labels, int nx, int ny, int64_t nvox, int walls2d)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    uint8_t l = 0;
    if (walls2d) {
        const int y = (int)((v / nx) % ny);
        if (y == 0 || y == ny - 1) l = 2;
    }
    labels[v] = l;
}

// One block per primitive; threads sweep its bounding box. Concurrent writes
// of the value 1 to one byte are benign (same value), and inert walls are
// never overwritten.
__global__ void voxelize_kernel(uint8_t *labels, const int64_t *prims, int dim, int nx, int ny,
                                int nz, int walls_y, int bx)
{
    const int64_t *pr = prims + 4 * (int64_t)blockIdx.x;
    const int64_t r = pr[0], cx = pr[1], cy = pr[2], cz = pr[3];
    const int64_t i0 = fdiv256(cx - r) - 1, i1 = fdiv256(cx + r) + 1;
    const int64_t j0 = fdiv256(cy - r) - 1, j1 = fdiv256(cy + r) + 1;
    int64_t k0 = 0, k1 = 0;
    if (dim == 3) {
        k0 = fdiv256(cz - r) - 1;
        k1 = fdiv256(cz + r) + 1;
    }
    const int64_t ni = i1 - i0 + 1, nj = j1 - j0 + 1, nk = k1 - k0 + 1;
    const int64_t total = ni * nj * nk;
    const int64_t r2 = r * r;
    for (int64_t t = threadIdx.x; t < total; t += blockDim.x) {
        const int64_t i = i0 + t % ni;
        const int64_t j = j0 + (t / ni) % nj;
        const int64_t k = k0 + t / (ni * nj);
        if (i < bx || i >= nx - bx) continue;
        int jj;
        if (dim == 2 && walls_y) {
            if (j < 0 || j >= ny) continue;
            jj = (int)j;
        } else {
            jj = wrapi(j, ny);
        }
        const int kk = dim == 3 ? wrapi(k, nz) : 0;
        const int64_t dx = 128 * (2 * i + 1) - cx;
        const int64_t dy = 128 * (2 * j + 1) - cy;
        const int64_t dz = dim == 3 ? 128 * (2 * k + 1) - cz : 0;
        if (dx * dx + dy * dy + dz * dz <= r2) {
            uint8_t *l = labels + ((int64_t)kk * ny + jj) * nx + i;
            if (*l != 2) *l = 1;
        }
    }
}

// Straight fibres, one block per fibre. A voxel centre within r of the core
// line o + t d lies, in its plane across the dominant axis a of d, within
// r |d| / |d_a| of the point where the line crosses that plane (the in-plane
// distance is at most the 3D distance divided by |d_a| / |d|). Each thread
// takes (plane, window cell) pairs of a window one voxel wider than that
// radius; the exact integer test |(c - o) x d|^2 <= r^2 |d|^2 decides. No
// wrap; x is clipped to the interior slab.
__global__ void voxelize_fibres_kernel(uint8_t *labels, const int64_t *fib, int nx, int ny, int nz, int bx)
{
    const int64_t *F = fib + 8 * (int64_t)blockIdx.x;
    const int64_t r = F[0];
    const int64_t o[3] = {F[1], F[2], F[3]}, d[3] = {F[4], F[5], F[6]};
    int a = 0;
    for (int k = 1; k < 3; ++k)
        if ((d[k] < 0 ? -d[k] : d[k]) > (d[a] < 0 ? -d[a] : d[a])) a = k;
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const int lo[3] = {bx, 0, 0}, hi[3] = {nx - bx, ny, nz};
    const int64_t dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const int64_t r2dd = r * r * dd;
    const double da = (double)(d[a] < 0 ? -d[a] : d[a]);
    const int W = (int)ceil((double)r / 256.0 * sqrt((double)dd) / da) + 1;
    const int side = 2 * W + 1;
    const int64_t cells = (int64_t)side * side;
    const int64_t total = (int64_t)(hi[a] - lo[a]) * cells;
    for (int64_t t = threadIdx.x; t < total; t += blockDim.x) {
        const int ia = lo[a] + (int)(t / cells);
        const int rem = (int)(t % cells);
        const double tt = (double)(128 * (2 * (int64_t)ia + 1) - o[a]) / (double)d[a];
        const double pb = ((double)o[b] + tt * (double)d[b]) / 256.0 - 0.5;
        const double pc = ((double)o[c] + tt * (double)d[c]) / 256.0 - 0.5;
        const int ib = (int)floor(pb + 0.5) - W + rem % side;
        const int ic = (int)floor(pc + 0.5) - W + rem / side;
        if (ib < lo[b] || ib >= hi[b] || ic < lo[c] || ic >= hi[c]) continue;
        int64_t idx[3];
        idx[a] = ia;
        idx[b] = ib;
        idx[c] = ic;
        const int64_t vx = 128 * (2 * idx[0] + 1) - o[0];
        const int64_t vy = 128 * (2 * idx[1] + 1) - o[1];
        const int64_t vz = 128 * (2 * idx[2] + 1) - o[2];
        const int64_t ax = vy * d[2] - vz * d[1], ay = vz * d[0] - vx * d[2], az = vx * d[1] - vy * d[0];
        if (ax * ax + ay * ay + az * az <= r2dd) labels[(idx[2] * ny + idx[1]) * nx + idx[0]] = 1;
    }
}

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;                        // voxels per thread
constexpr int kScanBlock = kScanThreads * kScanItems; // voxels per block

__device__ inline int block_exclusive_scan(int x, int *sm, int *total)
{
    // Hillis-Steele over 256 values in LDS; deterministic.
    const int t = threadIdx.x;
    sm[t] = x;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int y = t >= off ? sm[t - off] : 0;
        __syncthreads();
        sm[t] += y;
        __syncthreads();
    }
    const int incl = sm[t];
    *total = sm[kScanThreads - 1];
    __syncthreads();
    return incl - x;
}

__device__ inline int load_flags(const uint8_t *labels, int64_t nvox, int64_t base, uint8_t fl[kScanItems])
{
    int cnt = 0;
    if (base + kScanItems <= nvox && (((uintptr_t)(labels + base)) & 15) == 0) {
        const uint4 w = *reinterpret_cast<const uint4 *>(labels + base);
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            fl[k] = ((words[k >> 2] >> (8 * (k & 3))) & 0xff) == 0;
            cnt += fl[k];
        }
    } else {
        for (int k = 0; k < kScanItems; ++k) {
            const int64_t v = base + k;
            fl[k] = (v < nvox) && labels[v] == 0;
            cnt += fl[k];
        }
    }
    return cnt;
}

__global__ void count_kernel(const uint8_t *labels, int64_t nvox, int *blk)
{
    __shared__ int sm[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint8_t fl[kScanItems];
    const int cnt = load_flags(labels, nvox, base, fl);
    int total;
    block_exclusive_scan(cnt, sm, &total);
    if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

// Single block: exclusive scan of the per-block counts in place; total -> nfluid.
__global__ void scan_blocks_kernel(int *blk, int64_t nblk, int64_t *nfluid)
{
    __shared__ int sm[kScanThreads];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        const int x = i < nblk ? blk[i] : 0;
        int total;
        const int ex = block_exclusive_scan(x, sm, &total);
        if (i < nblk) blk[i] = (int)(carry + ex);
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *nfluid = carry;
}

__global__ void scatter_kernel(const uint8_t *labels, int64_t nvox, const int *blk, int *map, int *fluid)
{
    __shared__ int sm[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint8_t fl[kScanItems];
    const int cnt = load_flags(labels, nvox, base, fl);
    int total;
    int rank = blk[blockIdx.x] + block_exclusive_scan(cnt, sm, &total);
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t v = base + k;
        if (v >= nvox) break;
        if (fl[k]) {
            map[v] = rank;
            fluid[rank] = (int)v;
            ++rank;
        } else {
            map[v] = labels[v] == 1 ? kElectrode : kInert;
        }
    }
}

// Brick enumeration index e -> voxel coordinates; false for padding voxels.
__device__ inline bool brick_voxel(const Bricks &k, int nx, int ny, int nz, int64_t e, int64_t *v)
{
    const int V = k.bsx + k.bsy + k.bsz;
    const int64_t b = e >> V;
    const int l = (int)(e & ((1 << V) - 1));
    const int x = (int)((b % k.nbx) << k.bsx) | (l & ((1 << k.bsx) - 1));
    const int y = (int)(((b / k.nbx) % k.nby) << k.bsy) | ((l >> k.bsx) & ((1 << k.bsy) - 1));
    const int z = (int)((b / ((int64_t)k.nbx * k.nby)) << k.bsz) | (l >> (k.bsx + k.bsy));
    if (x >= nx || y >= ny || z >= nz) return false;
    *v = ((int64_t)z * ny + y) * nx + x;
    return true;
}

__device__ inline int load_brick_flags(const uint8_t *labels, int nx, int ny, int nz, const Bricks &k,
                                       int64_t E, int64_t base, uint8_t fl[kScanItems],
                                       int64_t vv[kScanItems])
{
    int cnt = 0;
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t e = base + i;
        int64_t v = -1;
        const bool in = e < E && brick_voxel(k, nx, ny, nz, e, &v);
        vv[i] = in ? v : -1;
        fl[i] = in && labels[v] == 0;
        cnt += fl[i];
    }
    return cnt;
}

__device__ inline uint32_t pack_voxel(const Bricks &k, int nx, int ny, int64_t v)
{
    const int x = (int)(v % nx);
    const int64_t t = v / nx;
    return pack_xyz(k, x, (int)(t % ny), (int)(t / ny));
}

__global__ void count_brick_kernel(const uint8_t *labels, int nx, int ny, int nz, Bricks k, int64_t E,
                                   int *blk)
{
    __shared__ int sm[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint8_t fl[kScanItems];
    int64_t vv[kScanItems];
    const int cnt = load_brick_flags(labels, nx, ny, nz, k, E, base, fl, vv);
    int total;
    block_exclusive_scan(cnt, sm, &total);
    if (threadIdx.x == 0) blk[blockIdx.x] = total;
}

__global__ void scatter_brick_kernel(const uint8_t *labels, const int *lexmap, int nx, int ny, int nz,
                                     Bricks k, int64_t E, const int *blk, int *imap, uint32_t *ifluid,
                                     int *lex2int)
{
    __shared__ int sm[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint8_t fl[kScanItems];
    int64_t vv[kScanItems];
    const int cnt = load_brick_flags(labels, nx, ny, nz, k, E, base, fl, vv);
    int total;
    int rank = blk[blockIdx.x] + block_exclusive_scan(cnt, sm, &total);
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t e = base + i;
        if (e >= E) break;
        const int64_t v = vv[i];
        if (fl[i]) {
            imap[e] = rank;
            ifluid[rank] = pack_voxel(k, nx, ny, v);
            lex2int[lexmap[v]] = rank;
            ++rank;
        } else {
            imap[e] = (v >= 0 && labels[v] == 1) ? kElectrode : kInert;
        }
    }
}

__global__ void permute_kernel(const float *src, float *dst, const int *lex2int, int n_f, int P, int d,
                               int to_lex)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_f * d) return;
    const int c = (int)(t / n_f), k = (int)(t % n_f);
    const int n = lex2int[k];
    if (to_lex)
        dst[(size_t)c * n_f + k] = src[(size_t)c * P + n];
    else
        dst[(size_t)c * P + n] = src[(size_t)c * n_f + k];
}

template <class T>
__global__ void fill_kernel(T *p, T v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
hipError_t fill(T *p, T v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    fill_kernel<T><<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init_labels(uint8_t *labels, int nx, int ny, int nz, int walls2d, hipStream_t s)
{
    const int64_t nvox = (int64_t)nx * ny * nz;
    init_labels_kernel<<<(unsigned)((nvox + 255) / 256), 256, 0, s>>>(labels, nx, ny, nvox, walls2d);
    return hipGetLastError();
}

hipError_t launch_voxelize(uint8_t *labels, const int64_t *prims, int64_t nprims, int dim, int nx,
                           int ny, int nz, int walls_y, int buffer_x, hipStream_t s)
{
    if (nprims <= 0) return hipSuccess;
    voxelize_kernel<<<(unsigned)nprims, 256, 0, s>>>(labels, prims, dim, nx, ny, nz, walls_y, buffer_x);
    return hipGetLastError();
}

hipError_t launch_voxelize_fibres(uint8_t *labels, const int64_t *fibres, int64_t nfib, int nx, int ny, int nz,
                                  int buffer_x, hipStream_t s)
{
    if (nfib > 0) voxelize_fibres_kernel<<<(unsigned)nfib, 256, 0, s>>>(labels, fibres, nx, ny, nz, buffer_x);
    return hipGetLastError();
}

int64_t compact_blocks(int64_t nvox) { return (nvox + kScanBlock - 1) / kScanBlock; }

hipError_t launch_compact(const uint8_t *labels, int64_t nvox, int *map, int *fluid, int *blk,
                          int64_t *nfluid, hipStream_t s)
{
    const int64_t nblk = compact_blocks(nvox);
    count_kernel<<<(unsigned)nblk, kScanThreads, 0, s>>>(labels, nvox, blk);
    scan_blocks_kernel<<<1, kScanThreads, 0, s>>>(blk, nblk, nfluid);
    scatter_kernel<<<(unsigned)nblk, kScanThreads, 0, s>>>(labels, nvox, blk, map, fluid);
    return hipGetLastError();
}

int64_t brick_enum_size(const Bricks &bk)
{
    return ((int64_t)bk.nbx * bk.nby * bk.nbz) << (bk.bsx + bk.bsy + bk.bsz);
}

hipError_t launch_compact_bricks(const uint8_t *labels, const int *lexmap, int nx, int ny, int nz,
                                 const Bricks &bk, int *imap, uint32_t *ifluid, int *lex2int, int *blk,
                                 int64_t *nfluid, hipStream_t s)
{
    const int64_t E = brick_enum_size(bk);
    const int64_t nblk = compact_blocks(E);
    count_brick_kernel<<<(unsigned)nblk, kScanThreads, 0, s>>>(labels, nx, ny, nz, bk, E, blk);
    scan_blocks_kernel<<<1, kScanThreads, 0, s>>>(blk, nblk, nfluid);
    scatter_brick_kernel<<<(unsigned)nblk, kScanThreads, 0, s>>>(labels, lexmap, nx, ny, nz, bk, E, blk,
                                                                 imap, ifluid, lex2int);
    return hipGetLastError();
}

hipError_t launch_permute(const float *src, float *dst, const int *lex2int, int n_f, int P, int d,
                          int to_lex, hipStream_t s)
{
    const int64_t n = (int64_t)n_f * d;
    if (n <= 0) return hipSuccess;
    permute_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, dst, lex2int, n_f, P, d, to_lex);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) { return fill<float>(p, v, n, s); }
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) { return fill<uint32_t>(p, v, n, s); }
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) { return fill<double>(p, v, n, s); }

}  // namespace cdi
