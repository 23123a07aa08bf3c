// aux.hip -- read-only passes over the lattice state (moments of the stored
// populations, the positivity bound of the explicit Nernst-Planck step) and
// the fixed-order FP64 reductions behind the residual, the adsorbed amount and
// the solute mass.
#include "device_common.h"

namespace cdi {

namespace {

// Moments of the stored state (what the next step would see), including the
// inlet/outlet extrapolation for boundary nodes with a fluid interior
// neighbour. rho, u, j are optional outputs.
template <class L, int ST, int ODD>
__global__ __launch_bounds__(256) void moments_kernel(Grid g, Phys p, int nee, const void *F,
                                                      const float4 *M, const float *rref, float *rho, float *u,
                                                      float *j)
{
    constexpr int Q = L::Q, D = L::D;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.n_f) return;
    int x, y, z;
    unpack_xyz(g, g.fluid[n], x, y, z);
    int src = n, sx = x;
    bool inlet = false;
    if (nee && g.inout && (x == 0 || x == g.nx - 1)) {
        const int c = nb_map<L>(g, x, y, z, x == 0 ? 1 : 2, false);
        if (c >= 0) {
            src = c;
            sx = x == 0 ? 1 : g.nx - 2;
            inlet = x == 0;
        }
    }
    int nb[Q];
    nb[0] = src;
#pragma unroll
    for (int i = 1; i < Q; ++i)
        nb[i] = (ODD || !kPlain<ST>) ? nb_map<L>(g, sx, y, z, i, g.periodic_x) : kOutside;
    float f[Q];
    // FP32 storage: relative to the plane reference of the node read (see PlaneRef)
    const PlaneRef pr = kPlain<ST> ? plane_ref<0>(g, rref, rref, sx) : PlaneRef{0.f, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    float ref = pr.rout;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        f[i] = gather<L, ST, ODD>(F, g.P, nb, src, i, M, p);
        if (kPlain<ST>) f[i] = rel_pop<L, ODD>(f[i], i, nb, pr);
    }
    if (src != n) {
        float fb[Q];
        const float rb = kPlain<ST> ? plane_ref<0>(g, rref, rref, x).rout : 0.f;
        nee_populations<L>(p, inlet, f, fb, ref, rb);
        ref = rb;
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = fb[i];
    }
    float drho, jx, jy, jz;
    lat_moments<L>(f, drho, jx, jy, jz);
    if (p.forced) {
        jx += 0.5f * p.F[0];
        jy += 0.5f * p.F[1];
        jz += 0.5f * p.F[2];
    }
    const float rh = 1.f + ref + drho;
    const float ri = __builtin_amdgcn_rcpf(rh);
    const int P = g.P;
    if (rho) rho[n] = rh;
    if (u) {
        u[n] = jx * ri;
        u[P + n] = jy * ri;
        if (D == 3) u[2 * (size_t)P + n] = jz * ri;
    }
    if (j) {
        j[n] = jx;
        j[P + n] = jy;
        if (D == 3) j[2 * (size_t)P + n] = jz;
    }
}

// One workgroup per x plane: the mean of drho over the plane's fluid voxels,
// summed in FP64 in a fixed order (each thread a fixed set of voxels, then a
// fixed tree over the threads).
__global__ __launch_bounds__(256) void plane_means_kernel(Grid g, const float *drho, float *rref)
{
    __shared__ double ss[256];
    __shared__ int sc[256];
    const int x = blockIdx.x;
    const int64_t cells = (int64_t)g.ny * g.nz;
    double sum = 0;
    int cnt = 0;
    for (int64_t k = threadIdx.x; k < cells; k += 256) {
        const int y = (int)(k % g.ny), z = (int)(k / g.ny);
        const int m = g.map[brick_index(g.bk, x, y, z)];
        if (m >= 0) {
            sum += (double)ldu(drho, (uint32_t)m);
            ++cnt;
        }
    }
    ss[threadIdx.x] = sum;
    sc[threadIdx.x] = cnt;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            ss[threadIdx.x] += ss[threadIdx.x + h];
            sc[threadIdx.x] += sc[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) rref[x] = sc[0] > 0 ? (float)(ss[0] / sc[0]) : 0.f;
}

template <class L>
__global__ __launch_bounds__(256) void build_nbr_kernel(Grid g, int *nbr)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.n_f) return;
    int x, y, z;
    unpack_xyz(g, g.fluid[n], x, y, z);
    NbCtx c;
    nb_ctx<L>(g, x, y, z, g.periodic_x, c);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) nbr[(size_t)(i - 1) * g.P + n] = nb_get<L>(g, c, i);
}

__global__ void tile_heads_kernel(Grid g, uint32_t *heads)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t * kTile < g.n_f) heads[t] = g.fluid[t * kTile];
}

template <int D>
__global__ void j_from_m_kernel(Grid g, const float4 *M, float *j)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.n_f) return;
    const float4 m = M[n];
    const float r = 1.f + m.x;
    j[n] = r * m.y;
    j[g.P + n] = r * m.z;
    if (D == 3) j[2 * (size_t)g.P + n] = r * m.w;
}

// Single block of 1024 threads; fixed summation order.
__global__ __launch_bounds__(1024) void reduce_tiles_kernel(const double *in, int ntiles, int stride,
                                                            int width, double *out)
{
    __shared__ double sm[1024];
    for (int k = 0; k < width; ++k) {
        double s = 0;
        for (int t = threadIdx.x; t < ntiles; t += 1024) s += in[(size_t)t * stride + k];
        sm[threadIdx.x] = s;
        __syncthreads();
        for (int h = 512; h > 0; h >>= 1) {
            if (threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = sm[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void max_tiles_kernel(const double *in, int ntiles, double *out)
{
    __shared__ double sm[1024];
    double s = 0;
    for (int t = threadIdx.x; t < ntiles; t += 1024) s = fmax(s, in[t]);
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (threadIdx.x < h) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

__global__ __launch_bounds__(kTile) void mass_kernel(Grid g, const float *C, const __half2 *Clo, double *part)
{
    const int n = blockIdx.x * kTile + threadIdx.x;
    double v[2] = {0, 0};
    if (n < g.n_f) {
        const __half2 lo = Clo[n];
        v[0] = (double)C[n] + lo_decode(__low2half(lo));
        v[1] = (double)C[g.P + n] + lo_decode(__high2half(lo));
    }
    __shared__ double sm[(kTile / 64) * 2];
    double s[2];
    block_sum<2>(v, sm, s);
    if (threadIdx.x == 0) {
        part[2 * (size_t)blockIdx.x] = s[0];
        part[2 * (size_t)blockIdx.x + 1] = s[1];
    }
}

__device__ inline float bern(float x) { return x == 0.f ? 1.f : x / expm1f(x); }

// dt * (sum of the coefficients multiplying C_P in the outflow), per node,
// maximum over the block. Positivity of the explicit update needs <= 1.
template <class L>
__global__ __launch_bounds__(kTile) void stability_kernel(Grid g, Phys p, const float *j, double *part)
{
    constexpr int D = L::D;
    const int n = blockIdx.x * kTile + threadIdx.x;
    float worst = 0.f;
    if (n < g.n_f) {
        int x, y, z;
        unpack_xyz(g, g.fluid[n], x, y, z);
        const int P = g.P;
        const float psiP = p.psi ? p.psi[n] : 0.f;
        // the faces' neighbours, then their flux and potential, all loaded
        // before the species' face loops (a load inside a divergent branch
        // waits for its data before the next face starts); across an x end
        // the periodic neighbour, used only by periodic ions
        int mf[2 * D];
        float jN[2 * D], psiN[2 * D];
#pragma unroll
        for (int k = 0; k < 2 * D; ++k) {
            const int sgi = (k & 1) ? -1 : 1;
            const bool xb = k < 2 && (x + sgi < 0 || x + sgi >= g.nx);
            mf[k] = (g.nbr && !xb) ? g.nbr[(size_t)k * P + n]
                                   : nb_map<L>(g, x, y, z, k + 1, xb ? true : (bool)g.periodic_x);
        }
#pragma unroll
        for (int k = 0; k < 2 * D; ++k) {
            const int q = mf[k] >= 0 ? mf[k] : n;
            jN[k] = j[(size_t)(k >> 1) * P + q];
            psiN[k] = p.psi ? p.psi[q] : 0.f;
        }
        for (int s = 0; s < 2; ++s) {
            const float Ds = p.D[s];
            float dg = 0.f;
            for (int k = 0; k < 2 * D; ++k) {
                const int axis = k >> 1;
                const int sgi = (k & 1) ? -1 : 1;
                const float sg = (float)sgi;
                const bool xb = axis == 0 && (x + sgi < 0 || x + sgi >= g.nx);
                if (xb && p.npx != kNpxPeriodic) {
                    if (p.npx == kNpxClosed) continue;
                    const float dpsi = p.psi ? 0.f : -sg * p.dpsi_dx;
                    if (sgi < 0) {
                        const float w = -p.u_in - p.z[s] * Ds * dpsi;
                        dg += Ds * bern(-w / Ds);
                    } else {
                        const float w = j[n] - p.z[s] * Ds * dpsi;
                        dg += p.npx == kNpxDirichlet ? Ds * bern(-w / Ds) : fmaxf(w, 0.f);
                    }
                    continue;
                }
                const int m = mf[k];
                if (m == kElectrode) {
                    dg += p.keff[s];
                } else if (m >= 0) {
                    const float un = 0.5f * (j[(size_t)axis * P + n] + jN[k]) * sg;
                    const float dpsi = p.psi ? psiN[k] - psiP : (axis == 0 ? -sg * p.dpsi_dx : 0.f);
                    const float w = un - p.z[s] * Ds * dpsi;
                    dg += Ds * bern(-w / Ds);
                }
            }
            worst = fmaxf(worst, p.dt * dg);
        }
    }
    __shared__ float sm[kTile];
    sm[threadIdx.x] = worst;
    __syncthreads();
    for (int h = kTile / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

}  // namespace

hipError_t launch_build_nbr(int dim, const Grid &g, int *nbr, hipStream_t s)
{
    const unsigned blocks = (unsigned)((g.n_f + 255) / 256);
    if (blocks == 0) return hipSuccess;
    if (dim == 2)
        build_nbr_kernel<D2Q9><<<blocks, 256, 0, s>>>(g, nbr);
    else
        build_nbr_kernel<D3Q19><<<blocks, 256, 0, s>>>(g, nbr);
    return hipGetLastError();
}

hipError_t launch_tile_heads(const Grid &g, uint32_t *heads, hipStream_t s)
{
    const int tiles = g.P / kTile;
    if (tiles == 0) return hipSuccess;
    tile_heads_kernel<<<(tiles + 255) / 256, 256, 0, s>>>(g, heads);
    return hipGetLastError();
}

namespace {

template <class L>
void launch_moments_l(int st, int odd, unsigned blocks, int nee, const Grid &g, const Phys &p, const void *f,
                      const float4 *M, const float *rref, float *rho, float *u, float *j, hipStream_t s)
{
#define MK(S, O) moments_kernel<L, S, O><<<blocks, 256, 0, s>>>(g, p, nee, f, M, rref, rho, u, j)
    if (st == kMom)
        MK(kMom, 0);
    else if (st == kH16)
        odd == kPull ? MK(kH16, kPull) : odd ? MK(kH16, 1) : MK(kH16, 0);
    else if (st == kF16)
        odd == kPull ? MK(kF16, kPull) : odd ? MK(kF16, 1) : MK(kF16, 0);
    else
        odd == kPull ? MK(kF32, kPull) : odd ? MK(kF32, 1) : MK(kF32, 0);
#undef MK
}

}  // namespace

hipError_t launch_moments(int dim, int st, int odd, int nee, const Grid &g, const Phys &p,
                          const void *f, const float4 *M, const float *rref, float *rho, float *u, float *j,
                          hipStream_t s)
{
    const unsigned blocks = (unsigned)((g.n_f + 255) / 256);
    if (blocks == 0) return hipSuccess;
    if (st < kF32 || st > kH16) return hipErrorInvalidValue;
    if (dim == 2)
        launch_moments_l<D2Q9>(st, odd, blocks, nee, g, p, f, M, rref, rho, u, j, s);
    else
        launch_moments_l<D3Q19>(st, odd, blocks, nee, g, p, f, M, rref, rho, u, j, s);
    return hipGetLastError();
}

hipError_t launch_plane_means(const Grid &g, const float *drho, float *rref, hipStream_t s)
{
    if (g.nx <= 0) return hipSuccess;
    plane_means_kernel<<<g.nx, 256, 0, s>>>(g, drho, rref);
    return hipGetLastError();
}

hipError_t launch_j_from_m(int dim, const Grid &g, const float4 *M, float *j, hipStream_t s)
{
    const unsigned blocks = (unsigned)((g.n_f + 255) / 256);
    if (blocks == 0) return hipSuccess;
    if (dim == 2)
        j_from_m_kernel<2><<<blocks, 256, 0, s>>>(g, M, j);
    else
        j_from_m_kernel<3><<<blocks, 256, 0, s>>>(g, M, j);
    return hipGetLastError();
}

hipError_t launch_reduce_tiles(const double *in, int ntiles, int stride, int width, double *out,
                               hipStream_t s)
{
    reduce_tiles_kernel<<<1, 1024, 0, s>>>(in, ntiles, stride, width, out);
    return hipGetLastError();
}

hipError_t launch_mass(const Grid &g, const float *C, const __half2 *Clo, double *part, double *out, hipStream_t s)
{
    const int tiles = g.P / kTile;
    if (tiles == 0) return hipSuccess;
    mass_kernel<<<tiles, kTile, 0, s>>>(g, C, Clo, part);
    reduce_tiles_kernel<<<1, 1024, 0, s>>>(part, tiles, 2, 2, out);
    return hipGetLastError();
}

hipError_t launch_stability(int dim, const Grid &g, const Phys &p, const float *j, double *part,
                            double *out, hipStream_t s)
{
    const int tiles = g.P / kTile;
    if (tiles == 0) return hipSuccess;
    if (dim == 2)
        stability_kernel<D2Q9><<<tiles, kTile, 0, s>>>(g, p, j, part);
    else
        stability_kernel<D3Q19><<<tiles, kTile, 0, s>>>(g, p, j, part);
    max_tiles_kernel<<<1, 1024, 0, s>>>(part, tiles, out);
    return hipGetLastError();
}

}  // namespace cdi
