// device_common.h -- device helpers shared by the step and auxiliary kernels:
// neighbour lookup through the fluid index map, the BGK equilibrium, the AA
// storage rules, the inlet/outlet extrapolation and block reductions.
//
// AA storage rules (Bailey et al. 2009). With the stored state at parity 0
// ("A"), the post-streaming population f_i(x) sits in node x, slot i; a step
// reads it there, collides, and writes f*_i back into node x, slot opp(i).
// With the state at parity 1 ("B"), f_i(x) sits in node x - e_i, slot opp(i)
// when that voxel is fluid, else in node x, slot i (it was reflected); a step
// reads it there and writes f*_i into node x + e_i, slot i (fluid), or into
// node x, slot opp(i) (half-way bounce-back off a solid face, the no-flow
// rule). Each node reads and writes the same set of slots, so a step is
// race-free in place.
//
// FP16 storage keeps, instead of f - w_i, the post-collision deviation from
// the emitting node's equilibrium, times hs; the emitter's moments
// (rho - 1, u) are kept in FP32. The emitter of f_i(x) is x - e_i if that
// voxel is fluid, else x itself (which sent it in direction opp(i)).
//
// Pull streaming (ODD = kPull) keeps two arrays: a step reads f_i(x) from
// node x - e_i, slot i of the input array when that voxel is fluid, else from
// node x, slot opp(i) (its own reflected population), and writes f*_i into
// node x, slot i of the output array.
//
// Moment storage keeps the moments alone: with tau = 1 and no body force the
// BGK post-collision populations are exactly the equilibrium of the node's
// moments (the FP16 deviations above are then identically zero), so f_i(x)
// is the emitter's equilibrium and no population is stored; the AA parity
// plays no role.
#pragma once

#include "cdi_internal.h"

namespace cdi {

// Element idx of an array whose base is the same for the whole wave. The
// address is formed as base + a 32-bit byte offset, which the hardware takes
// as a scalar base plus one vector offset: no 64-bit address arithmetic per
// lane, and one offset serves every array indexed by the same node. The host
// keeps idx * sizeof(T) below 2^32.
template <class T>
__device__ __forceinline__ T ldu(const T *base, uint32_t idx)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + idx * (uint32_t)sizeof(T));
}

template <class T>
__device__ __forceinline__ void stu(T *base, uint32_t idx, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * (uint32_t)sizeof(T)) = v;
}

// blockIdx -> tile: workgroups are dealt round-robin over the 8 XCDs, each
// with its own L2; this keeps consecutive tiles on one XCD so that the y/z
// neighbours a tile touches were mostly fetched by the same L2.
__device__ inline int xcd_tile(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int xcd = b & 7, k = b >> 3;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

// Tile processed by this workgroup: its XCD-local position, through the
// (band, z) schedule when there is one.
__device__ inline int block_tile(const Grid &g)
{
    const int pos = xcd_tile(blockIdx.x, gridDim.x);
    return g.sched ? g.sched[pos] : pos;
}

// map value of the neighbour of (x,y,z) along direction i: fluid index,
// kElectrode, kInert, or kOutside past an open x end. y and z wrap.
template <class L>
__device__ inline int nb_map(const Grid &g, int x, int y, int z, int i, bool periodic_x)
{
    int xn = x + L::ex[i];
    if (xn < 0 || xn >= g.nx) {
        if (!periodic_x) return kOutside;
        xn = xn < 0 ? xn + g.nx : xn - g.nx;
    }
    int yn = y + L::ey[i];
    yn = yn < 0 ? yn + g.ny : (yn >= g.ny ? yn - g.ny : yn);
    int zn = z;
    if (L::D == 3) {
        zn = z + L::ez[i];
        zn = zn < 0 ? zn + g.nz : (zn >= g.nz ? zn - g.nz : zn);
    }
    return g.map[brick_index(g.bk, xn, yn, zn)];
}

__device__ inline void unpack_xyz(const Grid &g, uint32_t c, int &x, int &y, int &z)
{
    x = (int)(c & ((1u << g.bk.cbx) - 1));
    y = (int)((c >> g.bk.cbx) & ((1u << g.bk.cby) - 1));
    z = (int)(c >> (g.bk.cbx + g.bk.cby));
}

// Neighbour lookup context of one voxel: for each axis and offset -1/0/+1,
// that axis's share of the neighbour's brick-ordered index. The brick part
// (above the in-brick bits) and the in-brick part occupy disjoint bits, so a
// neighbour's index is the plain sum of its three axis shares: one three-way
// add per lattice direction. Coordinates wrap on every axis (the index is
// always in range); xo marks offsets beyond an open x end.
struct NbCtx {
    uint32_t X[3], Y[3], Z[3];
    bool xo[3];
};

template <class L>
__device__ inline void nb_ctx(const Grid &g, int x, int y, int z, bool periodic_x, NbCtx &c)
{
    const Bricks &k = g.bk;
    const int V = k.bsx + k.bsy + k.bsz;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int xn = x + d - 1;
        bool out = false;
        if (xn < 0 || xn >= g.nx) {
            out = !periodic_x;
            xn = xn < 0 ? xn + g.nx : xn - g.nx;
        }
        c.xo[d] = out;
        c.X[d] = ((uint32_t)(xn >> k.bsx) << V) | (uint32_t)(xn & ((1 << k.bsx) - 1));
        int yn = y + d - 1;
        yn = yn < 0 ? yn + g.ny : (yn >= g.ny ? yn - g.ny : yn);
        c.Y[d] = ((uint32_t)((yn >> k.bsy) * k.nbx) << V) | ((uint32_t)(yn & ((1 << k.bsy) - 1)) << k.bsx);
        if (L::D == 3) {
            int zn = z + d - 1;
            zn = zn < 0 ? zn + g.nz : (zn >= g.nz ? zn - g.nz : zn);
            c.Z[d] = ((uint32_t)((zn >> k.bsz) * k.nbx * k.nby) << V) |
                     ((uint32_t)(zn & ((1 << k.bsz) - 1)) << (k.bsx + k.bsy));
        } else {
            c.Z[d] = 0;
        }
    }
}

// map value of the neighbour along direction i (see nb_map). Past an open x
// end the wrapped voxel is read (always in range) and replaced by kOutside.
template <class L>
__device__ inline int nb_get(const Grid &g, const NbCtx &c, int i)
{
    const int dx = L::ex[i] + 1, dy = L::ey[i] + 1, dz = L::ez[i] + 1;
    const int m = ldu(g.map, c.X[dx] + c.Y[dy] + c.Z[dz]);
    return (L::ex[i] != 0 && c.xo[dx]) ? kOutside : m;
}

// BGK equilibrium minus w_i for a direction of weight w, from rho - 1, u and
// e.u: quadratic in u, or its linear (Stokes) part.
__device__ inline float feq_bar_eu(float w, float drho, float eu, float ux, float uy, float uz, int linear)
{
    const float rho = 1.f + drho;
    if (linear) return w * (drho + 3.f * rho * eu);
    const float uu = ux * ux + uy * uy + uz * uz;
    return w * (drho + rho * (3.f * eu + 4.5f * eu * eu - 1.5f * uu));
}

// The same for lattice direction i.
template <class L>
__device__ inline float feq_bar(int i, float drho, float ux, float uy, float uz, int linear)
{
    const float eu = L::ex[i] * ux + L::ey[i] * uy + L::ez[i] * uz;
    return feq_bar_eu(L::w[i], drho, eu, ux, uy, uz, linear);
}

// Population plane i of node n (planes P apart).
template <int FP16>
__device__ inline float ld(const void *F, int P, int i, int n)
{
    const size_t o = (size_t)i * P + n;
    if (FP16) return __half2float(reinterpret_cast<const __half *>(F)[o]);
    return reinterpret_cast<const float *>(F)[o];
}

template <int FP16>
__device__ inline void st(void *F, int P, int i, int n, float v)
{
    const size_t o = (size_t)i * P + n;
    if (FP16)
        reinterpret_cast<__half *>(F)[o] = __float2half_rn(v);
    else
        reinterpret_cast<float *>(F)[o] = v;
}

// Stored value behind the incoming population i of node n (FP32 f - w_i or
// the scaled FP16 deviation; nothing with moment storage).
template <class L, int ST, int ODD>
__device__ inline float gather_raw(const void *F, int P, const int *nb, int n, int i)
{
    if (ST == kMom) return 0.f;
    const int j = L::opp[i];
    const bool fl = (i != 0) && nb[j] >= 0;
    if (ODD == kPull) return fl ? ld<ST == kF16>(F, P, i, nb[j]) : ld<ST == kF16>(F, P, j, n);
    if (!ODD || i == 0 || !fl) return ld<ST == kF16>(F, P, i, n);
    return ld<ST == kF16>(F, P, j, nb[j]);
}

// FP16 and moment storage: f_i - w_i from the stored value and the emitter's
// moments m. The emitter x - e_i sent it along e_i; a reflected one (fl
// false) was sent by x along e_opp(i) = -e_i, which only flips the sign of
// e.u (w_opp(i) = w_i).
template <class L, int ST>
__device__ inline float from_emitter(float raw, int i, bool fl, float4 m, const Phys &p)
{
    const float eu = L::ex[i] * m.y + L::ey[i] * m.z + L::ez[i] * m.w;
    const float fe = feq_bar_eu(L::w[i], m.x, fl ? eu : -eu, m.y, m.z, m.w, p.linear_eq);
    return ST == kMom ? fe : fe + raw * p.hs_inv;
}

// Incoming f_i - w_i of node n (nb: map values of n's neighbours; M: the
// emitters' moments, FP16 and moment storage; ST: kF32, kF16 or kMom).
template <class L, int ST, int ODD>
__device__ inline float gather(const void *F, int P, const int *nb, int n, int i, const float4 *M,
                               const Phys &p)
{
    const float raw = gather_raw<L, ST, ODD>(F, P, nb, n, i);
    if (ST == kF32) return raw;
    const int j = L::opp[i];
    const bool fl = (i != 0) && nb[j] >= 0;
    return from_emitter<L, ST>(raw, i, fl, ldu(M, (uint32_t)(fl ? nb[j] : n)), p);
}

// Store the outgoing value of direction i (FP32: f* - w_i; FP16: scaled
// deviation; moment storage: nothing). F: the array written.
template <class L, int ST, int ODD>
__device__ inline void scatter(void *F, int P, const int *nb, int n, int i, float v)
{
    if (ST == kMom) return;
    constexpr bool H = ST == kF16;
    if (ODD == kPull)
        st<H>(F, P, i, n, v);
    else if (!ODD || i == 0)
        st<H>(F, P, L::opp[i], n, v);
    else if (nb[i] >= 0)
        st<H>(F, P, i, nb[i], v);
    else
        st<H>(F, P, L::opp[i], n, v);
}

// Non-equilibrium extrapolation (Guo, Zheng & Shi 2002) for the inlet
// (velocity u_in) or outlet (density rho_out) node next to the interior node
// whose post-streaming populations are fc: the boundary takes the target
// equilibrium plus the interior node's non-equilibrium part.
template <class L>
__device__ inline void nee_populations(const Phys &p, bool inlet, const float (&fc)[L::Q],
                                       float (&fb)[L::Q])
{
    float dr = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        dr += fc[i];
        jx += L::ex[i] * fc[i];
        jy += L::ey[i] * fc[i];
        jz += L::ez[i] * fc[i];
    }
    const float ri = 1.f / (1.f + dr);
    const float ux = jx * ri, uy = jy * ri, uz = jz * ri;
    const float tdr = inlet ? dr : p.rho_out - 1.f;
    const float tx = inlet ? p.u_in : ux, ty = inlet ? 0.f : uy, tz = inlet ? 0.f : uz;
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        fb[i] = feq_bar<L>(i, tdr, tx, ty, tz, p.linear_eq) +
                (fc[i] - feq_bar<L>(i, dr, ux, uy, uz, p.linear_eq));
}

// Scharfetter-Gummel flux from P to N with normal drift w, Pe = w / D:
// D [B(-Pe) C_P - B(Pe) C_N], B(x) = x / (e^x - 1). With Bs(x) = B(x) + x/2 =
// (x/2) coth(x/2), an even function, this is exactly
//   D Bs(Pe) (C_P - C_N) + (w/2) (C_P + C_N):
// a symmetric diffusive part and a central advective part, with no sign
// cases. Seen from N the operands are C_P - C_N negated, the same C_P + C_N,
// the same Pe^2 and w/2 negated, so the two cells of a face form exactly
// opposite values. Bs needs only Pe^2: below |Pe| = 1/2 its series
// 1 + x^2/12 - x^4/720 + x^6/30240 (next term below 3e-8 there), above the
// closed form with the hardware exponential (e^|x| - 1 >= 0.64, no
// cancellation). hw = w / 2, invD2 = 2 / D.
__device__ inline float sg_flux(float D, float invD2, float hw, float cp, float cn)
{
    const float pe = hw * invD2;
    const float x2 = pe * pe;
    float bs;
    if (x2 < 0.25f) {
        bs = fmaf(x2, fmaf(x2, fmaf(x2, 1.f / 30240.f, -1.f / 720.f), 1.f / 12.f), 1.f);
    } else {
        const float a = fabsf(pe);
        const float e = __expf(a);
        bs = 0.5f * a * (e + 1.f) * __builtin_amdgcn_rcpf(e - 1.f);
    }
    return fmaf(D * bs, cp - cn, hw * (cp + cn));
}

// Sum over the block in a fixed order (wave shuffles, then the waves in
// order); the result is valid in thread 0. sm holds (blockDim/64) * N doubles.
template <int N>
__device__ inline void block_sum(double (&v)[N], double *sm, double (&out)[N])
{
    // a wave whose lanes all hold 0 (most waves, for the inlet/outlet and
    // adsorption amounts) skips the shuffles: its sum is 0 either way
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (__ballot(v[k] != 0.0))
            for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) sm[wave * N + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double s = 0;
            for (int w = 0; w < nw; ++w) s += sm[w * N + k];
            out[k] = s;
        }
    }
}

}  // namespace cdi
