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
        // brick-row products as 24-bit multiplies (full rate; the 32-bit
        // multiply issues at a quarter): below 2^30 voxels, no brick count or
        // brick index reaches 2^24
        c.Y[d] = (__umul24((uint32_t)(yn >> k.bsy), (uint32_t)k.nbx) << V) |
                 ((uint32_t)(yn & ((1 << k.bsy) - 1)) << k.bsx);
        if (L::D == 3) {
            int zn = z + d - 1;
            zn = zn < 0 ? zn + g.nz : (zn >= g.nz ? zn - g.nz : zn);
            c.Z[d] = (__umul24((uint32_t)(zn >> k.bsz), (uint32_t)(k.nbx * k.nby)) << V) |
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

// acc + c v for a lattice vector component c (-1, 0 or 1 on D2Q9 and D3Q19;
// a constant once a direction loop is unrolled): the product with 0 is
// dropped and the others become an add or a subtraction. The compiler may not
// drop 0 * v by itself (under IEEE rules it is NaN for an infinite v); the
// value is the same, up to the sign of a zero.
__device__ __forceinline__ float lat_add(float acc, int c, float v)
{
    return c == 0 ? acc : (c > 0 ? acc + v : acc - v);
}

// e_i . u, from -0 (the exact additive identity: -0 + v is v for every v).
template <class L>
__device__ __forceinline__ float lat_dot(int i, float ux, float uy, float uz)
{
    return lat_add(lat_add(lat_add(-0.f, L::ex[i], ux), L::ey[i], uy), L::ez[i], uz);
}

// Zeroth and first moments of f: d = sum_i f_i, j = sum_i e_i f_i.
template <class L>
__device__ __forceinline__ void lat_moments(const float (&f)[L::Q], float &d, float &jx, float &jy, float &jz)
{
    d = jx = jy = jz = -0.f;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        d += f[i];
        jx = lat_add(jx, L::ex[i], f[i]);
        jy = lat_add(jy, L::ey[i], f[i]);
        jz = lat_add(jz, L::ez[i], f[i]);
    }
}

// 1 / rho from rho - 1: the hardware reciprocal (within 1 ulp), one
// instruction where an IEEE division takes ten. Every kernel that forms u =
// j / rho uses it, so they all form the same u.
__device__ __forceinline__ float inv_rho(float drho) { return __builtin_amdgcn_rcpf(1.f + drho); }

// BGK equilibrium less w_i (1 + R), R a reference density deviation, split
// into per-node terms so that a direction costs two fused multiply-adds and
// a product: with dr = rho - 1 - R it is w_i (a + e.u (b + c e.u)), where
// a = dr - (3/2) rho u.u, b = 3 rho and c = (9/2) rho; the linear (Stokes)
// part has a = dr and c = 0.
struct EqTerms {
    float a, b, c;
};

__device__ inline EqTerms eq_terms(float dr, float rho, float ux, float uy, float uz, int linear)
{
    if (linear) return EqTerms{dr, 3.f * rho, 0.f};
    const float uu = ux * ux + uy * uy + uz * uz;
    return EqTerms{fmaf(-1.5f * rho, uu, dr), 3.f * rho, 4.5f * rho};
}

__device__ __forceinline__ float feq_eu(float w, const EqTerms &t, float eu)
{
    return w * fmaf(eu, fmaf(t.c, eu, t.b), t.a);
}

// direction i of the node whose terms are t
template <class L>
__device__ __forceinline__ float feq_dir(int i, const EqTerms &t, float ux, float uy, float uz)
{
    return feq_eu(L::w[i], t, lat_dot<L>(i, ux, uy, uz));
}

// one direction of weight w, from dr = rho - 1 - R, rho and e.u, where each
// direction has its own moments (the emitters' equilibria of the FP16 and
// moment storages): the same polynomial, evaluated directly
__device__ inline float feq_rel_eu(float w, float dr, float rho, float eu, float ux, float uy, float uz, int linear)
{
    if (linear) return w * (dr + 3.f * rho * eu);
    const float uu = ux * ux + uy * uy + uz * uz;
    return w * (dr + rho * (3.f * eu + 4.5f * eu * eu - 1.5f * uu));
}

// The same with R = 0 (equilibrium minus w_i, from rho - 1).
__device__ inline float feq_bar_eu(float w, float drho, float eu, float ux, float uy, float uz, int linear)
{
    return feq_rel_eu(w, drho, 1.f + drho, eu, ux, uy, uz, linear);
}

// FP32 population storage holds f_i - w_i (1 + R[x_s]), where x_s is the x
// plane of the node whose slot holds the value (pull streaming: the emitter,
// the node that collided it; AA: the node written to) and R[x] is a reference
// density deviation per x plane (the plane mean of rho - 1, renewed now and
// then: the stored values then carry only the local fluctuations, which FP32
// rounds far more finely than f - w_i near a pressure drop). A step reads
// with table Rin and writes with table Rout (equal except on the step that
// renews R) and works with g_i = f_i - w_i (1 + Rout[x]) = stored +
// w_i (Rin[x_s] - Rout[x]). A value written into the slot of the neighbour
// x + e_i (AA, odd parity) is stored as g + w_i (Rout[x] - Rout[x + e_x]).
struct PlaneRef {
    float rout;   // Rout[x]
    float dIn[3]; // Rin[x - ex] - Rout[x], ex = -1, 0, 1
    float dOut[3];// Rout[x] - Rout[x + ex]
};

// (dOut only for the odd AA parity, which writes into neighbours' slots)
template <int ODD>
__device__ inline PlaneRef plane_ref(const Grid &g, const float *rin, const float *rout, int x)
{
    PlaneRef r{0.f, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    if (!rin) return r;
    const int xm = x > 0 ? x - 1 : (g.periodic_x ? g.nx - 1 : 0);
    const int xp = x < g.nx - 1 ? x + 1 : (g.periodic_x ? 0 : g.nx - 1);
    r.rout = ldu(rout, (uint32_t)x);
    r.dIn[0] = ldu(rin, (uint32_t)xp) - r.rout;  // ex = -1: the slot's node is at x + 1
    r.dIn[1] = ldu(rin, (uint32_t)x) - r.rout;
    r.dIn[2] = ldu(rin, (uint32_t)xm) - r.rout;  // ex = +1: at x - 1
    if (ODD == 1) {
        r.dOut[0] = r.rout - ldu(rout, (uint32_t)xm);
        r.dOut[2] = r.rout - ldu(rout, (uint32_t)xp);
    }
    return r;
}

// g_i from the stored value read for direction i (ODD: the kernels' parity
// argument) of a node whose neighbours are nb.
template <class L, int ODD>
__device__ __forceinline__ float rel_pop(float raw, int i, const int *nb, const PlaneRef &r)
{
    const bool fl = (i != 0) && nb[L::opp[i]] >= 0;
    const bool there = ODD != 0 && fl;  // pull or odd parity: read in the emitter's slot
    return raw + L::w[i] * (there ? r.dIn[L::ex[i] + 1] : r.dIn[1]);
}

// The value to store for outgoing g_i (relative to Rout[x]).
template <class L, int ODD>
__device__ __forceinline__ float stored_pop(float g, int i, const int *nb, const PlaneRef &r)
{
    if (ODD != 1 || i == 0) return g;  // written into the node's own slot
    return nb[i] >= 0 ? g + L::w[i] * r.dOut[L::ex[i] + 1] : g;
}

// Populations are stored in blocks of 64 nodes, one wave: block k holds the
// Q directions of nodes 64k .. 64k + 63, direction by direction (64
// consecutive values each). A wave's access to one direction is one
// contiguous run of 256 bytes (FP32) as with whole planes, but the Q streams
// of a block lie in one region of Q x 256 bytes instead of Q planes far
// apart. Measured on the 512^3 electrode against whole planes of P values:
// FP32 fused step 3 % and flow-only step 6 % faster (blocks of 256 nodes:
// 0.5 % slower than 64). P is a multiple of the 256-node tile, so every block
// is whole.
constexpr int kPopBlockLog = 6;

// (the node's part, one 64-bit product, and the direction's constant part
// apart, so that a node's Q accesses share the first and fold the second
// into the instructions' offsets)
template <int Q, class T>
__device__ __forceinline__ T *pop_at(void *F, int q, int n)
{
    T *const node = reinterpret_cast<T *>(F) + (size_t)(uint32_t)(n >> kPopBlockLog) * (Q << kPopBlockLog) +
                    (n & ((1 << kPopBlockLog) - 1));
    return node + (q << kPopBlockLog);
}
template <int Q, class T>
__device__ __forceinline__ const T *pop_at(const void *F, int q, int n)
{
    const T *const node = reinterpret_cast<const T *>(F) +
                          (size_t)(uint32_t)(n >> kPopBlockLog) * (Q << kPopBlockLog) + (n & ((1 << kPopBlockLog) - 1));
    return node + (q << kPopBlockLog);
}

// Value of direction a at node na, or of direction b at node nb (one of the
// two per lane).
template <int FP16, int Q>
__device__ __forceinline__ float ld_pair(const void *F, int a, int na, int b, int nb, bool first)
{
    const int q = first ? a : b, m = first ? na : nb;
    if (FP16) return __half2float(*pop_at<Q, __half>(F, q, m));
    return *pop_at<Q, float>(F, q, m);
}

template <int FP16, int Q>
__device__ __forceinline__ void st_pair(void *F, int a, int na, int b, int nb, bool first, float v)
{
    const int q = first ? a : b, m = first ? na : nb;
    if (FP16)
        *pop_at<Q, __half>(F, q, m) = __float2half_rn(v);
    else
        *pop_at<Q, float>(F, q, m) = v;
}

// Stored value behind the incoming population i of node n (FP32 f - w_i or
// the scaled FP16 deviation; nothing with moment storage).
template <class L, int ST, int ODD>
__device__ inline float gather_raw(const void *F, int P, const int *nb, int n, int i)
{
    if (ST == kMom) return 0.f;
    constexpr bool H = kHalfPop<ST>;
    const int j = L::opp[i];
    const bool fl = (i != 0) && nb[j] >= 0;
    // pull: plane i of the emitter x - e_i, or the node's own reflected plane j
    if (ODD == kPull) return ld_pair<H, L::Q>(F, i, nb[j], j, n, fl);
    // AA: plane i of the node itself, or (odd parity, fluid emitter) plane j of the emitter
    return ld_pair<H, L::Q>(F, i, n, j, nb[j], !ODD || i == 0 || !fl);
}

// FP16 and moment storage: f_i - w_i from the stored value and the emitter's
// moments m. The emitter x - e_i sent it along e_i; a reflected one (fl
// false) was sent by x along e_opp(i) = -e_i, which only flips the sign of
// e.u (w_opp(i) = w_i).
template <class L, int ST>
__device__ inline float from_emitter(float raw, int i, bool fl, float4 m, const Phys &p)
{
    // the full product, zeros included: with every component of m used, the
    // compiler keeps each emitter's float4 one load (lat_dot let it narrow the
    // loads of directions that need fewer components into several, and the
    // moment storage's fused step took 7 % longer)
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
    if (ST == kH16) return raw * p.hs_inv;
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
    constexpr bool H = kHalfPop<ST>;
    const int j = L::opp[i];
    if (ODD == kPull)
        st_pair<H, L::Q>(F, i, n, i, n, true, v);  // the node's own slot i
    else
        // even parity (or the rest direction): the node's own plane opp(i); odd
        // parity: plane i of the fluid neighbour x + e_i, else (reflected) plane opp(i)
        st_pair<H, L::Q>(F, j, n, i, nb[i], !ODD || i == 0 || nb[i] < 0, v);
}

// Non-equilibrium extrapolation (Guo, Zheng & Shi 2002) for the inlet
// (velocity u_in) or outlet (density rho_out) node next to the interior node
// whose post-streaming populations are fc: the boundary takes the target
// equilibrium plus the interior node's non-equilibrium part. fc is relative to
// the interior node's reference rc (fc_i = f_i - w_i (1 + rc)), fb is returned
// relative to the boundary node's rb (0 and 0 for f - w_i storage).
template <class L>
__device__ inline void nee_populations(const Phys &p, bool inlet, const float (&fc)[L::Q], float (&fb)[L::Q],
                                       float rc = 0.f, float rb = 0.f)
{
    float dr, jx, jy, jz;
    lat_moments<L>(fc, dr, jx, jy, jz);
    const float rho = 1.f + rc + dr;
    const float ri = __builtin_amdgcn_rcpf(rho);
    const float ux = jx * ri, uy = jy * ri, uz = jz * ri;
    // target: inlet (rho of the interior node, u_in), outlet (rho_out, u of the interior node)
    const float trho = inlet ? rho : p.rho_out;
    const float tx = inlet ? p.u_in : ux, ty = inlet ? 0.f : uy, tz = inlet ? 0.f : uz;
    const float tdr = inlet ? (rc + dr) - rb : (p.rho_out - 1.f) - rb;
    const EqTerms te = eq_terms(tdr, trho, tx, ty, tz, p.linear_eq), ce = eq_terms(dr, rho, ux, uy, uz, p.linear_eq);
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        fb[i] = feq_dir<L>(i, te, tx, ty, tz) + (fc[i] - feq_dir<L>(i, ce, ux, uy, uz));
}

// Concentrations are stored as an FP32 value and an FP16 remainder per
// species (times 2^24): value + remainder carry the explicit update's sum to
// about 2^-35 of C, so increments far below half an FP32 ulp accumulate in the
// remainder instead of being dropped. (Rounded to FP32 alone, the update
// stalls wherever a cell's change per step falls below half an ulp, which
// near a steady state left C up to 1e-3 off after 20000 steps.) A remainder
// too large for FP16 (|C| beyond 2^15) is dropped.
__device__ __forceinline__ float lo_decode(__half h) { return __half2float(h) * (1.f / 16777216.f); }
__device__ __forceinline__ __half lo_encode(float lo)
{
    const float t = lo * 16777216.f;
    return __float2half_rn(fabsf(t) < 65000.f ? t : 0.f);
}

// a + b = s + e exactly, s = fl(a + b) (Knuth's TwoSum).
__device__ __forceinline__ float two_sum(float a, float b, float &e)
{
    const float s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
    return s;
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

// Sum of v over the wave in a fixed order, the same value in every lane:
// neighbouring pairs, then quads, then eights and rows of 16 by DPP lane
// permutations within each row of 16 lanes (VALU only, no LDS), then the four
// rows' sums, each read from the row's first lane, in row order. Every lane
// of the wave must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_plus(float v)
{
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float wave_sum(float v)
{
    v = dpp_plus<0xB1>(v);   // quad_perm [1,0,3,2]: pairs
    v = dpp_plus<0x4E>(v);   // quad_perm [2,3,0,1]: quads
    v = dpp_plus<0x124>(v);  // row_ror:4: two quads
    v = dpp_plus<0x128>(v);  // row_ror:8: the row of 16
    const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
    return ((r0 + r1) + r2) + r3;
}

// Per-tile FP64 accumulation of N per-lane FP32 amounts: each wave sums its
// lanes (wave_sum; a wave whose lanes all hold 0 skips it), thread 0 adds the
// waves' sums in wave order in FP64 and adds the nonzero totals to acc[0..N).
// Called by every thread of the block; sm holds (blockDim/64) * N doubles.
template <int N>
__device__ inline void tile_accumulate(const float (&v)[N], double *sm, double *acc)
{
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float w = __ballot(v[k] != 0.f) ? wave_sum(v[k]) : 0.f;
        if ((threadIdx.x & 63) == 0) sm[wave * N + k] = (double)w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double t = 0;
            for (int w = 0; w < nw; ++w) t += sm[w * N + k];
            if (t != 0.0) acc[k] += t;
        }
    }
    __syncthreads();
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
