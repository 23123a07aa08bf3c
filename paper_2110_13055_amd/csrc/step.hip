// step.hip -- the hot path: one lattice Boltzmann step (Eq. 7 with the BGK
// collision of Eq. 8, half-way bounce-back at solid faces) fused with one
// explicit finite-volume Nernst-Planck step (Eq. 3) and the adsorption flux
// of Eq. (6), over the compacted fluid nodes. The AA storage rules and the
// FP16 deviation format are described in device_common.h.
//
// The ions see the mass flux j = rho u. In a fused step the Nernst-Planck
// part reads the flux of the previous step (jin, or the FP16 moments) for the
// node and its face neighbours, while the LBM part writes the flux of this
// step. Face fluxes are Scharfetter-Gummel; the two sides of a face compute
// exactly opposite values, so solute is conserved to the rounding of the
// update. Per tile, the adsorbed / inflow / outflow amounts of the step are
// summed over each wave's 64 nodes in FP32, then over the tile's waves in
// FP64, in a fixed order, and added to that tile's own FP64 accumulator slot.
//
// Inlet/outlet planes (x = 0 and x = nx - 1): the node one plane inside owns
// the post-streaming populations the extrapolation needs, so its thread also
// advances the boundary node (no separate pass over the scattered planes).
#include "device_common.h"

namespace cdi {

namespace {

// Odd AA parity with FP32 or FP16 populations: the tile stages the slots of
// its own 256 nodes in LDS. Every slot has exactly one reader, which is also
// its writer (the AA rule above), so a slot whose reader lies in the tile is
// read from and written to LDS, and the owner loads it before and stores it
// after the step, both coalesced; a slot read by a node of another tile is
// left to that node's global load and store. Nodes of the inlet/outlet planes
// (advanced by their interior partner under extrapolation) write through
// global memory, so their slots are never stored back by an owner. On the
// 512^3 electrode about 29 % of the slots lie outside their reader's tile;
// staged, the FP32 fused odd step took 3.39 ms instead of 3.73, the FP32
// flow-only one 2.55 instead of 2.87, the FP16 fused one 2.76 instead of
// 2.87 (its flow-only step gains about 1 %).
// On lattices whose working set stays largely in the memory-side cache the
// extra work and barrier do not pay (96^3 to 160^3 electrodes stepped 5-13 %
// slower staged), so the host stages an instance's odd steps only from a
// tile count on (Grid::stage_odd); kStageOdd names the steps that may be
// staged.
//
// Stage layout: Q planes of kTile elements in the storage type, then kTile
// spare elements, one per thread. Every lane issues the LDS access (a lane
// whose slot lies outside the tile reads or writes its spare element) and
// only the global access is predicated; the stage is addressed through a
// pointer in the LDS address space, so that the compiler cannot fold an LDS
// and a global load into one generic-address access (which goes through the
// vector memory path and waits on both counters).
template <class L, int ST, int ODD, int LBM, int NP>
constexpr bool kStageOdd = LBM && ODD == 1 && (ST == kF32 || ST == kH16);

template <int ST>
using StageT = typename std::conditional<kHalfPop<ST>, uint16_t, float>::type;  // FP16 as its bits

typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
template <int ST>
using LdsT = typename std::conditional<kHalfPop<ST>, lds_u16, lds_f32>::type;

template <class L>
constexpr int kStageElems = (L::Q + 1) * kTile;

template <int ST>
__device__ __forceinline__ float pop_float(StageT<ST> v)
{
    if constexpr (kHalfPop<ST>) return __half2float(__ushort_as_half(v));
    else return v;
}

template <int ST>
__device__ __forceinline__ StageT<ST> pop_stored(float v)
{
    if constexpr (kHalfPop<ST>) return __half_as_ushort(__float2half_rn(v));
    else return v;
}

// Where incoming population i of node n (odd parity) is stored: plane pl of
// node nd; in: nd lies in the tile starting at base.
template <class L>
__device__ __forceinline__ bool staged_slot(const int *nb, int n, int i, int base, int &pl, uint32_t &loc)
{
    const int j = L::opp[i];
    const bool fl = (i != 0) && nb[j] >= 0;
    pl = fl ? j : i;
    loc = (uint32_t)((fl ? nb[j] : n) - base);
    return loc < (uint32_t)kTile;
}

// The stored values behind the Q incoming populations of node n (odd
// parity): all stage reads first, then the global loads of the slots outside
// the tile (into the same registers, for those lanes only), so that the
// stage reads are waited for once rather than before every global load.
template <class L, int ST>
__device__ __forceinline__ void staged_gather(const void *F, int P, const int *nb, int n, const LdsT<ST> *stage,
                                              int base, StageT<ST> (&raw)[L::Q])
{
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int pl;
        uint32_t loc;
        const bool in = staged_slot<L>(nb, n, i, base, pl, loc);
        raw[i] = stage[in ? pl * kTile + (int)loc : L::Q * kTile + (int)threadIdx.x];
    }
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        int pl;
        uint32_t loc;
        if (!staged_slot<L>(nb, n, i, base, pl, loc))  // a fluid emitter: plane opp(i) of it
            raw[i] = *pop_at<L::Q, StageT<ST>>(F, L::opp[i], nb[L::opp[i]]);
    }
}

// Store outgoing value v of direction i (odd parity); lds_ok false for the
// nodes whose slots go through global memory.
template <class L, int ST>
__device__ __forceinline__ void staged_scatter(void *F, int P, const int *nb, int n, int i, float v,
                                               LdsT<ST> *stage, int base, bool lds_ok)
{
    const int j = L::opp[i];
    const bool own = i == 0 || nb[i] < 0;
    const uint32_t loc = (uint32_t)((own ? n : nb[i]) - base);
    const bool in = lds_ok && loc < (uint32_t)kTile;
    stage[in ? (own ? j : i) * kTile + (int)loc : L::Q * kTile + (int)threadIdx.x] = pop_stored<ST>(v);
    if (!in) st_pair<kHalfPop<ST>, L::Q>(F, j, n, i, nb[i], own, v);
}

// Moments, residual terms, collision and the AA store of one node whose
// incoming populations (minus w_i) are f; NP: also store the mass flux j for
// the ions of the next step (FP32; the other storages carry it in Mout).
// FP32 storage: f_i - w_i (1 + pr.rout) on entry, and values stored relative
// to the plane references of pr (see PlaneRef); the other storages pass zeros.
template <class L, int ST, int ODD, int NP, bool STAGE = false>
__device__ __attribute__((always_inline)) inline void lbm_node(const Phys &p, const Bufs &b, int P, int n, const int *nb,
                                const float (&f)[L::Q], const PlaneRef &pr, double (&res)[2],
                                LdsT<ST> *stage = nullptr, int base = 0, bool lds_ok = false)
{
    constexpr int Q = L::Q, D = L::D;
    float drho, jx, jy, jz;  // drho: rho - 1 - pr.rout
    lat_moments<L>(f, drho, jx, jy, jz);
    if (p.forced) {  // Guo forcing: u = (sum e f + F/2) / rho
        jx += 0.5f * p.F[0];
        jy += 0.5f * p.F[1];
        jz += 0.5f * p.F[2];
    }
    const float rho = 1.f + pr.rout + drho;
    const float rinv = __builtin_amdgcn_rcpf(rho);
    const float ux = jx * rinv, uy = jy * rinv, uz = jz * rinv;
    if (b.flags & kResid) {
        float px, py, pz;
        if (!kPlain<ST>) {
            const float4 m = ldu(b.Min, (uint32_t)n);
            px = m.y;
            py = m.z;
            pz = m.w;
        } else {
            px = ldu(b.ubuf, (uint32_t)n);
            py = ldu(b.ubuf + P, (uint32_t)n);
            pz = D == 3 ? ldu(b.ubuf + 2 * (size_t)P, (uint32_t)n) : 0.f;
        }
        const double dx = (double)ux - px, dy = (double)uy - py, dz = (double)uz - pz;
        res[0] += dx * dx + dy * dy + dz * dz;
        res[1] += (double)ux * ux + (double)uy * uy + (double)uz * uz;
    }
    if (kPlain<ST> && (b.flags & kStoreU)) {
        stu(b.ubuf, (uint32_t)n, ux);
        stu(b.ubuf + P, (uint32_t)n, uy);
        if (D == 3) stu(b.ubuf + 2 * (size_t)P, (uint32_t)n, uz);
        stu(b.ubuf + (size_t)D * P, (uint32_t)n, pr.rout + drho);  // rho - 1, for the plane references
    }
    if (!kPlain<ST>) stu(b.Mout, (uint32_t)n, make_float4(drho, ux, uy, uz));
    if (NP && kPlain<ST>) {
        stu(b.jout, (uint32_t)n, jx);
        stu(b.jout + P, (uint32_t)n, jy);
        if (D == 3) stu(b.jout + 2 * (size_t)P, (uint32_t)n, jz);
    }
    if (ST == kMom) return;  // the post-collision state is the equilibrium of Mout
    const EqTerms eq = eq_terms(drho, rho, ux, uy, uz, p.linear_eq);
    const float om = p.omega;
    // FP16 populations are stored times hs
    const float sc = ST == kH16 ? p.hs : 1.f;
    if (kPlain<ST> && om == 1.f && !p.forced) {
        // tau = 1: BGK (Eq. 8) relaxes every population to the equilibrium
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float v = sc * stored_pop<L, ODD>(feq_dir<L>(i, eq, ux, uy, uz), i, nb, pr);
            if (STAGE)
                staged_scatter<L, ST>(b.f, P, nb, n, i, v, stage, base, lds_ok);
            else
                scatter<L, ST, ODD>(ODD == kPull ? b.f2 : b.f, P, nb, n, i, v);
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float fe = feq_dir<L>(i, eq, ux, uy, uz);
        float src = 0.f;
        if (p.forced) {  // Guo, Zheng & Shi (2002) source term
            const float eu = lat_dot<L>(i, ux, uy, uz);
            src = p.fcoef * L::w[i] *
                  ((3.f * (L::ex[i] - ux) + 9.f * eu * L::ex[i]) * p.F[0] +
                   (3.f * (L::ey[i] - uy) + 9.f * eu * L::ey[i]) * p.F[1] +
                   (3.f * (L::ez[i] - uz) + 9.f * eu * L::ez[i]) * p.F[2]);
        }
        float out;
        if (ST == kF16)
            out = ((1.f - om) * (f[i] - fe) + src) * p.hs;
        else
            out = sc * stored_pop<L, ODD>(f[i] - om * (f[i] - fe) + src, i, nb, pr);
        if (STAGE)
            staged_scatter<L, ST>(b.f, P, nb, n, i, out, stage, base, lds_ok);
        else
            scatter<L, ST, ODD>(ODD == kPull ? b.f2 : b.f, P, nb, n, i, out);
    }
}

// One 256-node tile of one instance (all threads of the workgroup call it;
// sm: (kTile/64)*6 doubles of LDS; stg: the stage of kStageOdd steps).
template <class L, int ST, int ODD, int LBM, int NP, int BATCH = 0, int STG = 0>
__device__ __attribute__((always_inline)) inline void step_tile(const Grid &g, const Phys &p, const Bufs &b, int tile, double *sm,
                                                             StageT<ST> *stage)
{
    constexpr int Q = L::Q, D = L::D;
    constexpr bool kStage = STG && kStageOdd<L, ST, ODD, LBM, NP>;
    LdsT<ST> *const stg = (LdsT<ST> *)stage;
    const int base = tile * kTile;
    const int n = tile * kTile + threadIdx.x;
    const bool active = n < g.n_f;
    const int P = g.P;
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    double res[2] = {0, 0};

    // coordinates and neighbour map values of the node
    int x = 0, y = 0, z = 0;
    int nb[Q];
    bool edge = false;
    // odd parity, staged: the node's own slots are loaded between its
    // coordinates and its neighbours' map values (the three in flight
    // together: each wait is for the earliest), and stored into the stage
    // after the lookups are issued
    StageT<ST> own[kStage ? Q : 1];
    if (active) {
        const uint32_t packed = ldu(g.fluid, (uint32_t)n);
        if constexpr (kStage) {
#pragma unroll
            for (int q = 0; q < Q; ++q) own[q] = *pop_at<Q, StageT<ST>>(b.f, q, n);
        }
        unpack_xyz(g, packed, x, y, z);
        constexpr bool need_all = LBM && (ODD || !kPlain<ST>);
        edge = LBM && g.inout && (b.flags & kNee) && (x <= 1 || x >= g.nx - 2);
        nb[0] = n;
        // the list, when the instance has one, for the steps that carry the ions
        // (measured on the 512^3 electrode: ion-only -6 %, fused moments -5 %,
        // FP16 deviations -3 %, FP16 populations -1.5 % AA / -5.5 % pull); the
        // fused FP32 step runs equally fast either way and moves 59 B/node less
        // without it, and flow-only steps stream their populations at the copy
        // rate already and only pay for the list's bytes (+10 %): those two
        // look their neighbours up
        constexpr bool kList = NP && !(LBM && ST == kF32);
        if (kList && g.nbr) {  // precomputed: independent of the coordinates
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const bool want = need_all || (NP && i <= 2 * D) || (edge && i <= 2);
                nb[i] = want ? ldu(g.nbr + (size_t)(i - 1) * P, (uint32_t)n) : kOutside;
            }
        } else {
            NbCtx ctx;
            nb_ctx<L>(g, x, y, z, g.periodic_x, ctx);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const bool want = need_all || (NP && i <= 2 * D) || (edge && i <= 2);
                nb[i] = want ? nb_get<L>(g, ctx, i) : kOutside;
            }
        }
        if constexpr (kStage) {
#pragma unroll
            for (int q = 0; q < Q; ++q) stg[q * kTile + threadIdx.x] = own[q];
        }
    }

    // Fused step, in this order: the ions' own and face-neighbour
    // concentrations (and with FP32 storage their mass fluxes) are loaded;
    // the flow's incoming populations are gathered; the ion update (which
    // needs only the previous step's flux) is computed and stored; then the
    // collision. The ions' loads overlap the flow's, and the ions' inputs
    // are dead before the collision's register peak. With FP16 and moment
    // storage the face neighbours' moments are loaded once for both parts
    // (the flow's emitters, the ions' mass flux). Measured on the 512^3
    // electrode against loading the ions' inputs after the flow's stores:
    // FP32 -16 %, moments -17 %, FP16 -16 % per fused step. An ion-only step
    // loads them the same way, all before its face loop, where a load inside
    // a divergent branch would wait for its data before the next face starts
    // (its flux is always the stored one): -27 % per ion-only step.
    constexpr bool kEarly = NP;
    constexpr bool kEarlyJ = kEarly && (kPlain<ST> || !LBM);
    // with a potential field, the neighbours' potential too, where the flux
    // is loaded early (ion-only step 1.18 -> 0.96 ms, FP32 fused 3.50 ->
    // 3.27 ms on the 512^3 electrode, same waves per SIMD); not in the
    // batched kernels, whose per-instance descriptor leaves no registers to
    // spare (their ion-only and FP16 / moment fused forms lose a wave per
    // SIMD, which costs the served requests, all in the ramp, 10 %)
    constexpr bool kEarlyPsi = kEarlyJ && !BATCH;
    float ec[2] = {0.f, 0.f}, ej[3] = {0.f, 0.f, 0.f};
    __half2 elo = __floats2half2_rn(0.f, 0.f);
    float ecn[2 * D][2], ejn[2 * D], epsi[2 * D];
    if (kEarly && active) {
        ec[0] = ldu(b.Cin, (uint32_t)n);
        ec[1] = ldu(b.Cin + P, (uint32_t)n);
        elo = ldu(b.Clin, (uint32_t)n);
        if (kEarlyJ) {
            ej[0] = ldu(b.jin, (uint32_t)n);
            ej[1] = ldu(b.jin + P, (uint32_t)n);
            ej[2] = D == 3 ? ldu(b.jin + 2 * (size_t)P, (uint32_t)n) : 0.f;
        }
#pragma unroll
        for (int k = 0; k < 2 * D; ++k) {
            const int m = nb[k + 1];
            const bool fl = m >= 0;
            ecn[k][0] = fl ? ldu(b.Cin, (uint32_t)m) : 0.f;
            ecn[k][1] = fl ? ldu(b.Cin + P, (uint32_t)m) : 0.f;
            ejn[k] = (fl && kEarlyJ) ? ldu(b.jin + (size_t)(k >> 1) * P, (uint32_t)m) : 0.f;
            epsi[k] = (kEarlyPsi && p.psi) ? ldu(p.psi, (uint32_t)(fl ? m : n)) : 0.f;
        }
    }
    if (kStage) __syncthreads();
    const bool nee = g.inout && (b.flags & kNee);
    // FP16 / moment storage, fused: the node's own and its face neighbours' moments
    float4 mface[2 * D], mown = make_float4(0.f, 0.f, 0.f, 0.f);
    bool have_m = false;

    // the flow's incoming populations (the collision follows the ions)
    float f[Q];
    bool do_flow = false;
    PlaneRef pr{0.f, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};  // FP32: the node's plane references
    {
        if (LBM && active) {
            // a boundary node with a fluid interior neighbour is advanced by that neighbour
            const bool by_partner = edge && ((x == 0 && nb[1] >= 0) || (x == g.nx - 1 && nb[2] >= 0));
            if (!by_partner) {
                do_flow = true;
                if (!kPlain<ST> && NP) {
#pragma unroll
                    for (int k = 0; k < 2 * D; ++k)
                        mface[k] = nb[k + 1] >= 0 ? ldu(b.Min, (uint32_t)nb[k + 1]) : make_float4(0.f, 0.f, 0.f, 0.f);
                    mown = ldu(b.Min, (uint32_t)n);
                    have_m = true;
                    // the incoming populations in groups of 6 directions: the
                    // group's edge emitters' moments are loaded together (the
                    // node's own where the emitter is solid, the same values as
                    // mown), then used; one at a time each load waited for its
                    // data before the next was issued. Measured on the 512^3
                    // electrode: moments 2.45 -> 2.01 ms, FP16 3.48 -> 3.25 ms
                    // per fused step (groups of 4: 2.10 / 3.38; of 10 the
                    // registers cost a wave per SIMD)
                    constexpr int kG = 6;
#pragma unroll
                    for (int i0 = 0; i0 < Q; i0 += kG) {
                        float4 mg[kG];
#pragma unroll
                        for (int u = 0; u < kG; ++u) {
                            const int i = i0 + u;
                            if (i >= Q) break;
                            const int j = L::opp[i];
                            const bool fl = (i != 0) && nb[j] >= 0;
                            if (i == 0)
                                mg[u] = mown;
                            else if (j <= 2 * D)
                                mg[u] = fl ? mface[j - 1] : mown;
                            else
                                mg[u] = ldu(b.Min, (uint32_t)(fl ? nb[j] : n));
                        }
#pragma unroll
                        for (int u = 0; u < kG; ++u) {
                            const int i = i0 + u;
                            if (i >= Q) break;
                            const int j = L::opp[i];
                            const bool fl = (i != 0) && nb[j] >= 0;
                            f[i] = from_emitter<L, ST>(gather_raw<L, ST, ODD>(b.f, P, nb, n, i), i, fl, mg[u], p);
                        }
                    }
                } else if (!kPlain<ST>) {
                    // flow only: all emitters' moments loaded first, then used
                    // (moments 1.73 -> 1.27 ms, FP16 3.08 -> 2.53 ms per flow
                    // step; groups of 6: 1.34 / 2.64)
                    constexpr int kG = Q;
#pragma unroll
                    for (int i0 = 0; i0 < Q; i0 += kG) {
                        float4 mg[kG];
#pragma unroll
                        for (int u = 0; u < kG; ++u) {
                            const int i = i0 + u;
                            if (i >= Q) break;
                            const int j = L::opp[i];
                            const bool fl = (i != 0) && nb[j] >= 0;
                            mg[u] = ldu(b.Min, (uint32_t)(fl ? nb[j] : n));
                        }
#pragma unroll
                        for (int u = 0; u < kG; ++u) {
                            const int i = i0 + u;
                            if (i >= Q) break;
                            const int j = L::opp[i];
                            const bool fl = (i != 0) && nb[j] >= 0;
                            f[i] = from_emitter<L, ST>(gather_raw<L, ST, ODD>(b.f, P, nb, n, i), i, fl, mg[u], p);
                        }
                    }
                } else {
                    pr = plane_ref<ODD>(g, b.rin, b.rout, x);
                    if (kStage) {
                        const float sc = ST == kH16 ? p.hs_inv : 1.f;
                        StageT<ST> raw[Q];
                        staged_gather<L, ST>(b.f, P, nb, n, stg, base, raw);
#pragma unroll
                        for (int i = 0; i < Q; ++i) f[i] = rel_pop<L, ODD>(sc * pop_float<ST>(raw[i]), i, nb, pr);
                    } else {
#pragma unroll
                        for (int i = 0; i < Q; ++i)
                            f[i] = rel_pop<L, ODD>(gather<L, ST, ODD>(b.f, P, nb, n, i, b.Min, p), i, nb, pr);
                    }
                }
            }
        }
    }

    // the ions: face fluxes of the explicit finite-volume update
    {
        if (NP && active) {
            const float cP[2] = {ec[0], ec[1]};
            float jP[3];
            const bool jm = !kPlain<ST> && (b.flags & kJFromM);
            if (jm) {
                const float4 m = have_m ? mown : ldu(b.Min, (uint32_t)n);
                const float r = 1.f + m.x;
                jP[0] = r * m.y;
                jP[1] = r * m.z;
                jP[2] = r * m.w;
            } else if (kEarlyJ) {
                jP[0] = ej[0];
                jP[1] = ej[1];
                jP[2] = ej[2];
            } else {
                jP[0] = ldu(b.jin, (uint32_t)n);
                jP[1] = ldu(b.jin + P, (uint32_t)n);
                jP[2] = D == 3 ? ldu(b.jin + 2 * (size_t)P, (uint32_t)n) : 0.f;
            }
            const float psiP = p.psi ? ldu(p.psi, (uint32_t)n) : 0.f;
            // per species: 2/D, and (z D)/2 so that half the drift is hw = u/2 - (z D/2) dpsi
            const float invD2[2] = {2.f * p.invD[0], 2.f * p.invD[1]};
            const float hzD[2] = {0.5f * p.z[0] * p.D[0], 0.5f * p.z[1] * p.D[1]};
            float out[2] = {0.f, 0.f}, fa[2] = {0.f, 0.f}, fi[2] = {0.f, 0.f}, fo[2] = {0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 2 * D; ++k) {
                const int i = k + 1;
                const int axis = k >> 1;
                const int sgi = (k & 1) ? -1 : 1;
                const float sg = (float)sgi;
                const bool xb = axis == 0 && (x + sgi < 0 || x + sgi >= g.nx);
                if (xb && p.npx != kNpxPeriodic) {
                    if (p.npx == kNpxClosed) continue;
                    const float dpsi = p.psi ? 0.f : -sg * p.dpsi_dx;
                    if (sgi < 0) {  // inlet face: ghost at c0, inflow u_in
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            const float hw = -0.5f * p.u_in - hzD[s] * dpsi;
                            const float F = sg_flux(p.D[s], invD2[s], hw, cP[s], p.c0);
                            out[s] += F;
                            fi[s] -= F;
                        }
                    } else {  // outlet face
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            const float hw = 0.5f * jP[0] - hzD[s] * dpsi;
                            float F;
                            if (p.npx == kNpxDirichlet) {
                                F = sg_flux(p.D[s], invD2[s], hw, cP[s], p.c_out);
                            } else {  // open: drift carries C_P out, or feed c0 in
                                const float w = 2.f * hw;
                                F = fmaxf(w, 0.f) * cP[s] + fminf(w, 0.f) * p.c0;
                            }
                            out[s] += F;
                            fo[s] += F;
                        }
                    }
                    continue;
                }
                int m = nb[i];
                const bool early = kEarly && !xb;  // the loaded neighbour (not a periodic re-lookup)
                if (xb) m = nb_map<L>(g, x, y, z, i, true);  // periodic ions, open flow
                if (m == kElectrode) {  // adsorbing face, Eq. (6)
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const float F = p.keff[s] * cP[s];
                        out[s] += F;
                        fa[s] += F;
                    }
                } else if (m >= 0) {
                    float jN;
                    if (jm) {
                        const float4 mm = (have_m && !xb) ? mface[k] : ldu(b.Min, (uint32_t)m);
                        jN = (1.f + mm.x) * (axis == 0 ? mm.y : (axis == 1 ? mm.z : mm.w));
                    } else {
                        jN = (early && kEarlyJ) ? ejn[k] : ldu(b.jin + (size_t)axis * P, (uint32_t)m);
                    }
                    // half the face-normal drift: advection by the mean flux of the
                    // two cells, migration down the potential difference
                    const float hun = 0.25f * (jP[axis] + jN) * sg;
                    const bool mig = p.psi || axis == 0;  // the ramp has no y/z gradient
                    const float dpsi = p.psi ? (kEarlyPsi && early ? epsi[k] : ldu(p.psi, (uint32_t)m)) - psiP
                                             : -sg * p.dpsi_dx;
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const float hw = mig ? hun - hzD[s] * dpsi : hun;
                        out[s] += sg_flux(p.D[s], invD2[s], hw, cP[s],
                                          early ? ecn[k][s] : ldu(b.Cin + (size_t)s * P, (uint32_t)m));
                    }
                }
                // inert wall: no flux
            }
            // forward Euler into value + remainder (see lo_encode)
            float e0, e1;
            stu(b.Cout, (uint32_t)n, two_sum(cP[0], lo_decode(__low2half(elo)) - p.dt * out[0], e0));
            stu(b.Cout + P, (uint32_t)n, two_sum(cP[1], lo_decode(__high2half(elo)) - p.dt * out[1], e1));
            stu(b.Clout, (uint32_t)n, __halves2half2(lo_encode(e0), lo_encode(e1)));
            acc[0] = p.dt * fa[0];
            acc[1] = p.dt * fa[1];
            acc[2] = p.dt * fi[0];
            acc[3] = p.dt * fi[1];
            acc[4] = p.dt * fo[0];
            acc[5] = p.dt * fo[1];
        }
    }

    // the flow: collide and stream (and the residual terms on request)
    if (LBM && do_flow) {
        lbm_node<L, ST, ODD, NP, kStage>(p, b, P, n, nb, f, pr, res, stg, base,
                                         !(nee && (x == 0 || x == g.nx - 1)));
        const bool inl = edge && x == 1 && nb[2] >= 0;
        const bool outl = edge && x == g.nx - 2 && nb[1] >= 0;
        if (inl || outl) {
            const int bn = inl ? nb[2] : nb[1];
            const int xb = inl ? 0 : g.nx - 1;
            int nbb[Q];
            nbb[0] = bn;
#pragma unroll
            for (int i = 1; i < Q; ++i) nbb[i] = nb_map<L>(g, xb, y, z, i, false);  // rare path
            float fb[Q];
            PlaneRef pb{0.f, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
            if (kPlain<ST>) pb = plane_ref<ODD>(g, b.rin, b.rout, xb);
            nee_populations<L>(p, inl, f, fb, pr.rout, pb.rout);
            lbm_node<L, ST, ODD, NP, kStage>(p, b, P, bn, nbb, fb, pb, res, stg, base, false);
        }
    }
    if (kStage) {
        // the owner stores back each slot whose reader (and writer) is in the
        // tile: node x - e_q for slot q when that voxel is fluid, else the node
        __syncthreads();
        if (active) {
            // all stage reads first, then the stores (one wait for the reads)
            StageT<ST> v[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) v[q] = stg[q * kTile + threadIdx.x];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int r = L::opp[q];
                const bool fl = q != 0 && nb[r] >= 0;
                const int c = fl ? nb[r] : n;
                const int xc = fl ? x - L::ex[q] : x;
                if ((uint32_t)(c - base) < (uint32_t)kTile && !(nee && (xc == 0 || xc == g.nx - 1)))
                    *pop_at<Q, StageT<ST>>(b.f, q, n) = v[q];
            }
        }
        if (BATCH) __syncthreads();  // a next tile's loads would reuse the stage
    }
    if (LBM && (b.flags & kResid)) {
        double s[2];
        block_sum<2>(res, sm, s);
        if (threadIdx.x == 0) {
            b.resid[2 * (size_t)tile] = s[0];
            b.resid[2 * (size_t)tile + 1] = s[1];
        }
        __syncthreads();
    }

    if (NP) tile_accumulate<6>(acc, sm, b.acc + (size_t)tile * 8);
}

template <class L, int ST, int ODD, int LBM, int NP, int STG>
__global__ __launch_bounds__(kTile) void step_kernel(Grid g, Phys p, Bufs b)
{
    __shared__ double sm[(kTile / 64) * 6];
    __shared__ StageT<ST> stage[STG ? kStageElems<L> : 1];
    extern __shared__ double lds_pad[];  // sized at launch: occupancy cap only
    (void)lds_pad;
    step_tile<L, ST, ODD, LBM, NP, 0, STG>(g, p, b, block_tile(g), sm, stage);
}

// A batch member's descriptor is read from memory, and a pointer read from
// memory is a generic address to the compiler: its accesses become flat
// instructions, which take the vector memory path and count on both wait
// counters. Read through the constant address space (the descriptors do not
// change during a launch), the pointers are known to address global memory
// and their accesses are global ones.
__device__ __forceinline__ void load_inst(const BatchInst *inst, int k, Grid &g, Phys &p, Bufs &b)
{
    g = inst[k].g;
    p = inst[k].p;
    b = inst[k].b;
    typedef const __attribute__((address_space(4))) BatchInst const_inst_t;
    const_inst_t &c = ((const_inst_t *)inst)[k];
    g.fluid = c.g.fluid;
    g.map = c.g.map;
    g.sched = c.g.sched;
    g.nbr = c.g.nbr;
    p.psi = c.p.psi;
    b.f = c.b.f;
    b.f2 = c.b.f2;
    b.Min = c.b.Min;
    b.Mout = c.b.Mout;
    b.jin = c.b.jin;
    b.jout = c.b.jout;
    b.Cin = c.b.Cin;
    b.Cout = c.b.Cout;
    b.Clin = c.b.Clin;
    b.Clout = c.b.Clout;
    b.acc = c.b.acc;
    b.resid = c.b.resid;
    b.ubuf = c.b.ubuf;
    b.rin = c.b.rin;
    b.rout = c.b.rout;
}

// Many instances in one persistent launch per step class (LBM parity and
// mode): workgroup w takes entries w, w + G, w + 2G, ... of the class's list
// of (instance, tile) pairs. Each instance carries its own lattice,
// parameters and buffers, so uneven sizes share the launch; the descriptor is
// copied once per tile into registers. Tile results do not depend on which
// workgroup computes them.
template <class L, int ST, int ODD, int LBM, int NP>
__global__ __launch_bounds__(kTile) void batch_kernel(const BatchInst *__restrict__ inst,
                                                      const int2 *__restrict__ tiles, int ntiles)
{
    __shared__ double sm[(kTile / 64) * 6];
    extern __shared__ double lds_pad[];
    (void)lds_pad;
    // workgroups are dealt round-robin over the 8 XCDs: each XCD takes one
    // contiguous eighth of the list, so neighbouring tiles share its L2
    const int G = (int)gridDim.x, w = (int)blockIdx.x;
    int lo = 0, hi = ntiles, first = w, stride = G;
    if (G >= 8) {
        const int x = w & 7;
        lo = (int)((int64_t)ntiles * x / 8);
        hi = (int)((int64_t)ntiles * (x + 1) / 8);
        first = lo + (w >> 3);
        stride = (G - x + 7) >> 3;
    }
    for (int q = first; q < hi; q += stride) {
        const int2 e = tiles[q];
        Grid g;
        Phys p;
        Bufs b;
        load_inst(inst, e.x, g, p, b);
        step_tile<L, ST, ODD, LBM, NP, 1>(g, p, b, e.y, sm, nullptr);  // not staged
    }
}

// Dynamic LDS of an occupancy cap (pad bytes beside the kernels' own small
// scratch), less what a staged odd step declares itself, so that the cap
// admits the same number of workgroups per CU for every step class.
template <class L, int ST, int STG>
size_t cap_lds(int pad)
{
    const size_t stage = STG ? sizeof(StageT<ST>) * kStageElems<L> : 0;
    return (size_t)pad > stage ? (size_t)pad - stage : 0;
}

template <class L, int ST>
void launch_batch_t(int cls, const BatchInst *inst, const int2 *tiles, int ntiles, int wg, int pad,
                    hipStream_t s)
{
    const size_t lds = (size_t)pad;
    constexpr int O1 = ST == kMom ? 0 : 1;      // moment storage has no AA parity
    constexpr int OP = ST == kMom ? 0 : kPull;  // nor streaming of populations
    switch (cls) {
    case kClassFlowEven: batch_kernel<L, ST, 0, 1, 0><<<wg, kTile, lds, s>>>(inst, tiles, ntiles); break;
    case kClassFlowOdd: batch_kernel<L, ST, O1, 1, 0><<<wg, kTile, lds, s>>>(inst, tiles, ntiles); break;
    case kClassFlowPull: batch_kernel<L, ST, OP, 1, 0><<<wg, kTile, lds, s>>>(inst, tiles, ntiles); break;
    case kClassFusedEven: batch_kernel<L, ST, 0, 1, 1><<<wg, kTile, lds, s>>>(inst, tiles, ntiles); break;
    case kClassFusedOdd: batch_kernel<L, ST, O1, 1, 1><<<wg, kTile, lds, s>>>(inst, tiles, ntiles); break;
    case kClassFusedPull: batch_kernel<L, ST, OP, 1, 1><<<wg, kTile, lds, s>>>(inst, tiles, ntiles); break;
    default: batch_kernel<L, kF32, 0, 0, 1><<<wg, kTile, lds, s>>>(inst, tiles, ntiles); break;
    }
}

template <class L, int ST, int ODD, int LBM, int NP>
void launch_t(const Grid &g, const Phys &p, const Bufs &b, hipStream_t s)
{
    const unsigned T = (unsigned)(g.P / kTile);
    if constexpr (kStageOdd<L, ST, ODD, LBM, NP>) {
        if (g.stage_odd) {
            step_kernel<L, ST, ODD, LBM, NP, 1><<<T, kTile, cap_lds<L, ST, 1>(g.lds_pad), s>>>(g, p, b);
            return;
        }
    }
    step_kernel<L, ST, ODD, LBM, NP, 0><<<T, kTile, (size_t)g.lds_pad, s>>>(g, p, b);
}

template <class L, int ST, int ODD>
void launch_mode(int lbm, int np, const Grid &g, const Phys &p, const Bufs &b, hipStream_t s)
{
    if (lbm && np)
        launch_t<L, ST, ODD, 1, 1>(g, p, b, s);
    else if (lbm)
        launch_t<L, ST, ODD, 1, 0>(g, p, b, s);
    else
        launch_t<L, kF32, 0, 0, 1>(g, p, b, s);
}

template <class L>
void launch_prec(int st, int odd, int lbm, int np, const Grid &g, const Phys &p, const Bufs &b,
                 hipStream_t s)
{
    if (st == kMom) {
        launch_mode<L, kMom, 0>(lbm, np, g, p, b, s);
    } else if (st == kH16) {
        if (odd == kPull)
            launch_mode<L, kH16, kPull>(lbm, np, g, p, b, s);
        else if (odd)
            launch_mode<L, kH16, 1>(lbm, np, g, p, b, s);
        else
            launch_mode<L, kH16, 0>(lbm, np, g, p, b, s);
    } else if (st == kF16) {
        if (odd == kPull)
            launch_mode<L, kF16, kPull>(lbm, np, g, p, b, s);
        else if (odd)
            launch_mode<L, kF16, 1>(lbm, np, g, p, b, s);
        else
            launch_mode<L, kF16, 0>(lbm, np, g, p, b, s);
    } else {
        if (odd == kPull)
            launch_mode<L, kF32, kPull>(lbm, np, g, p, b, s);
        else if (odd)
            launch_mode<L, kF32, 1>(lbm, np, g, p, b, s);
        else
            launch_mode<L, kF32, 0>(lbm, np, g, p, b, s);
    }
}

template <class L>
void launch_batch_l(int st, int cls, const BatchInst *inst, const int2 *tiles, int ntiles, int wg, int pad,
                    hipStream_t s)
{
    if (st == kMom)
        launch_batch_t<L, kMom>(cls, inst, tiles, ntiles, wg, pad, s);
    else if (st == kH16)
        launch_batch_t<L, kH16>(cls, inst, tiles, ntiles, wg, pad, s);
    else if (st == kF16)
        launch_batch_t<L, kF16>(cls, inst, tiles, ntiles, wg, pad, s);
    else
        launch_batch_t<L, kF32>(cls, inst, tiles, ntiles, wg, pad, s);
}

}  // namespace

hipError_t launch_batch(int dim, int st, int cls, const BatchInst *inst, const int2 *tiles, int ntiles,
                        int workgroups, int lds_pad, hipStream_t s)
{
    if (ntiles <= 0 || workgroups <= 0) return hipSuccess;
    if (cls < 0 || cls >= kClasses || st < kF32 || st > kH16) return hipErrorInvalidValue;
    if (dim == 2)
        launch_batch_l<D2Q9>(st, cls, inst, tiles, ntiles, workgroups, lds_pad, s);
    else
        launch_batch_l<D3Q19>(st, cls, inst, tiles, ntiles, workgroups, lds_pad, s);
    return hipGetLastError();
}

hipError_t launch_step(int dim, int st, int odd, int lbm, int np, const Grid &g, const Phys &p,
                       const Bufs &b, hipStream_t s)
{
    if (g.P <= 0) return hipSuccess;
    if (st < kF32 || st > kH16) return hipErrorInvalidValue;
    if (dim == 2)
        launch_prec<D2Q9>(st, odd, lbm, np, g, p, b, s);
    else
        launch_prec<D3Q19>(st, odd, lbm, np, g, p, b, s);
    return hipGetLastError();
}

}  // namespace cdi
