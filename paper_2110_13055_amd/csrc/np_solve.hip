// np_solve.hip -- implicit ion transport: backward-Euler steps and the steady
// state of the Nernst-Planck equations, Eq. (3), with the adsorption law of
// Eq. (6), for a frozen flow and potential (the paper discretises Eq. 3 with
// an implicit finite-volume method, Sec. 2).
//
// The cell balance is the explicit step's: Scharfetter-Gummel face fluxes
// F = alpha C_P - beta C_N with alpha = D Bs(Pe) + w/2, beta = D Bs(Pe) -
// w/2 (w the face-normal drift, Bs(x) = (x/2) coth(x/2)), k_eff C_P on
// electrode faces, the inlet ghost at c0, the open or Dirichlet outlet. The
// coefficients are evaluated in FP32 exactly as the explicit step does; the
// operator is applied in FP64. For species s the outflow is A_s C - b_s; a
// backward-Euler step solves (I/dt + A_s) C' = C/dt + b_s and the steady
// state A_s C = b_s, both by BiCGSTAB (van der Vorst 1992) with the diagonal
// as right preconditioner, both species in the same kernels with their own
// scalars. Persistent workgroups and fixed-order partial sums as in pot.hip:
// every workgroup derives the same scalars, and the iterate does not depend
// on timing or on how often the host checks.
//
// Iteration k (species s, K = diag). The directions are stored
// preconditioned, p^ = K^-1 p and s^ = K^-1 s, so that the operator gathers
// no diagonals (measured on the 512^3 electrode, together with issuing every
// load of a node before its per-face branches: 7.33 -> 5.89 ms per iteration):
//   dir     stop test on |r_k|; beta = (rho_k / rho_{k-1}) (alpha / omega);
//           p^ = K^-1 (r - beta omega v) + beta p^
//   apply   v = A p^; partial rhat . v
//   sdir    alpha = rho_k / (rhat . v); s^ = K^-1 (r - alpha v)
//   apply   t = A s^; partials t . s (s = K s^), t . t
//   update  omega = (t . s) / (t . t); x += alpha p^ + omega s^;
//           r = K s^ - omega t; partials rho_{k+1} = rhat . r, |r|^2
// A species whose residual met the tolerance is frozen (its partials stop
// changing, so every later test repeats the decision).
#include "cdi_internal.h"
#include "device_common.h"
#include "np_solve_internal.h"
#include "reduce_common.h"

namespace cdi {

namespace {

// Partial-sum regions, 2 species x G doubles each.
enum { kRv = 0, kTs = 1, kTt = 2, kRho0 = 3, kRho1 = 4, kRr = 5, kBb = 6, kRegions = 7 };

__device__ inline double *reg(const NpsArgs &a, int r, int s) { return a.part + ((size_t)r * 2 + s) * gridDim.x; }

// alpha, beta of a face from the half drift hw (the explicit step's Bs).
__device__ inline void sg_coef(float D, float invD2, float hw, float &al, float &be)
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
    const float db = D * bs;
    al = db + hw;
    be = db - hw;
}

// Faces of node n: neighbour map values, and per species the coefficient of
// the node's own concentration (al) and either the neighbour's (be, fluid
// faces) or the ghost's constant term (be, open x-end faces), so that a
// face's outflow is al C_P - be C_N or al C_P - be; b = the sum of the ghost
// terms (the constant inflow); diag = sum of al.
template <class L>
struct NpNode {
    int m[2 * L::D];
    float al[2][2 * L::D], be[2][2 * L::D];
    double b[2];
    float diag[2];
};

template <class L>
__device__ inline void np_node(const Grid &g, const Phys &p, const float *j, int n, NpNode<L> &c)
{
    constexpr int D = L::D;
    const int P = g.P;
    // every load is issued before the per-face branches (a load inside a
    // divergent branch waits for its data before the next face starts): the
    // six neighbours, then the flux (and potential) of each, at the node
    // itself where the face is not fluid. The neighbours come from the list
    // when the instance has one built with the ions' x periodicity (read
    // with the node's data), else through the coordinates and the map.
    if (g.nbr && (p.npx == kNpxPeriodic) == (g.periodic_x != 0)) {
#pragma unroll
        for (int k = 0; k < 2 * D; ++k) c.m[k] = ldu(g.nbr + (size_t)k * P, (uint32_t)n);
    } else {
        int x, y, z;
        unpack_xyz(g, ldu(g.fluid, (uint32_t)n), x, y, z);
        NbCtx ctx;
        nb_ctx<L>(g, x, y, z, p.npx == kNpxPeriodic, ctx);
#pragma unroll
        for (int k = 0; k < 2 * D; ++k) c.m[k] = nb_get<L>(g, ctx, k + 1);
    }
    float jP[3], jN[2 * D], psiN[2 * D];
    jP[0] = ldu(j, (uint32_t)n);
    jP[1] = ldu(j + P, (uint32_t)n);
    jP[2] = D == 3 ? ldu(j + (size_t)2 * P, (uint32_t)n) : 0.f;
    const float psiP = p.psi ? ldu(p.psi, (uint32_t)n) : 0.f;
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        const uint32_t q = (uint32_t)(c.m[k] >= 0 ? c.m[k] : n);
        jN[k] = ldu(j + (size_t)(k >> 1) * P, q);
        psiN[k] = p.psi ? ldu(p.psi, q) : 0.f;
    }
    const float invD2[2] = {2.f * p.invD[0], 2.f * p.invD[1]};
    const float hzD[2] = {0.5f * p.z[0] * p.D[0], 0.5f * p.z[1] * p.D[1]};
    c.b[0] = c.b[1] = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        const int i = k + 1;
        const int axis = k >> 1;
        const int sgi = (k & 1) ? -1 : 1;
        const float sg = (float)sgi;
        const int m = c.m[k];
#pragma unroll
        for (int s = 0; s < 2; ++s) c.al[s][k] = c.be[s][k] = 0.f;
        if (m == kOutside) {  // an open x end (the ions are not periodic)
            if (p.npx == kNpxClosed) continue;
            const float dpsi = p.psi ? 0.f : -sg * p.dpsi_dx;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                float al, be;
                if (sgi < 0) {  // inlet: ghost at c0, inflow u_in
                    sg_coef(p.D[s], invD2[s], -0.5f * p.u_in - hzD[s] * dpsi, al, be);
                    be *= p.c0;
                } else if (p.npx == kNpxDirichlet) {
                    sg_coef(p.D[s], invD2[s], 0.5f * jP[0] - hzD[s] * dpsi, al, be);
                    be *= p.c_out;
                } else {  // open outlet: drift carries C_P out, or feed c0 in
                    const float w = 2.f * (0.5f * jP[0] - hzD[s] * dpsi);
                    al = fmaxf(w, 0.f);
                    be = -fminf(w, 0.f) * p.c0;
                }
                c.al[s][k] = al;
                c.be[s][k] = be;
                c.b[s] += (double)be;
            }
        } else if (m == kElectrode) {
#pragma unroll
            for (int s = 0; s < 2; ++s) c.al[s][k] = p.keff[s];
        } else if (m >= 0) {
            const float hun = 0.25f * (jP[axis] + jN[k]) * sg;
            const bool mig = p.psi || axis == 0;  // the ramp has no y/z gradient
            const float dpsi = p.psi ? psiN[k] - psiP : -sg * p.dpsi_dx;
#pragma unroll
            for (int s = 0; s < 2; ++s) sg_coef(p.D[s], invD2[s], mig ? hun - hzD[s] * dpsi : hun, c.al[s][k], c.be[s][k]);
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        float d = 0.f;
#pragma unroll
        for (int k = 0; k < 2 * D; ++k) d += c.al[s][k];
        c.diag[s] = d;
    }
}

template <class L>
__global__ __launch_bounds__(kTile) void nps_setup_kernel(NpsArgs a)
{
    __shared__ double sm[kTile / 64];
    int t0, t1;
    tile_range(a.g.P / kTile, t0, t1);
    const int P = a.g.P;
    double bb[2] = {0, 0}, rho[2] = {0, 0}, rr[2] = {0, 0};
    for (int t = t0; t < t1; ++t) {
        const int n = t * kTile + threadIdx.x;
        double xv[2] = {0, 0}, rv[2] = {0, 0};
        float dv[2] = {1.f, 1.f};
        if (n < a.g.n_f) {
            NpNode<L> c;
            np_node<L>(a.g, a.p, a.j, n, c);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                xv[s] = a.C[s * P + n];
                double ax = (c.diag[s] + a.idt) * xv[s];
#pragma unroll
                for (int k = 0; k < 2 * L::D; ++k)
                    if (c.m[k] >= 0) ax -= (double)c.be[s][k] * a.C[s * P + c.m[k]];
                const double rhs = a.idt * xv[s] + c.b[s];
                rv[s] = rhs - ax;
                dv[s] = (float)(c.diag[s] + a.idt);
                if (!(dv[s] > 0.f)) dv[s] = 1.f;  // a cell with no outflow at all (an isolated closed pocket)
                bb[s] += rhs * rhs;
                rho[s] += rv[s] * rv[s];
                rr[s] += rv[s] * rv[s];
            }
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            stu(a.x, (uint32_t)(s * P + n), xv[s]);
            stu(a.r, (uint32_t)(s * P + n), rv[s]);
            stu(a.rh, (uint32_t)(s * P + n), rv[s]);
            stu(a.pv, (uint32_t)(s * P + n), 0.0);
            stu(a.v, (uint32_t)(s * P + n), 0.0);
            stu(a.dg, (uint32_t)(s * P + n), dv[s]);
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double s_bb = wg_sum(bb[s], sm), s_rho = wg_sum(rho[s], sm), s_rr = wg_sum(rr[s], sm);
        if (threadIdx.x == 0) {
            reg(a, kBb, s)[blockIdx.x] = s_bb;
            reg(a, kRho0, s)[blockIdx.x] = s_rho;
            reg(a, kRr, s)[blockIdx.x] = s_rr;
            // iteration -1 leaves alpha = omega = 1: r.v = rho_0, t.s = t.t = 1
            reg(a, kRv, s)[blockIdx.x] = s_rho;
            reg(a, kTs, s)[blockIdx.x] = blockIdx.x == 0 ? 1.0 : 0.0;
            reg(a, kTt, s)[blockIdx.x] = blockIdx.x == 0 ? 1.0 : 0.0;
        }
    }
}

// Per-species stop decision from the |r|^2 partials (the same in every workgroup).
__device__ inline void species_active(const NpsArgs &a, double *sm, bool (&act)[2], double (&rr)[2])
{
    const int G = gridDim.x;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        rr[s] = region_sum(reg(a, kRr, s), G, sm);
        act[s] = !(rr[s] <= a.state[kNsThr + s]);
    }
}

__global__ __launch_bounds__(kTile) void nps_state_kernel(NpsArgs a, int G, double tol)
{
    __shared__ double sm[kTile / 64];
    for (int s = 0; s < 2; ++s) {
        const double bb = region_sum(a.part + ((size_t)kBb * 2 + s) * G, G, sm);
        const double rr = region_sum(a.part + ((size_t)kRr * 2 + s) * G, G, sm);
        if (threadIdx.x == 0) {
            a.state[kNsBb + s] = bb;
            a.state[kNsThr + s] = tol * tol * bb;
            a.state[kNsRr + s] = rr;
            a.state[kNsIters + s] = 0;
            a.state[kNsActive + s] = rr <= tol * tol * bb ? 0.0 : 1.0;
        }
    }
    if (threadIdx.x == 0) a.state[kNsDone] = (a.state[kNsActive] == 0 && a.state[kNsActive + 1] == 0) ? 1.0 : 0.0;
}

// dir: stop test and the new direction.
__global__ __launch_bounds__(kTile) void nps_dir_kernel(NpsArgs a, int k)
{
    __shared__ double sm[kTile / 64];
    __shared__ int stop;
    if (stopped_at(a.state, kNsDone, &stop)) return;
    const int G = gridDim.x;
    bool act[2];
    double rr[2];
    species_active(a, sm, act, rr);
    double beta[2] = {0, 0}, omega[2] = {1, 1};
    bool bad = false;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double rho_new = region_sum(reg(a, k & 1 ? kRho1 : kRho0, s), G, sm);
        const double rho_old = region_sum(reg(a, k & 1 ? kRho0 : kRho1, s), G, sm);
        const double rv = region_sum(reg(a, kRv, s), G, sm);
        const double ts = region_sum(reg(a, kTs, s), G, sm), tt = region_sum(reg(a, kTt, s), G, sm);
        if (k == 0) continue;  // p = r
        const double alpha = rho_old / rv;
        omega[s] = ts / tt;
        beta[s] = (rho_new / rho_old) * (alpha / omega[s]);
        if (act[s] && !(isfinite(beta[s]) && isfinite(rr[s]))) bad = true;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int s = 0; s < 2; ++s) {
            a.state[kNsActive + s] = act[s] ? 1.0 : 0.0;
            a.state[kNsRr + s] = rr[s];
            if (act[s]) a.state[kNsIters + s] = k;
        }
        if (bad) a.state[kNsDone] = 2.0;
        else if (!act[0] && !act[1]) a.state[kNsDone] = 1.0;
    }
    if (bad || (!act[0] && !act[1])) return;
    int t0, t1;
    tile_range(a.g.P / kTile, t0, t1);
    const int P = a.g.P;
    for (int t = t0; t < t1; ++t) {
        const int n = t * kTile + threadIdx.x;
        if (n >= a.g.n_f) continue;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!act[s]) continue;
            const uint32_t q = (uint32_t)(s * P + n);
            const double d = (double)ldu(a.dg, q);
            const double pn = k == 0 ? ldu(a.r, q) / d
                                     : (ldu(a.r, q) - beta[s] * omega[s] * ldu(a.v, q)) / d + beta[s] * ldu(a.pv, q);
            stu(a.pv, q, pn);
        }
    }
}

// y = (idt I + A) in for the active species (in = p^ or s^, already
// preconditioned), with partials: WHICH 0 (y = v): rhat . v; WHICH 1 (y = t):
// t . s with s = K s^, t . t.
template <class L, int WHICH>
__global__ __launch_bounds__(kTile) void nps_apply_kernel(NpsArgs a)
{
    __shared__ double sm[kTile / 64];
    __shared__ int stop;
    if (stopped_at(a.state, kNsDone, &stop)) return;
    const bool act[2] = {a.state[kNsActive] != 0.0, a.state[kNsActive + 1] != 0.0};
    const double *in = WHICH == 0 ? a.pv : a.sv;
    double *out = WHICH == 0 ? a.v : a.t;
    int t0, t1;
    tile_range(a.g.P / kTile, t0, t1);
    const int P = a.g.P;
    double d0[2] = {0, 0}, d1[2] = {0, 0};
    for (int t = t0; t < t1; ++t) {
        const int n = t * kTile + threadIdx.x;
        if (n >= a.g.n_f) continue;
        NpNode<L> c;
        np_node<L>(a.g, a.p, a.j, n, c);
        // both species' neighbour values (stored preconditioned), all
        // gathered before any is used (the node's own where the face is not
        // fluid; not applied there)
        double vN[2][2 * L::D], vP[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int f = 0; f < 2 * L::D; ++f)
                vN[s][f] = ldu(in, (uint32_t)(s * P + (c.m[f] >= 0 ? c.m[f] : n)));
            vP[s] = ldu(in, (uint32_t)(s * P + n));
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!act[s]) continue;
            const uint32_t q = (uint32_t)(s * P + n);
            const double yP = vP[s];
            double y = ((double)c.diag[s] + a.idt) * yP;
#pragma unroll
            for (int f = 0; f < 2 * L::D; ++f)
                if (c.m[f] >= 0) y -= (double)c.be[s][f] * vN[s][f];
            stu(out, q, y);
            if (WHICH == 0) {
                d0[s] += ldu(a.rh, q) * y;
            } else {
                d0[s] += y * (yP * (double)ldu(a.dg, q));
                d1[s] += y * y;
            }
        }
    }
    const int G = gridDim.x;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        if (!act[s]) continue;  // a frozen species keeps its last partials
        const double s0 = wg_sum(d0[s], sm);
        const double s1 = WHICH == 1 ? wg_sum(d1[s], sm) : 0.0;
        if (threadIdx.x == 0) {
            if (WHICH == 0) {
                a.part[((size_t)kRv * 2 + s) * G + blockIdx.x] = s0;
            } else {
                a.part[((size_t)kTs * 2 + s) * G + blockIdx.x] = s0;
                a.part[((size_t)kTt * 2 + s) * G + blockIdx.x] = s1;
            }
        }
    }
}

// s^ = K^-1 (r - alpha v)
__global__ __launch_bounds__(kTile) void nps_sdir_kernel(NpsArgs a, int k)
{
    __shared__ double sm[kTile / 64];
    __shared__ int stop;
    if (stopped_at(a.state, kNsDone, &stop)) return;
    const bool act[2] = {a.state[kNsActive] != 0.0, a.state[kNsActive + 1] != 0.0};
    const int G = gridDim.x;
    double alpha[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
        alpha[s] = region_sum(reg(a, k & 1 ? kRho1 : kRho0, s), G, sm) / region_sum(reg(a, kRv, s), G, sm);
    int t0, t1;
    tile_range(a.g.P / kTile, t0, t1);
    const int P = a.g.P;
    for (int t = t0; t < t1; ++t) {
        const int n = t * kTile + threadIdx.x;
        if (n >= a.g.n_f) continue;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!act[s]) continue;
            const uint32_t q = (uint32_t)(s * P + n);
            stu(a.sv, q, (ldu(a.r, q) - alpha[s] * ldu(a.v, q)) / (double)ldu(a.dg, q));
        }
    }
}

// x += alpha p^ + omega s^; r = K s^ - omega t; partials rho_{k+1}, |r|^2
__global__ __launch_bounds__(kTile) void nps_update_kernel(NpsArgs a, int k)
{
    __shared__ double sm[kTile / 64];
    __shared__ int stop;
    if (stopped_at(a.state, kNsDone, &stop)) return;
    const bool act[2] = {a.state[kNsActive] != 0.0, a.state[kNsActive + 1] != 0.0};
    const int G = gridDim.x;
    double alpha[2], omega[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        alpha[s] = region_sum(reg(a, k & 1 ? kRho1 : kRho0, s), G, sm) / region_sum(reg(a, kRv, s), G, sm);
        omega[s] = region_sum(reg(a, kTs, s), G, sm) / region_sum(reg(a, kTt, s), G, sm);
    }
    int t0, t1;
    tile_range(a.g.P / kTile, t0, t1);
    const int P = a.g.P;
    double rho[2] = {0, 0}, rr[2] = {0, 0};
    for (int t = t0; t < t1; ++t) {
        const int n = t * kTile + threadIdx.x;
        if (n >= a.g.n_f) continue;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!act[s]) continue;
            const uint32_t q = (uint32_t)(s * P + n);
            const double sh = ldu(a.sv, q);
            stu(a.x, q, ldu(a.x, q) + alpha[s] * ldu(a.pv, q) + omega[s] * sh);
            const double rn = sh * (double)ldu(a.dg, q) - omega[s] * ldu(a.t, q);
            stu(a.r, q, rn);
            rho[s] += ldu(a.rh, q) * rn;
            rr[s] += rn * rn;
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        if (!act[s]) continue;
        const double s_rho = wg_sum(rho[s], sm), s_rr = wg_sum(rr[s], sm);
        if (threadIdx.x == 0) {
            a.part[((size_t)(k & 1 ? kRho0 : kRho1) * 2 + s) * G + blockIdx.x] = s_rho;
            a.part[((size_t)kRr * 2 + s) * G + blockIdx.x] = s_rr;
        }
    }
}

// The stop test before iteration k, alone (one workgroup).
__global__ __launch_bounds__(kTile) void nps_check_kernel(NpsArgs a, int k, int G)
{
    __shared__ double sm[kTile / 64];
    if (a.state[kNsDone] != 0.0) return;
    bool act[2];
    for (int s = 0; s < 2; ++s) {
        const double rr = region_sum(a.part + ((size_t)kRr * 2 + s) * G, G, sm);
        act[s] = !(rr <= a.state[kNsThr + s]);
        if (threadIdx.x == 0) {
            if (!isfinite(rr)) a.state[kNsDone] = 2.0;
            a.state[kNsRr + s] = rr;
            if (act[s]) a.state[kNsIters + s] = k;
        }
    }
    if (threadIdx.x == 0 && a.state[kNsDone] == 0.0 && !act[0] && !act[1]) a.state[kNsDone] = 1.0;
}

// The FP64 solution as FP32 concentrations with their remainders.
__global__ __launch_bounds__(kTile) void nps_store_kernel(const double *x, float *C, __half2 *Clo, int P, int n_f)
{
    const int n = blockIdx.x * kTile + threadIdx.x;
    if (n >= n_f) return;
    const float c0 = (float)x[n], c1 = (float)x[P + n];
    C[n] = c0;
    C[P + n] = c1;
    Clo[n] = __halves2half2(lo_encode((float)(x[n] - c0)), lo_encode((float)(x[P + n] - c1)));
}

// Rates of adsorption, inflow and outflow of C (per tile, FP64).
template <class L>
__global__ __launch_bounds__(kTile) void nps_rates_kernel(Grid g, Phys p, const float *C, const float *j, double scale,
                                                          double *acc, double *part)
{
    __shared__ double sm[(kTile / 64) * 6];
    const int tile = blockIdx.x;
    const int n = tile * kTile + threadIdx.x;
    const int P = g.P;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (n < g.n_f) {
        NpNode<L> c;
        np_node<L>(g, p, j, n, c);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double cp = C[s * P + n];
#pragma unroll
            for (int f = 0; f < 2 * L::D; ++f) {
                const int m = c.m[f];
                if (m == kElectrode) {
                    v[s] += (double)c.al[s][f] * cp;  // adsorbed
                } else if (m == kOutside) {
                    const double F = (double)c.al[s][f] * cp - (double)c.be[s][f];
                    if (f & 1)
                        v[2 + s] -= F;  // the -x face is the inlet: inflow
                    else
                        v[4 + s] += F;  // outflow
                }
            }
        }
    }
    double out[6];
    block_sum<6>(v, sm, out);
    if (threadIdx.x == 0) {
        if (acc) {
            double *a = acc + (size_t)tile * 8;
            for (int k = 0; k < 6; ++k) a[k] += scale * out[k];
        } else {
            for (int k = 0; k < 6; ++k) part[(size_t)tile * 6 + k] = out[k];
        }
    }
}

}  // namespace

uint64_t nps_part_doubles() { return (uint64_t)kRegions * 2 * kNpsMaxWorkgroups; }

hipError_t nps_workgroups(int dim, int ntiles, int *G)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const void *k = dim == 2 ? (const void *)nps_apply_kernel<D2Q9, 1> : (const void *)nps_apply_kernel<D3Q19, 1>;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kTile, 0);
    if (e != hipSuccess) return e;
    // at most 4 per CU (measured on the 512^3 electrode: 5.68 ms per
    // iteration at 4, 5.90 at the occupancy limit of 5, 6.05 at 3): fewer
    // tiles in flight per XCD leave more of its L2 to the neighbours' lines
    if (per_cu > kNpsWorkgroupsPerCU) per_cu = kNpsWorkgroupsPerCU;
    long long g = (long long)cus * (per_cu > 0 ? per_cu : 1);
    g = g < kNpsMaxWorkgroups ? g : kNpsMaxWorkgroups;
    *G = (int)(ntiles < g ? ntiles : g);
    return hipSuccess;
}

hipError_t launch_nps_setup(int dim, const NpsArgs &a, int G, double tol, hipStream_t s)
{
    if (dim == 2)
        nps_setup_kernel<D2Q9><<<G, kTile, 0, s>>>(a);
    else
        nps_setup_kernel<D3Q19><<<G, kTile, 0, s>>>(a);
    nps_state_kernel<<<1, kTile, 0, s>>>(a, G, tol);
    return hipGetLastError();
}

hipError_t launch_nps_iter(int dim, const NpsArgs &a, int G, int k, hipStream_t s)
{
    nps_dir_kernel<<<G, kTile, 0, s>>>(a, k);
    if (dim == 2)
        nps_apply_kernel<D2Q9, 0><<<G, kTile, 0, s>>>(a);
    else
        nps_apply_kernel<D3Q19, 0><<<G, kTile, 0, s>>>(a);
    nps_sdir_kernel<<<G, kTile, 0, s>>>(a, k);
    if (dim == 2)
        nps_apply_kernel<D2Q9, 1><<<G, kTile, 0, s>>>(a);
    else
        nps_apply_kernel<D3Q19, 1><<<G, kTile, 0, s>>>(a);
    nps_update_kernel<<<G, kTile, 0, s>>>(a, k);
    return hipGetLastError();
}

hipError_t launch_nps_check(const NpsArgs &a, int G, int k, hipStream_t s)
{
    nps_check_kernel<<<1, kTile, 0, s>>>(a, k, G);
    return hipGetLastError();
}

hipError_t launch_nps_store(const NpsArgs &a, float *Cout, __half2 *Clo, hipStream_t s)
{
    const int tiles = a.g.P / kTile;
    if (tiles > 0) nps_store_kernel<<<tiles, kTile, 0, s>>>(a.x, Cout, Clo, a.g.P, a.g.n_f);
    return hipGetLastError();
}

hipError_t launch_nps_rates(int dim, const Grid &g, const Phys &p, const float *C, const float *j, double scale,
                            double *acc, double *part, double *out, hipStream_t s)
{
    const int tiles = g.P / kTile;
    if (tiles == 0) return hipSuccess;
    if (dim == 2)
        nps_rates_kernel<D2Q9><<<tiles, kTile, 0, s>>>(g, p, C, j, scale, acc, part);
    else
        nps_rates_kernel<D3Q19><<<tiles, kTile, 0, s>>>(g, p, C, j, scale, acc, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !out) return e;
    return launch_reduce_tiles(part, tiles, 6, 6, out, s);
}

}  // namespace cdi
