// pot.hip -- the electric potential of Poisson's equation, Eq. (4), with the
// charge density of Eq. (5) and the electrode's Dirichlet value (Sec. 2),
// solved on the compacted fluid lattice by Jacobi-preconditioned conjugate
// gradients inside mixed-precision iterative refinement: the iterate x and
// each round's residual b - A x are FP64, each round's correction solve runs
// CG on FP32 vectors (dot products and alpha, beta in FP64), and a round that
// no longer gains hands over to CG on the FP64 vectors.
//
// Discretisation (finite volumes, one unknown per fluid cell centre, psi in
// thermal voltages): a face between two fluid cells carries psi_N - psi_P; a
// face on an electrode voxel carries 2 (psi_e - psi_P) (the Dirichlet value
// sits on the face, half a cell away); an inert face carries nothing; an x
// end face is Dirichlet (value psi_x), field-free, or periodic. A cell
// balances its face fluxes against the charge term src * sum_i z_i C_i, src =
// kappa2 / (2 c0). As A psi = b: A_PP = number of fluid faces + 2 per
// Dirichlet face, A_PN = -1 per fluid face, b_P = src sum z C + 2 sum psi_face.
//
// The CG vectors are in internal node order (stride P). Every kernel
// runs G persistent workgroups; workgroup c (its XCD-contiguous position)
// owns the contiguous tile range [c T / G, (c + 1) T / G), so an XCD sweeps
// one contiguous eighth of the lattice and finds the tiles above and below
// in its own L2. A dot product is one FP64 partial per workgroup; the kernel
// that needs the total sums the G partials itself, in a fixed order, so
// every workgroup derives the same alpha and beta and the result does not
// depend on timing. Iteration k runs two kernels:
//   dirspmv  stop when |r_k| <= tol |b|; else beta = rz_k / rz_{k-1},
//            p_k = z_k + beta p_{k-1} (z = r / diag), q = A p_k, partial p.q
//   axpy     alpha = rz_k / p.q; x += alpha p_k; r -= alpha q; partials r.z, r.r
// The search direction alternates between two buffers (a node reads its
// neighbours' old p while they write their new one), and so do the r.z
// partials, by the parity of k, so no kernel overwrites a value another
// workgroup of the same kernel may still read. After the stop every later
// launch returns at once.
#include "cdi_internal.h"
#include "device_common.h"
#include "pot_internal.h"
#include "reduce_common.h"

namespace cdi {

namespace {

// Partial-sum regions, G doubles each.
// kRo: |r|^2 of the FP64 residual of a refinement round.
enum { kRz0 = 0, kRz1 = 1, kRr = 2, kPq = 3, kBb = 4, kNd = 5, kRo = 6, kRegions = 7 };

// nodes per thread (tiles per pass) of the stencil and update kernels
constexpr int kPotNodes = 2;

// The vectors a CG iteration works on: FP64 (x, r, q, p, p2) or the FP32
// set of a refinement round's correction (xf, rf, qf, pf, pf2).
template <class T>
struct Vecs;
template <>
struct Vecs<double> {
    __device__ static double *x(const PotArgs &a) { return a.x; }
    __device__ static double *r(const PotArgs &a) { return a.r; }
    __device__ static double *q(const PotArgs &a) { return a.q; }
    __device__ static double *p(const PotArgs &a) { return a.p; }
    __device__ static double *p2(const PotArgs &a) { return a.p2; }
};
template <>
struct Vecs<float> {
    __device__ static float *x(const PotArgs &a) { return a.xf; }
    __device__ static float *r(const PotArgs &a) { return a.rf; }
    __device__ static float *q(const PotArgs &a) { return a.qf; }
    __device__ static float *p(const PotArgs &a) { return a.pf; }
    __device__ static float *p2(const PotArgs &a) { return a.pf2; }
};

// Whether the solve has stopped, read once per workgroup so that all its
// waves take the same branch (a stop may be recorded by workgroup 0 of the
// running kernel; every workgroup then skips the same update either way).
__device__ inline bool stopped(const double *state, int *flag) { return stopped_at(state, kStDone, flag); }

// Face neighbours (map values) of node n: from the neighbour list, or
// looked up through the voxel map after the node's coordinates.
template <class L, int NBR>
__device__ inline void face_maps(const PotArgs &a, int n, int (&m)[2 * L::D])
{
    if (NBR) {
#pragma unroll
        for (int k = 0; k < 2 * L::D; ++k) m[k] = ldu(a.nbr + (size_t)k * a.g.P, (uint32_t)n);  // plane k
        return;
    }
    int x, y, z;
    unpack_xyz(a.g, ldu(a.g.fluid, (uint32_t)n), x, y, z);
    NbCtx c;
    nb_ctx<L>(a.g, x, y, z, a.xbc[0] == kPsixPeriodic, c);
#pragma unroll
    for (int k = 0; k < 2 * L::D; ++k) m[k] = nb_get<L>(a.g, c, k + 1);
}

// Set-up of a solve: x = the start field (or 0), the diagonal byte per
// node, and the partials |b|^2 and the count of Dirichlet faces. The start's
// residual is formed by the first refinement round. Faces from the
// neighbour list where there is one (NBR).
template <class L, int NBR>
__global__ __launch_bounds__(kTile) void pot_setup_kernel(PotArgs a)
{
    __shared__ double sm[kTile / 64];
    int t0, t1;
    tile_range(a.g.P / kTile, t0, t1);
    const int P = a.g.P;
    double bb = 0, nd = 0;
    for (int t = t0; t < t1; ++t) {
        const int n = t * kTile + threadIdx.x;
        double xv = 0;
        int diag = 0;
        if (n < a.g.n_f) {
            int m[2 * L::D];
            face_maps<L, NBR>(a, n, m);
#pragma unroll
            for (int k = 0; k < 2 * L::D; ++k)
                diag += m[k] >= 0 ? 1
                                  : (m[k] == kElectrode ||
                                     (m[k] == kOutside && a.xbc[k & 1 ? 0 : 1] == kPsixDirichlet)) ? 2 : 0;
            double b = a.src * ((double)a.z[0] * ldu(a.C, (uint32_t)n) +
                                (double)a.z[1] * ldu(a.C, (uint32_t)(P + n)));
            xv = a.psi0 ? (double)ldu(a.psi0, (uint32_t)n) : 0.0;
#pragma unroll
            for (int k = 0; k < 2 * L::D; ++k) {
                if (m[k] == kElectrode) {
                    b += 2.0 * a.psi_e;
                    nd += 1;
                } else if (m[k] == kOutside && a.xbc[k & 1 ? 0 : 1] == kPsixDirichlet) {
                    b += 2.0 * a.psi_x[k & 1 ? 0 : 1];
                    nd += 1;
                }
            }
            bb += b * b;
        }
        stu(a.x, (uint32_t)n, xv);
        a.dg[n] = (uint8_t)diag;
    }
    const double s_bb = wg_sum(bb, sm), s_nd = wg_sum(nd, sm);
    if (threadIdx.x == 0) {
        const int G = gridDim.x;
        a.part[kBb * G + blockIdx.x] = s_bb;
        a.part[kNd * G + blockIdx.x] = s_nd;
    }
}

// The new search direction at one node: z + beta p with z = r / diag. Node n
// evaluates it for itself and for its neighbours with this one expression,
// so every copy of a node's value is the same number.
__device__ inline double new_dir(double r, int d, double p, double beta)
{
    const double z = d > 0 ? r / d : 0.0;
    return z + beta * p;
}

// The FP32 correction solves precondition with the hardware FP32 reciprocal
// of the diagonal (one instruction instead of an FP64 division; the
// preconditioner is diag(inv_diag_f(d))^-1, the same in every kernel that
// applies it, so CG stays consistent) and form the direction in FP32, the
// precision it is stored in: every copy of a node's direction, its own and
// its neighbours', is the same FP32 number, the one stored.
__device__ inline float inv_diag_f(int d) { return d > 0 ? __builtin_amdgcn_rcpf((float)d) : 0.f; }

__device__ inline float new_dir_f(float r, int d, float p, float beta)
{
    return __builtin_fmaf(beta, p, __fmul_rn(r, inv_diag_f(d)));
}

// Stop test on |r_k|^2 (the r.r partials of the last axpy); the same
// decision in every workgroup. Workgroup 0 records it.
__device__ inline bool stop_test(const PotArgs &a, int k, double *sm)
{
    const int G = gridDim.x;
    const double rr = region_sum(a.part + kRr * G, G, sm);
    const bool bad = !isfinite(rr);
    const bool stop = bad || rr <= a.state[kStTol2Bb];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.state[kStIters] = k;
        a.state[kStRr] = rr;
        if (stop) a.state[kStDone] = bad ? kDoneDiverged : kDoneConverged;
    }
    return stop;
}

// Iteration k, first half: stop test on r_k; beta = rz_k / rz_{k-1} (0 at
// k = 0, where the start's p already is z); p_k = z_k + beta p_{k-1} into
// the other direction buffer; q = A p_k; partial p_k . q. A node needs p_k
// of its fluid neighbours, which it forms from their r, diagonal and old p.
// NN nodes per thread (tiles t and t + 1 of the range), all loads issued
// before any arithmetic.
template <class L, int NBR, int NN, class T>
__global__ __launch_bounds__(kTile) void pot_dirspmv_kernel(PotArgs a, int k)
{
    using V = Vecs<T>;
    constexpr int F = 2 * L::D;
    __shared__ double sm[kTile / 64];
    __shared__ int stop;
    if (stopped(a.state, &stop)) return;
    const int G = gridDim.x;
    double beta = 0.0;
    if (k > 0) {
        if (stop_test(a, k, sm)) return;
        beta = region_sum(a.part + (k & 1 ? kRz1 : kRz0) * G, G, sm) /
               region_sum(a.part + (k & 1 ? kRz0 : kRz1) * G, G, sm);
    }
    const T *pold = k & 1 ? V::p2(a) : V::p(a);
    T *pnew = k & 1 ? V::p(a) : V::p2(a);
    const T *rv = V::r(a);
    int t0, t1;
    tile_range(a.g.P / kTile, t0, t1);
    double pq = 0;
    for (int t = t0; t < t1; t += NN) {
        int n[NN], m[NN][F];
        bool act[NN];
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            n[j] = (t + j) * kTile + threadIdx.x;
            act[j] = t + j < t1 && n[j] < a.g.n_f;
            if (act[j])
                face_maps<L, NBR>(a, n[j], m[j]);
            else
#pragma unroll
                for (int f = 0; f < F; ++f) m[j][f] = kInert;
        }
        T r0[NN], p0[NN], rm[NN][F], pm[NN][F];
        int d0[NN], dm[NN][F];
        // every load unconditional (index 0 where there is no node or no
        // fluid neighbour; the value is not used there): inside a divergent
        // branch each gather would wait for its data before the next
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            const uint32_t q0 = act[j] ? (uint32_t)n[j] : 0u;
            r0[j] = ldu(rv, q0);
            p0[j] = ldu(pold, q0);
            d0[j] = act[j] ? a.dg[q0] : 0;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const uint32_t qm = m[j][f] >= 0 ? (uint32_t)m[j][f] : 0u;
                rm[j][f] = ldu(rv, qm);
                pm[j][f] = ldu(pold, qm);
                dm[j][f] = a.dg[qm];
            }
        }
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            if (!act[j]) continue;
            T pt;
            double q;
            if constexpr (sizeof(T) == 4) {
                const float bf = (float)beta;
                pt = new_dir_f(r0[j], d0[j], p0[j], bf);
                q = (double)d0[j] * (double)pt;  // A p accumulated in FP64 (it cancels)
#pragma unroll
                for (int f = 0; f < F; ++f)
                    if (m[j][f] >= 0) q -= (double)new_dir_f(rm[j][f], dm[j][f], pm[j][f], bf);
            } else {
                const double pn = new_dir(r0[j], d0[j], p0[j], beta);
                q = d0[j] * pn;
#pragma unroll
                for (int f = 0; f < F; ++f)
                    if (m[j][f] >= 0) q -= new_dir(rm[j][f], dm[j][f], pm[j][f], beta);
                pt = pn;
            }
            // stored in T; the partial is formed from the stored values
            const T qt = (T)q;
            stu(pnew, (uint32_t)n[j], pt);
            stu(V::q(a), (uint32_t)n[j], qt);
            pq += (double)pt * (double)qt;
        }
    }
    const double s = wg_sum(pq, sm);
    if (threadIdx.x == 0) a.part[kPq * G + blockIdx.x] = s;
}

// Iteration k, second half: alpha = rz_k / (p_k . q); x += alpha p_k;
// r -= alpha q; partials rz_{k+1} (into the other r.z slot) and |r_{k+1}|^2.
template <class T>
__global__ __launch_bounds__(kTile) void pot_axpy_kernel(PotArgs a, int k)
{
    using V = Vecs<T>;
    __shared__ double sm[kTile / 64];
    __shared__ int stop;
    if (stopped(a.state, &stop)) return;
    const int G = gridDim.x;
    const double rz = region_sum(a.part + (k & 1 ? kRz1 : kRz0) * G, G, sm);
    const double pq = region_sum(a.part + kPq * G, G, sm);
    if (!(pq > 0.0) || !isfinite(rz / pq)) {  // breakdown: A p has no positive energy
        if (blockIdx.x == 0 && threadIdx.x == 0) a.state[kStDone] = kDoneBreakdown;
        return;
    }
    const double alpha = rz / pq;
    const T *pk = k & 1 ? V::p(a) : V::p2(a);
    T *xv = V::x(a), *rv = V::r(a);
    const T *qv = V::q(a);
    int t0, t1;
    tile_range(a.g.P / kTile, t0, t1);
    double rz1 = 0, rr = 0;
    // kPotNodes tiles per pass, all loads issued before any store (more
    // loads in flight per wave; index 0 where there is no node, not stored)
    for (int t = t0; t < t1; t += kPotNodes) {
        int n[kPotNodes];
        bool act[kPotNodes];
        T pv[kPotNodes], qv_[kPotNodes], xo[kPotNodes], ro[kPotNodes];
        int dv[kPotNodes];
#pragma unroll
        for (int j = 0; j < kPotNodes; ++j) {
            n[j] = (t + j) * kTile + threadIdx.x;
            act[j] = t + j < t1 && n[j] < a.g.n_f;
            const uint32_t q = act[j] ? (uint32_t)n[j] : 0u;
            pv[j] = ldu(pk, q);
            qv_[j] = ldu(qv, q);
            xo[j] = ldu(xv, q);
            ro[j] = ldu(rv, q);
            dv[j] = a.dg[q];
        }
#pragma unroll
        for (int j = 0; j < kPotNodes; ++j) {
            if (!act[j]) continue;
            stu(xv, (uint32_t)n[j], (T)(xo[j] + alpha * (double)pv[j]));
            const T rt = (T)(ro[j] - alpha * (double)qv_[j]);
            stu(rv, (uint32_t)n[j], rt);
            const double rn = rt;
            double zn;
            if constexpr (sizeof(T) == 4)
                zn = __fmul_rn((float)rt, inv_diag_f(dv[j]));  // the z the stencil kernel forms
            else
                zn = dv[j] > 0 ? rn / dv[j] : 0.0;
            rz1 += rn * zn;
            rr += rn * rn;
        }
    }
    const double s_rz = wg_sum(rz1, sm), s_rr = wg_sum(rr, sm);
    if (threadIdx.x == 0) {
        a.part[(k & 1 ? kRz0 : kRz1) * G + blockIdx.x] = s_rz;
        a.part[kRr * G + blockIdx.x] = s_rr;
    }
}

// The stop test of iteration k on its own (one workgroup), run after a batch
// of iterations ending with iteration k - 1: records the same decision the
// next iteration would take.
__global__ __launch_bounds__(kTile) void pot_check_kernel(PotArgs a, int k, int G)
{
    __shared__ double sm[kTile / 64];
    if (a.state[kStDone] != 0.0) return;  // one workgroup: written only by earlier kernels
    const double rr = region_sum(a.part + kRr * G, G, sm);
    if (threadIdx.x == 0) {
        const bool bad = !isfinite(rr);
        a.state[kStIters] = k;
        a.state[kStRr] = rr;
        if (bad || rr <= a.state[kStTol2Bb]) a.state[kStDone] = bad ? kDoneDiverged : kDoneConverged;
    }
}

// Totals of the set-up (one workgroup): |b|^2 and the Dirichlet faces.
__global__ __launch_bounds__(kTile) void pot_state_kernel(PotArgs a, int G, double tol)
{
    __shared__ double sm[kTile / 64];
    const double bb = region_sum(a.part + kBb * G, G, sm);
    const double nd = region_sum(a.part + kNd * G, G, sm);
    if (threadIdx.x == 0) {
        a.state[kStBb] = bb;
        a.state[kStTol2Bb] = tol * tol * bb;
        a.state[kStRr] = 0.0;  // the first refinement round measures it
        a.state[kStNdir] = nd;
        a.state[kStIters] = 0;
        a.state[kStDone] = 0.0;
    }
}

// Refinement round: the FP64 residual r = b - A x of the current x, its
// partial |r|^2 (kRo), and the start of an FP32 correction solve A d = r:
// rf = r, xf = 0, p = z = rf inv_diag_f(diag), partial rf . z (kRz0). F64: instead the
// start of FP64 CG iterations on x itself (r, p = z in FP64). Faces from the
// neighbour list where there is one (NBR), the diagonal from the set-up.
template <class L, int F64, int NBR>
__global__ __launch_bounds__(kTile) void pot_refine_kernel(PotArgs a)
{
    __shared__ double sm[kTile / 64];
    int t0, t1;
    tile_range(a.g.P / kTile, t0, t1);
    const int P = a.g.P;
    double rz = 0, ro = 0;
    for (int t = t0; t < t1; ++t) {
        const int n = t * kTile + threadIdx.x;
        float rf = 0.f, zf = 0.f;
        if (n < a.g.n_f) {
            int m[2 * L::D];
            face_maps<L, NBR>(a, n, m);
            const int diag = a.dg[n];
            double b = a.src * ((double)a.z[0] * ldu(a.C, (uint32_t)n) + (double)a.z[1] * ldu(a.C, (uint32_t)(P + n)));
            double ax = diag * ldu(a.x, (uint32_t)n);
            double xm[2 * L::D];  // loaded before use (index 0 where not fluid: unused)
#pragma unroll
            for (int k = 0; k < 2 * L::D; ++k) xm[k] = ldu(a.x, (uint32_t)(m[k] >= 0 ? m[k] : 0));
#pragma unroll
            for (int k = 0; k < 2 * L::D; ++k) {
                if (m[k] >= 0)
                    ax -= xm[k];
                else if (m[k] == kElectrode)
                    b += 2.0 * a.psi_e;
                else if (m[k] == kOutside && a.xbc[k & 1 ? 0 : 1] == kPsixDirichlet)
                    b += 2.0 * a.psi_x[k & 1 ? 0 : 1];
            }
            const double r = b - ax;
            ro += r * r;
            if (F64) {
                const double zd = diag > 0 ? r / diag : 0.0;
                stu(a.r, (uint32_t)n, r);
                stu(a.p, (uint32_t)n, zd);
                rz += r * zd;
            } else {
                rf = (float)r;
                zf = __fmul_rn(rf, inv_diag_f(diag));  // the z the stencil kernel forms
                rz += (double)rf * (double)zf;
            }
        } else if (F64) {
            stu(a.r, (uint32_t)n, 0.0);
            stu(a.p, (uint32_t)n, 0.0);
        }
        if (!F64) {
            stu(a.rf, (uint32_t)n, rf);
            stu(a.xf, (uint32_t)n, 0.f);
            stu(a.pf, (uint32_t)n, zf);
        }
    }
    const double s_rz = wg_sum(rz, sm), s_ro = wg_sum(ro, sm);
    if (threadIdx.x == 0) {
        const int G = gridDim.x;
        a.part[kRz0 * G + blockIdx.x] = s_rz;
        a.part[kRo * G + blockIdx.x] = s_ro;
    }
}

// After a refinement kernel (one workgroup): the outer stop test on the FP64
// residual, |r|^2 <= tol^2 |b|^2 (recorded in kStRr); else the correction
// solve runs until its residual falls by max(tol_min, tol |b| / |r|).
__global__ __launch_bounds__(kTile) void pot_refine_state_kernel(PotArgs a, int G, double tol, double tol_min)
{
    __shared__ double sm[kTile / 64];
    const double ro = region_sum(a.part + kRo * G, G, sm);
    if (threadIdx.x == 0) {
        const double bb = a.state[kStBb];
        a.state[kStRr] = ro;
        a.state[kStIters] = 0;
        if (!isfinite(ro)) {
            a.state[kStDone] = kDoneDiverged;
        } else if (ro <= tol * tol * bb) {
            a.state[kStDone] = kDoneConverged;
        } else {
            const double f2 = fmax(tol_min * tol_min, tol * tol * bb / ro);
            a.state[kStTol2Bb] = f2 * ro;
            a.state[kStDone] = 0.0;
        }
    }
}

// x += xf: the correction of a refinement round.
__global__ __launch_bounds__(kTile) void pot_correct_kernel(double *x, const float *xf, int n_f)
{
    const int n = blockIdx.x * kTile + threadIdx.x;
    if (n < n_f) x[n] += (double)xf[n];
}

__global__ __launch_bounds__(kTile) void pot_store_kernel(const double *x, float *psi, int n_f)
{
    const int n = blockIdx.x * kTile + threadIdx.x;
    if (n < n_f) psi[n] = (float)x[n];
}

}  // namespace

uint64_t pot_part_doubles() { return (uint64_t)kRegions * kPotMaxWorkgroups; }

// As many persistent workgroups as the stencil kernel (the largest register
// footprint of the solve) keeps resident on the device at once: a workgroup
// that had to wait for a free slot would double the kernel's time.
hipError_t pot_workgroups(int dim, int ntiles, bool nbr, int *G)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const void *k = dim == 2 ? (nbr ? (const void *)pot_dirspmv_kernel<D2Q9, 1, kPotNodes, double>
                                    : (const void *)pot_dirspmv_kernel<D2Q9, 0, kPotNodes, double>)
                             : (nbr ? (const void *)pot_dirspmv_kernel<D3Q19, 1, kPotNodes, double>
                                    : (const void *)pot_dirspmv_kernel<D3Q19, 0, kPotNodes, double>);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kTile, 0);
    if (e != hipSuccess) return e;
    // at most 4 per CU: with more, one tile step of all resident workgroups
    // outgrows an XCD's L2 before the neighbouring tiles are read again
    // (measured on the 512^3 electrode: 1.49 ms per iteration at 4, 1.55 at
    // the occupancy limit, 1.60 at 3)
    if (per_cu > kPotWorkgroupsPerCU) per_cu = kPotWorkgroupsPerCU;
    long long g = (long long)cus * (per_cu > 0 ? per_cu : 1);
    g = g < kPotMaxWorkgroups ? g : kPotMaxWorkgroups;
    *G = (int)(ntiles < g ? ntiles : g);
    return hipSuccess;
}

hipError_t launch_pot_setup(int dim, const PotArgs &a, int G, double tol, hipStream_t s)
{
    if (dim == 2)
        a.nbr ? pot_setup_kernel<D2Q9, 1><<<G, kTile, 0, s>>>(a) : pot_setup_kernel<D2Q9, 0><<<G, kTile, 0, s>>>(a);
    else
        a.nbr ? pot_setup_kernel<D3Q19, 1><<<G, kTile, 0, s>>>(a) : pot_setup_kernel<D3Q19, 0><<<G, kTile, 0, s>>>(a);
    pot_state_kernel<<<1, kTile, 0, s>>>(a, G, tol);
    return hipGetLastError();
}

template <class L, class T>
void pot_iter_l(const PotArgs &a, int G, int k, hipStream_t s)
{
    if (a.nbr)
        pot_dirspmv_kernel<L, 1, kPotNodes, T><<<G, kTile, 0, s>>>(a, k);
    else
        pot_dirspmv_kernel<L, 0, kPotNodes, T><<<G, kTile, 0, s>>>(a, k);
    pot_axpy_kernel<T><<<G, kTile, 0, s>>>(a, k);
}

hipError_t launch_pot_iter(int dim, const PotArgs &a, int G, int k, bool f32, hipStream_t s)
{
    if (dim == 2)
        f32 ? pot_iter_l<D2Q9, float>(a, G, k, s) : pot_iter_l<D2Q9, double>(a, G, k, s);
    else
        f32 ? pot_iter_l<D3Q19, float>(a, G, k, s) : pot_iter_l<D3Q19, double>(a, G, k, s);
    return hipGetLastError();
}

template <class L>
void refine_l(const PotArgs &a, int G, bool f64, hipStream_t s)
{
    if (a.nbr)
        f64 ? pot_refine_kernel<L, 1, 1><<<G, kTile, 0, s>>>(a) : pot_refine_kernel<L, 0, 1><<<G, kTile, 0, s>>>(a);
    else
        f64 ? pot_refine_kernel<L, 1, 0><<<G, kTile, 0, s>>>(a) : pot_refine_kernel<L, 0, 0><<<G, kTile, 0, s>>>(a);
}

hipError_t launch_pot_refine(int dim, const PotArgs &a, int G, double tol, double tol_min, bool f64, hipStream_t s)
{
    if (dim == 2)
        refine_l<D2Q9>(a, G, f64, s);
    else
        refine_l<D3Q19>(a, G, f64, s);
    pot_refine_state_kernel<<<1, kTile, 0, s>>>(a, G, tol, tol_min);
    return hipGetLastError();
}

hipError_t launch_pot_correct(const PotArgs &a, hipStream_t s)
{
    const int tiles = a.g.P / kTile;
    if (tiles > 0) pot_correct_kernel<<<tiles, kTile, 0, s>>>(a.x, a.xf, a.g.n_f);
    return hipGetLastError();
}

hipError_t launch_pot_check(const PotArgs &a, int G, int k, hipStream_t s)
{
    pot_check_kernel<<<1, kTile, 0, s>>>(a, k, G);
    return hipGetLastError();
}

hipError_t launch_pot_store(const PotArgs &a, float *psi, hipStream_t s)
{
    const int tiles = a.g.P / kTile;
    if (tiles > 0) pot_store_kernel<<<tiles, kTile, 0, s>>>(a.x, psi, a.g.n_f);
    return hipGetLastError();
}

}  // namespace cdi
