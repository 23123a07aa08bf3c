// cdi_api.hip -- host side of the C ABI declared in include/cdi.h: argument
// checks, workspace carving, step sequencing (AA parity, double buffers) and
// the synchronising read-backs. All arithmetic of the model runs in the
// kernels of geometry.hip and step.hip.
#include "cdi.h"
#include "cdi_internal.h"
#include "diag_internal.h"
#include "geometry_internal.h"
#include "np_solve_internal.h"
#include "geomgen.h"
#include "pot_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstring>
#include <new>
#include <algorithm>
#include <mutex>
#include <vector>

using namespace cdi;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(CDI_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

constexpr uint64_t kAlign = 256;
constexpr float kHalfScale = 4096.f;  // FP16 deviations are stored times 2^12

uint64_t up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Consumes an aligned slice of a workspace.
struct Carver {
    uint8_t *base;
    uint64_t off = 0;
    explicit Carver(void *b) : base((uint8_t *)b) {}
    template <class T>
    T *take(uint64_t bytes)
    {
        T *p = (T *)(base ? base + off : nullptr);
        off += up(bytes);
        return p;
    }
};

int check_geometry(const cdi_geometry *g)
{
    if (!g) return fail(CDI_E_INVALID, "geometry is NULL");
    if (g->dim != 2 && g->dim != 3) return fail(CDI_E_INVALID, "dim must be 2 or 3");
    const int nz = g->dim == 2 ? 1 : g->nz;
    if (g->nx < 4 || g->ny < 1 || nz < 1) return fail(CDI_E_INVALID, "lattice too small (nx >= 4)");
    const double nvox = (double)g->nx * g->ny * nz;
    if (nvox >= 2147483647.0) return fail(CDI_E_INVALID, "nx*ny*nz must be < 2^31");
    // the step kernels address the brick-ordered map with 32-bit byte offsets
    const double bricked = (double)((g->nx + 15) / 16 * 16) * ((g->ny + 15) / 16 * 16) *
                           (g->dim == 2 ? 1 : (nz + 15) / 16 * 16);
    if (bricked * 4.0 >= 4294967296.0) return fail(CDI_E_INVALID, "lattice too large for one instance (> 2^30 voxels)");
    {
        int bits = 0;
        for (int n : {g->nx, g->ny, nz}) {
            int b = 0;
            while ((1ll << b) < n) ++b;
            bits += b;
        }
        if (bits > 32) return fail(CDI_E_INVALID, "lattice too large: packed node coordinates need %d bits", bits);
        // the padded brick enumeration must stay below 2^31 as well
        const double padded = (double)((g->nx + 15) / 8 * 8) * ((g->ny + 15) / 8 * 8) * ((nz + 7) / 8 * 8);
        if (padded >= 2147483647.0) return fail(CDI_E_INVALID, "padded lattice must hold < 2^31 voxels");
    }
    if (g->kind == CDI_USER_LABELS) {
        if (!g->user_labels) return fail(CDI_E_INVALID, "user_labels is NULL");
        return CDI_OK;
    }
    if (g->kind == CDI_DISKS && g->dim != 2) return fail(CDI_E_INVALID, "disks need dim 2");
    if (g->kind == CDI_SPHERES && g->dim != 3) return fail(CDI_E_INVALID, "spheres need dim 3");
    if (g->kind == CDI_FIBRES && g->dim != 3) return fail(CDI_E_INVALID, "fibres need dim 3");
    if (g->kind != CDI_DISKS && g->kind != CDI_SPHERES && g->kind != CDI_FIBRES)
        return fail(CDI_E_INVALID, "unknown kind");
    if (g->kind == CDI_FIBRES && (g->nx > 1024 || g->ny > 1024 || nz > 1024 || g->r_max > 64))
        return fail(CDI_E_INVALID, "fibres: lattice edges <= 1024 and r_max <= 64 (exact int64 inside test)");
    if (!(g->porosity > 0 && g->porosity <= 1)) return fail(CDI_E_INVALID, "porosity out of (0, 1]");
    if (!(g->r_min > 0 && g->r_max >= g->r_min)) return fail(CDI_E_INVALID, "bad radius range");
    if (g->buffer_x < 0 || 2 * g->buffer_x >= g->nx) return fail(CDI_E_INVALID, "bad buffer_x");
    return CDI_OK;
}

int check_params(const cdi_params *p)
{
    if (!p) return fail(CDI_E_INVALID, "params is NULL");
    if (!(p->tau > 0.5)) return fail(CDI_E_UNSTABLE, "tau must exceed 1/2 (nu = (tau - 1/2)/3 > 0)");
    if (p->drive != CDI_INLET_OUTLET && p->drive != CDI_BODY_FORCE) return fail(CDI_E_INVALID, "bad drive");
    if (p->equilibrium != CDI_EQ_QUADRATIC && p->equilibrium != CDI_EQ_LINEAR)
        return fail(CDI_E_INVALID, "bad equilibrium");
    if (p->np_x_bc < 0 || p->np_x_bc > 3) return fail(CDI_E_INVALID, "bad np_x_bc");
    if (p->np_substeps < 1) return fail(CDI_E_INVALID, "np_substeps must be >= 1");
    if (p->precision != CDI_FP32 && p->precision != CDI_FP16_DEV && p->precision != CDI_MOMENTS &&
        p->precision != CDI_FP16)
        return fail(CDI_E_INVALID, "bad precision");
    if (p->streaming != CDI_STREAM_AA && p->streaming != CDI_STREAM_PULL)
        return fail(CDI_E_INVALID, "bad streaming");
    if (p->precision == CDI_MOMENTS && (p->tau != 1.0 || p->drive == CDI_BODY_FORCE))
        return fail(CDI_E_INVALID, "moment storage needs tau = 1 and no body force "
                                   "(only then is the post-collision state the local equilibrium)");
    if (!(p->D[0] > 0 && p->D[1] > 0)) return fail(CDI_E_INVALID, "diffusivities must be positive");
    return CDI_OK;
}

// Seeded primitives of the geometry (host). Returns CDI status.
int make_prims(const cdi_geometry *g, std::vector<geomgen_prim> &out, int64_t *nfluid_exact)
{
    out.clear();
    if (nfluid_exact) *nfluid_exact = -1;
    geomgen_prim *pp = nullptr;
    int64_t n = 0;
    int rc;
    if (g->kind == CDI_DISKS) {
        int64_t nf = 0;
        rc = geomgen_disks(g->nx, g->ny, g->buffer_x, g->walls_y, g->seed, g->porosity, g->r_min,
                           g->r_max, g->min_gap, &pp, &n, &nf);
        if (nfluid_exact) *nfluid_exact = nf;
    } else if (g->kind == CDI_SPHERES) {
        rc = geomgen_spheres(g->nx, g->ny, g->nz, g->buffer_x, g->seed, g->porosity, g->r_min,
                             g->r_max, &pp, &n);
    } else {
        return CDI_OK;
    }
    if (rc == GEOMGEN_E_JAMMED) return fail(CDI_E_GEOMETRY, "random sequential addition jammed before the porosity");
    if (rc != GEOMGEN_OK) return fail(CDI_E_INVALID, "primitive generator rejected the geometry (rc %d)", rc);
    out.assign(pp, pp + n);
    geomgen_free(pp);
    return CDI_OK;
}

// Seeded straight fibres of a CDI_FIBRES geometry (host).
int make_fibres(const cdi_geometry *g, std::vector<geomgen_fibre> &out)
{
    out.clear();
    geomgen_fibre *pp = nullptr;
    int64_t n = 0;
    const int rc = geomgen_fibres(g->nx, g->ny, g->nz, g->buffer_x, g->seed, g->porosity, g->r_min, g->r_max,
                                  &pp, &n);
    if (rc != GEOMGEN_OK) return fail(CDI_E_INVALID, "fibre generator rejected the geometry (rc %d)", rc);
    out.assign(pp, pp + n);
    geomgen_free(pp);
    return CDI_OK;
}

// Voxel-level workspace: labels, the public (lexicographic) fluid map and
// list, and the internal brick-ordered map, node list and permutation.
struct VoxLayout {
    uint8_t *labels;
    int *map, *fluid, *blk;
    int *imap, *lex2int, *blk2;
    uint32_t *ifluid;
    int64_t *nfluid, *nfluid2;
    int64_t *prims;
    Bricks bk;
    uint64_t bytes;
};

int64_t geom_nvox(const cdi_geometry *g) { return (int64_t)g->nx * g->ny * (g->dim == 2 ? 1 : g->nz); }

// bits needed to hold 0 .. n-1
int coord_bits(int n)
{
    int b = 0;
    while ((1ll << b) < n) ++b;
    return b;
}

// Bricks of 16x16x16 voxels in 3D and 16x16 in 2D (measured against 8^3,
// 16x8x8, 32x8x8 and 16x16x8 on the 512^3 electrode: fewer brick crossings,
// so the 16 lanes of a quarter-wave gather from fewer cache lines).
Bricks make_bricks(const cdi_geometry *g)
{
    Bricks k;
    const int nz = g->dim == 2 ? 1 : g->nz;
    k.bsx = 4;
    k.bsy = 4;
    k.bsz = g->dim == 2 ? 0 : 4;
    k.nbx = (g->nx + (1 << k.bsx) - 1) >> k.bsx;
    k.nby = (g->ny + (1 << k.bsy) - 1) >> k.bsy;
    k.nbz = (nz + (1 << k.bsz) - 1) >> k.bsz;
    k.cbx = coord_bits(g->nx);
    k.cby = coord_bits(g->ny);
    return k;
}

VoxLayout vox_layout(void *ws, const cdi_geometry *g, int64_t nprims)
{
    const int64_t nvox = geom_nvox(g);
    Carver c(ws);
    VoxLayout L;
    L.bk = make_bricks(g);
    const int64_t E = brick_enum_size(L.bk);
    L.labels = c.take<uint8_t>((uint64_t)nvox);
    L.map = c.take<int>(4ull * nvox);
    L.fluid = c.take<int>(4ull * nvox);
    L.blk = c.take<int>(4ull * (uint64_t)compact_blocks(nvox));
    L.imap = c.take<int>(4ull * E);
    L.ifluid = c.take<uint32_t>(4ull * nvox);
    L.lex2int = c.take<int>(4ull * nvox);
    L.blk2 = c.take<int>(4ull * (uint64_t)compact_blocks(E));
    L.nfluid = c.take<int64_t>(8);
    L.nfluid2 = c.take<int64_t>(8);
    L.prims = c.take<int64_t>(64ull * (uint64_t)(nprims > 0 ? nprims : 1));  // 8 int64 per fibre, 4 otherwise
    L.bytes = c.off;
    return L;
}

}  // namespace

struct NodeLayout {
    void *f;
    void *f2;    // pull streaming: the second population array
    float4 *M[2];
    float *j[2];
    float *ubuf;
    float *C[2];
    __half2 *Clo[2];  // the concentrations' FP16 remainders (both species per node)
    float *tmp;
    float *xfer;  // lexicographic staging for host copies (4 planes of N_f)
    float *psi;   // prescribed potential in internal node order
    float *rref[2];  // FP32 storage: plane reference tables (nx values each; see PlaneRef)
    double *acc, *resid, *part, *red;
    int *sched;
    int *nbr;    // neighbour list (Q-1 planes of P), built once
    double *diag;  // diagnostics scratch (per-tile and per-plane-chunk sums)
    void *base;  // start of the state a checkpoint carries (state_bytes from here)
    uint64_t state_bytes, bytes;
};

// Bytes per stored population of a storage kind.
static int pop_bytes(int st) { return st == kF32 ? 4 : (st == kF16 || st == kH16) ? 2 : 0; }
// the storages with FP32 moment buffers (their fused steps carry j there)
static bool moment_buffers(int st) { return st == kF16 || st == kMom; }
// the storages relative to plane references
static bool plain_pops(int st) { return st == kF32 || st == kH16; }

// Doubles of the diagnostics scratch: per-tile sums (3 per tile) or the
// vertical-profile partials (3 per x plane and z chunk) plus its result (3 nx).
static uint64_t diag_doubles(const cdi_geometry *g, int64_t P)
{
    const int64_t nz = g->dim == 2 ? 1 : g->nz;
    const int64_t prof = 3ll * g->nx * ((nz + 7) / 8) + 3ll * g->nx;
    const int64_t tiles = 6 * (P / kTile) + 6;  // diagnostics: 3 per tile; ion rates: 6 per tile
    return (uint64_t)(prof > tiles ? prof : tiles);
}

static NodeLayout node_layout(void *ws, int dim, int st, int pull, int64_t P, int64_t plane,
                              uint64_t ndiag, int64_t nx)
{
    const int Q = dim == 2 ? 9 : 19;
    const int64_t ntiles = P / kTile;
    const bool mb = moment_buffers(st);
    Carver c(ws);
    NodeLayout L;
    L.base = ws;
    L.f = c.take<void>((uint64_t)Q * P * pop_bytes(st));
    L.f2 = c.take<void>(pull ? (uint64_t)Q * P * pop_bytes(st) : 0);
    if (!pull || st == kMom) L.f2 = nullptr;
    L.M[0] = c.take<float4>(mb ? 16ull * P : 0);
    L.M[1] = c.take<float4>(mb ? 16ull * P : 0);
    if (!mb) L.M[0] = L.M[1] = nullptr;
    if (st == kMom) L.f = nullptr;
    L.j[0] = c.take<float>(4ull * dim * P);
    L.j[1] = c.take<float>(4ull * dim * P);
    L.ubuf = c.take<float>(4ull * (dim + 1) * P);
    L.C[0] = c.take<float>(8ull * P);
    L.C[1] = c.take<float>(8ull * P);
    L.Clo[0] = c.take<__half2>(4ull * P);
    L.Clo[1] = c.take<__half2>(4ull * P);
    L.tmp = c.take<float>(4ull * (1 + dim) * P);
    L.xfer = c.take<float>(16ull * P);
    L.psi = c.take<float>(4ull * P);
    L.rref[0] = c.take<float>(plain_pops(st) ? 4ull * nx : 0);
    L.rref[1] = c.take<float>(plain_pops(st) ? 4ull * nx : 0);
    if (!plain_pops(st)) L.rref[0] = L.rref[1] = nullptr;
    L.acc = c.take<double>(64ull * ntiles);
    L.resid = c.take<double>(16ull * ntiles);
    L.part = c.take<double>(16ull * ntiles);
    L.red = c.take<double>(64 * 8);
    L.state_bytes = c.off;  // everything a checkpoint must carry ends here
    L.sched = c.take<int>(4ull * ntiles);
    L.nbr = c.take<int>(4ull * (Q - 1) * P);
    L.diag = c.take<double>(8ull * ndiag);
    L.bytes = c.off;
    return L;
}

enum { J_INVALID = 0, J_VALID = 1, J_IN_M = 2 };

struct cdi_solver {
    cdi_geometry geom;
    cdi_params params;
    int dim, Q, inout;
    int st;    // storage: kF32, kF16, kMom or kH16
    int pull;  // pull streaming (two population arrays; fcur holds the state)
    int mb;  // moment buffers in use (kF16, kMom): j of a fused step lives in them
    int64_t nvox, nf;
    int P, ntiles;
    int device;  // the device current at initialisation (its buffers live there)
    hipStream_t stream;
    VoxLayout vox;
    NodeLayout node;
    int parity = 0, fcur = 0, mcur = 0, jcur = 0, ccur = 0, jstate = J_INVALID;
    int rcur = 0;   // FP32: the plane reference table of the stored state
    int rpend = 0;  // the next flow step renews it (reads with rref[rcur], writes with the other)
    int rlive = 0;  // the references have been renewed at least once (before, all are zero)
    int64_t flow_steps = 0, np_steps = 0;
    double ka, keff[2], porosity;
    cdi_tuning tuning{0, 0, 0, 0, 0};
    Grid g;
    Phys p;
};

namespace {

struct SnapHeader {
    uint64_t magic, bytes;
    int32_t parity, mcur, jcur, ccur, jstate, fcur;
    int32_t psi_on;  // the potential in use is the field in the state (else the ramp)
    int32_t rstate;  // rcur | rpend << 1 | rlive << 2
    int64_t flow_steps, np_steps, nf;
};
constexpr uint64_t kSnapMagic = 0x43444931534e4150ull;

// Population array holding the state, and the kernels' parity argument.
void *cur_pops(const cdi_solver *s) { return s->pull && s->fcur ? s->node.f2 : s->node.f; }
// FP32 / FP16 populations: the plane reference table of the stored state
// (nullptr while every reference is still zero, so the steps skip it).
const float *cur_rref(const cdi_solver *s) { return s->rlive ? s->node.rref[s->rcur] : nullptr; }
int stream_arg(const cdi_solver *s) { return s->pull ? kPull : s->parity; }

// Buffers of the next step of s (current double-buffer halves).
Bufs make_bufs(const cdi_solver *s, int flags)
{
    Bufs b{};
    b.f = cur_pops(s);
    b.f2 = s->pull ? (s->fcur ? s->node.f : s->node.f2) : nullptr;
    if (s->mb) {
        b.Min = s->node.M[s->mcur];
        b.Mout = s->node.M[s->mcur ^ 1];
    }
    b.jin = s->node.j[s->jcur];
    b.jout = s->node.j[s->jcur ^ 1];
    b.Cin = s->node.C[s->ccur];
    b.Cout = s->node.C[s->ccur ^ 1];
    b.Clin = s->node.Clo[s->ccur];
    b.Clout = s->node.Clo[s->ccur ^ 1];
    b.ubuf = s->node.ubuf;
    b.rin = cur_rref(s);
    b.rout = s->rpend ? s->node.rref[s->rcur ^ 1] : b.rin;
    if (s->rpend && !b.rin) b.rin = s->node.rref[s->rcur];  // the first renewal reads the zero table
    b.acc = s->node.acc;
    b.resid = s->node.resid;
    b.flags = flags | (s->flow_steps > 0 ? kNee : 0);
    return b;
}

// Host bookkeeping of one completed step (AA parity, buffer halves, counters).
void advance_state(cdi_solver *s, int lbm, int np)
{
    if (lbm) {
        if (s->rpend) {
            s->rcur ^= 1;
            s->rpend = 0;
        }
        s->parity ^= 1;
        if (s->pull) s->fcur ^= 1;
        if (s->mb) s->mcur ^= 1;
        if (np && !s->mb) s->jcur ^= 1;
        s->flow_steps++;
    }
    if (np) s->ccur ^= 1;
}

int step_once(cdi_solver *s, int lbm, int np, int flags)
{
    const Bufs b = make_bufs(s, flags);
    HIPCHK(launch_step(s->dim, s->st, stream_arg(s), lbm, np, s->g, s->p, b, s->stream));
    advance_state(s, lbm, np);
    return CDI_OK;
}

int ensure_j(cdi_solver *s)
{
    if (s->jstate == J_VALID) return CDI_OK;
    if (s->jstate == J_IN_M) {
        HIPCHK(launch_j_from_m(s->dim, s->g, s->node.M[s->mcur], s->node.j[s->jcur], s->stream));
    } else {
        HIPCHK(launch_moments(s->dim, s->st, stream_arg(s), s->flow_steps > 0, s->g, s->p, cur_pops(s),
                              s->mb ? s->node.M[s->mcur] : nullptr, cur_rref(s), nullptr, nullptr,
                              s->node.j[s->jcur], s->stream));
    }
    s->jstate = J_VALID;
    return CDI_OK;
}

int d2h(cdi_solver *s, void *dst, const void *src, uint64_t bytes);

// Positivity bound of the explicit ion update with the current flux field:
// *worst = max dt * (sum of outflow coefficients). Synchronises.
int check_stability(cdi_solver *s, double *worst)
{
    int rc = ensure_j(s);
    if (rc) return rc;
    HIPCHK(launch_stability(s->dim, s->g, s->p, s->node.j[s->jcur], s->node.part, s->node.red, s->stream));
    return d2h(s, worst, s->node.red, 8);
}

// Tile schedule for 3D lattices: tiles sorted by (band of kBandRows rows, z,
// y, index). Each XCD then sweeps its bands plane by plane, so the data of the
// planes above and below a tile was touched a few tiles earlier by the same
// XCD (L2 reuse) instead of a whole plane earlier.
constexpr int kBandRows = 16;

// XCD-local position of workgroup b of nb (as xcd_tile on the device).
int64_t xcd_position(int64_t b, int64_t nb)
{
    const int64_t q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Tile schedule (XCD-local position -> tile) for the tuning's order:
//  * bands: each XCD walks a contiguous run of (band of band_rows rows, z, y);
//  * columns: tiles sorted by (group of 8 brick layers, brick row, brick
//    column, layer in the group) and dealt to workgroups in that order, so
//    the 8 XCDs work at once on the 8 layers of a group at the same (x, y):
//    the layers above and below a tile are being fetched by the neighbouring
//    XCDs and are met in the memory-side cache;
//  * columns == 2: tiles sorted by the Morton (Z-order) index of their brick
//    and each XCD walks a contiguous run of that curve, so that a brick's
//    face neighbours along every axis are mostly a few bricks away in the
//    XCD's own sweep (in the plain order the brick above is a whole layer
//    of bricks later).
uint64_t morton3(uint64_t x, uint64_t y, uint64_t z)
{
    uint64_t m = 0;
    for (int b = 0; b < 21; ++b)
        m |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2);
    return m;
}

int build_schedule(cdi_solver *s, int band_rows, int columns)
{
    const int T = s->ntiles;
    if (s->dim != 3 || (band_rows <= 0 && !columns)) {
        s->g.sched = nullptr;
        s->tuning.band_rows = 0;
        s->tuning.columns = 0;
        return CDI_OK;
    }
    std::vector<uint32_t> heads(T);
    HIPCHK(launch_tile_heads(s->g, (uint32_t *)s->node.sched, s->stream));
    HIPCHK(hipMemcpyAsync(heads.data(), s->node.sched, 4ull * T, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    const Bricks &k = s->g.bk;
    const int64_t ny = s->g.ny;
    std::vector<int64_t> key(T);
    std::vector<int> order(T);
    for (int t = 0; t < T; ++t) {
        const uint32_t c = heads[t];
        const int64_t x = c & ((1u << k.cbx) - 1);
        const int64_t y = (c >> k.cbx) & ((1u << k.cby) - 1);
        const int64_t z = c >> (k.cbx + k.cby);
        if (columns == 2) {
            key[t] = (int64_t)morton3(x >> k.bsx, y >> k.bsy, z >> k.bsz);
        } else if (columns) {
            const int64_t bx = x >> k.bsx, by = y >> k.bsy, bz = z >> k.bsz;
            key[t] = (((bz >> 3) * k.nby + by) * k.nbx + bx) * 8 + (bz & 7);
        } else {
            key[t] = ((y / band_rows) * s->g.nz + z) * ny + y;
        }
        order[t] = t;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::vector<int> sched(T);
    if (columns == 1) {
        for (int64_t b = 0; b < T; ++b) sched[xcd_position(b, T)] = order[b];
    } else {
        sched = order;
    }
    HIPCHK(hipMemcpyAsync(s->node.sched, sched.data(), 4ull * T, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->g.sched = s->node.sched;
    s->tuning.band_rows = columns ? 0 : band_rows;
    s->tuning.columns = columns;
    return CDI_OK;
}

// Whether an instance of ntiles tiles stages its odd steps (cdi_tuning::stage_odd).
int stage_odd_for(int mode, int64_t ntiles)
{
    return mode == 1 || (mode == 0 && ntiles >= CDI_STAGE_MIN_TILES);
}

// LDS bytes that leave room for at most k step workgroups per CU.
int occupancy_pad(int k, int *pad)
{
    *pad = 0;
    if (k <= 0) return CDI_OK;
    int dev = 0, per_cu = 0, per_block = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
    HIPCHK(hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int static_lds = 1024;  // the step kernel's own reduction scratch, rounded up
    int want = per_cu / k - static_lds;
    want = want / 256 * 256;
    if (want <= 0 || want + static_lds > per_block)
        return fail(CDI_E_INVALID, "blocks_per_cu %d needs %d bytes of LDS per workgroup (limit %d)", k,
                    want + static_lds, per_block);
    // k + 1 workgroups must not fit
    if ((k + 1) * (want + static_lds) <= per_cu) want += 256;
    *pad = want;
    return CDI_OK;
}

int d2h(cdi_solver *s, void *dst, const void *src, uint64_t bytes)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CDI_OK;
}

int h2d(cdi_solver *s, void *dst, const void *src, uint64_t bytes)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CDI_OK;
}

// d planes of stride P in internal node order on the device <-> d planes of
// N_f in lexicographic (public) order on the host
int planes_d2h(cdi_solver *s, float *host, const float *dev, int d)
{
    HIPCHK(launch_permute(dev, s->node.xfer, s->vox.lex2int, (int)s->nf, s->P, d, 1, s->stream));
    HIPCHK(hipMemcpyAsync(host, s->node.xfer, 4ull * s->nf * d, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CDI_OK;
}

int planes_h2d(cdi_solver *s, float *dev, const float *host, int d)
{
    HIPCHK(hipMemcpyAsync(s->node.xfer, host, 4ull * s->nf * d, hipMemcpyHostToDevice, s->stream));
    HIPCHK(launch_permute(s->node.xfer, dev, s->vox.lex2int, (int)s->nf, s->P, d, 0, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return CDI_OK;
}

}  // namespace

extern "C" {

const char *cdi_last_error(void) { return g_err; }

int cdi_bandwidth_probe(int32_t mode, void *dst, const void *src, uint64_t bytes, uint32_t value, void *stream)
{
    if (mode != CDI_PROBE_COPY && mode != CDI_PROBE_READ && mode != CDI_PROBE_FILL)
        return fail(CDI_E_INVALID, "unknown probe mode %d", mode);
    if (!dst || (mode != CDI_PROBE_FILL && !src)) return fail(CDI_E_INVALID, "null buffer");
    if (bytes % 16 || ((uintptr_t)dst | (uintptr_t)(src ? src : dst)) % 16)
        return fail(CDI_E_INVALID, "buffers must be 16-byte aligned and bytes a multiple of 16");
    const uint64_t out_bytes = mode == CDI_PROBE_READ ? 16 * ((bytes + kStreamReadBlock - 1) / kStreamReadBlock) : bytes;
    if (mode != CDI_PROBE_FILL && bytes && (const uint8_t *)src < (uint8_t *)dst + out_bytes &&
        (uint8_t *)dst < (const uint8_t *)src + bytes)
        return fail(CDI_E_INVALID, "source and destination overlap");
    const int k = mode == CDI_PROBE_COPY ? kStreamCopy : mode == CDI_PROBE_READ ? kStreamRead : kStreamFill;
    HIPCHK(launch_stream(k, dst, src, bytes, value, (hipStream_t)stream));
    return CDI_OK;
}

int cdi_struct_size(const char *name, uint64_t *bytes)
{
    if (!name || !bytes) return fail(CDI_E_INVALID, "null argument");
    static const struct {
        const char *name;
        uint64_t size;
    } table[] = {{"cdi_geometry", sizeof(cdi_geometry)},     {"cdi_params", sizeof(cdi_params)},
                 {"cdi_plan_info", sizeof(cdi_plan_info)},   {"cdi_solver_info", sizeof(cdi_solver_info)},
                 {"cdi_tuning", sizeof(cdi_tuning)},         {"cdi_potential", sizeof(cdi_potential)},
                 {"cdi_potential_result", sizeof(cdi_potential_result)}, {"cdi_diag", sizeof(cdi_diag)}};
    for (const auto &e : table)
        if (std::strcmp(e.name, name) == 0) {
            *bytes = e.size;
            return CDI_OK;
        }
    return fail(CDI_E_INVALID, "unknown struct %s", name);
}

int cdi_flow_check(const cdi_geometry *geom, const cdi_params *params, double max_drho, double *drho_estimate)
{
    int rc = check_geometry(geom);
    if (rc) return rc;
    if ((rc = check_params(params)) != CDI_OK) return rc;
    if (!(max_drho >= 0)) return fail(CDI_E_INVALID, "bad max_drho");
    const double limit = max_drho > 0 ? max_drho : 0.5;
    double est = 0.0;
    if (params->drive == CDI_INLET_OUTLET) {
        // porosity and fluid-solid surface per volume of the electrode region
        const double a = geom->r_min, b = geom->r_max, phi_t = geom->porosity;
        double phi = phi_t, sv = 0.0;
        if (geom->kind == CDI_USER_LABELS) {
            const int nx = geom->nx, ny = geom->ny, nz = geom->dim == 2 ? 1 : geom->nz;
            int64_t fluid = 0, faces = 0, vol = 0;
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y)
                    for (int x = geom->buffer_x; x < nx - geom->buffer_x; ++x) {
                        const uint8_t l = geom->user_labels[((int64_t)z * ny + y) * nx + x];
                        ++vol;
                        if (l != 0) continue;
                        ++fluid;
                        const int d3 = geom->dim == 3;
                        const int nbs[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, d3}, {0, 0, -d3}};
                        for (int k = 0; k < (d3 ? 6 : 4); ++k) {
                            const int xn = x + nbs[k][0], yn = (y + nbs[k][1] + ny) % ny, zn = (z + nbs[k][2] + nz) % nz;
                            if (geom->user_labels[((int64_t)zn * ny + yn) * nx + xn] != 0) ++faces;
                        }
                    }
            phi = vol ? (double)fluid / vol : 1.0;
            sv = vol ? (double)faces / vol : 0.0;
        } else if (geom->kind == CDI_SPHERES || geom->kind == CDI_FIBRES) {
            // Boolean models: surface per volume phi (-ln phi) times 3 E[r^2]/E[r^3]
            // (spheres) or 2 / r (cylinders)
            const double er2 = b > a ? (b * b * b - a * a * a) / (3 * (b - a)) : a * a;
            const double er3 = b > a ? (b * b * b * b - a * a * a * a) / (4 * (b - a)) : a * a * a;
            sv = geom->kind == CDI_SPHERES ? 3.0 * phi * -std::log(phi) * er2 / er3 : 2.0 * phi * -std::log(phi) / a;
        } else {  // non-overlapping disks: perimeter per area (1 - phi) 2 E[r] / E[r^2]
            const double er2 = b > a ? (b * b * b - a * a * a) / (3 * (b - a)) : a * a;
            sv = (1.0 - phi) * 2.0 * 0.5 * (a + b) / er2;
        }
        if (sv > 0 && phi > 0 && phi < 1) {
            // Kozeny-Carman permeability and Darcy's law over the electrode's length
            const double k = phi * phi * phi / (5.0 * sv * sv);
            const double nu = (params->tau - 0.5) / 3.0;
            const double len = geom->nx - 2.0 * geom->buffer_x;
            est = 3.0 * nu * std::fabs(params->u_in) * len / k;  // rho = 3 p in lattice units
        }
    }
    if (drho_estimate) *drho_estimate = est;
    if (est > limit)
        return fail(CDI_E_UNSTABLE,
                    "the steady flow needs a density drop of about %.2g across the electrode (Kozeny-Carman), "
                    "beyond %.2g: outside the weakly compressible range of the lattice Boltzmann method", est, limit);
    g_err[0] = 0;
    return CDI_OK;
}

int cdi_plan(const cdi_geometry *geom, const cdi_params *params, cdi_plan_info *out)
{
    int rc = check_geometry(geom);
    if (rc) return rc;
    if (params && (rc = check_params(params)) != CDI_OK) return rc;
    if (!out) return fail(CDI_E_INVALID, "out is NULL");
    const int64_t nvox = geom_nvox(geom);
    int64_t nprims = 0, nf_est = -1;
    if (geom->kind == CDI_DISKS) {
        std::vector<geomgen_prim> pr;
        if ((rc = make_prims(geom, pr, &nf_est)) != CDI_OK) return rc;
        nprims = (int64_t)pr.size();
    } else if (geom->kind == CDI_SPHERES) {
        nprims = geomgen_sphere_count(geom->nx, geom->ny, geom->nz, geom->buffer_x, geom->porosity,
                                      geom->r_min, geom->r_max);
        if (nprims < 0) return fail(CDI_E_INVALID, "sphere generator rejected the geometry");
        nf_est = (int64_t)llround(geom->porosity * (double)nvox);
    } else if (geom->kind == CDI_FIBRES) {
        std::vector<geomgen_fibre> fb;
        if ((rc = make_fibres(geom, fb)) != CDI_OK) return rc;
        nprims = (int64_t)fb.size();
        nf_est = (int64_t)llround(geom->porosity * (double)nvox);
    } else {
        nf_est = 0;
        for (int64_t v = 0; v < nvox; ++v) nf_est += geom->user_labels[v] == 0;
    }
    out->n_vox = nvox;
    out->n_prims = nprims;
    out->n_fluid_est = nf_est;
    out->vox_bytes = vox_layout(nullptr, geom, nprims).bytes;
    const int dim = geom->dim;
    const int st = params ? params->precision : CDI_FP32;
    const int pull = params ? params->streaming == CDI_STREAM_PULL : 0;
    const int Q = dim == 2 ? 9 : 19;
    // the per-node arrays of node_layout: populations, moments, flux (two
    // sets), previous velocity and density, concentrations and remainders,
    // scratch, host staging, potential and the neighbour list; plus about
    // 1 B for the per-tile sums and the schedule
    out->node_bytes_per_fluid = (uint64_t)Q * pop_bytes(st) * (pull ? 2 : 1) + (moment_buffers(st) ? 32 : 0) +
                                8ull * dim + 4ull * (dim + 1) + 16 + 8 + 4ull * (1 + dim) + 16 + 4 +
                                4ull * (Q - 1) + 1;
    g_err[0] = 0;
    return CDI_OK;
}

int cdi_build_geometry(const cdi_geometry *geom, void *vox_ws, uint64_t vox_ws_bytes, void *stream,
                       int64_t *n_fluid)
{
    int rc = check_geometry(geom);
    if (rc) return rc;
    if (!vox_ws || ((uintptr_t)vox_ws % kAlign)) return fail(CDI_E_BUFFER, "vox_ws NULL or not 256-byte aligned");
    const int64_t nvox = geom_nvox(geom);
    std::vector<geomgen_prim> pr;
    std::vector<geomgen_fibre> fb;
    if (geom->kind == CDI_FIBRES) {
        if ((rc = make_fibres(geom, fb)) != CDI_OK) return rc;
    } else if ((rc = make_prims(geom, pr, nullptr)) != CDI_OK) {
        return rc;
    }
    const int64_t nprims = geom->kind == CDI_FIBRES ? (int64_t)fb.size() : (int64_t)pr.size();
    VoxLayout L = vox_layout(vox_ws, geom, nprims);
    if (vox_ws_bytes < L.bytes) return fail(CDI_E_BUFFER, "vox_ws too small: %llu < %llu",
                                            (unsigned long long)vox_ws_bytes, (unsigned long long)L.bytes);
    hipStream_t st = (hipStream_t)stream;
    const int nz = geom->dim == 2 ? 1 : geom->nz;
    if (geom->kind == CDI_USER_LABELS) {
        HIPCHK(hipMemcpyAsync(L.labels, geom->user_labels, (size_t)nvox, hipMemcpyHostToDevice, st));
    } else if (geom->kind == CDI_FIBRES) {
        if (nprims > 0)
            HIPCHK(hipMemcpyAsync(L.prims, fb.data(), sizeof(geomgen_fibre) * (size_t)nprims,
                                  hipMemcpyHostToDevice, st));
        HIPCHK(launch_init_labels(L.labels, geom->nx, geom->ny, nz, 0, st));
        HIPCHK(launch_voxelize_fibres(L.labels, L.prims, nprims, geom->nx, geom->ny, nz, geom->buffer_x, st));
    } else {
        if (nprims > 0)
            HIPCHK(hipMemcpyAsync(L.prims, pr.data(), sizeof(geomgen_prim) * (size_t)nprims,
                                  hipMemcpyHostToDevice, st));
        HIPCHK(launch_init_labels(L.labels, geom->nx, geom->ny, nz, geom->dim == 2 && geom->walls_y, st));
        HIPCHK(launch_voxelize(L.labels, L.prims, nprims, geom->dim, geom->nx, geom->ny, nz,
                               geom->walls_y, geom->buffer_x, st));
    }
    HIPCHK(launch_compact(L.labels, nvox, L.map, L.fluid, L.blk, L.nfluid, st));
    HIPCHK(launch_compact_bricks(L.labels, L.map, geom->nx, geom->ny, nz, L.bk, L.imap, L.ifluid,
                                 L.lex2int, L.blk2, L.nfluid2, st));
    int64_t nf[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&nf[0], L.nfluid, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&nf[1], L.nfluid2, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (nf[0] != nf[1]) return fail(CDI_E_DEVICE, "fluid counts disagree (%lld vs %lld)", (long long)nf[0],
                                    (long long)nf[1]);
    if (n_fluid) *n_fluid = nf[0];
    if (nf[0] == 0) return fail(CDI_E_GEOMETRY, "geometry has no fluid voxel");
    g_err[0] = 0;
    return CDI_OK;
}

int cdi_node_bytes(const cdi_geometry *geom, const cdi_params *params, int64_t n_fluid, uint64_t *bytes)
{
    int rc = check_geometry(geom);
    if (rc) return rc;
    if ((rc = check_params(params)) != CDI_OK) return rc;
    if (!bytes || n_fluid <= 0) return fail(CDI_E_INVALID, "bad n_fluid or bytes pointer");
    const int64_t P = (n_fluid + kTile - 1) / kTile * kTile;
    *bytes = node_layout(nullptr, geom->dim, params->precision, params->streaming == CDI_STREAM_PULL, P,
                         (int64_t)geom->ny * (geom->dim == 2 ? 1 : geom->nz), diag_doubles(geom, P), geom->nx).bytes;
    return CDI_OK;
}

int cdi_flow_init(const cdi_geometry *geom, const cdi_params *params, void *vox_ws, uint64_t vox_ws_bytes,
                  void *node_ws, uint64_t node_ws_bytes, int64_t n_fluid, void *stream, cdi_solver **out)
{
    int rc = check_geometry(geom);
    if (rc) return rc;
    if ((rc = check_params(params)) != CDI_OK) return rc;
    if (!out) return fail(CDI_E_INVALID, "out is NULL");
    if (!vox_ws || !node_ws || ((uintptr_t)vox_ws % kAlign) || ((uintptr_t)node_ws % kAlign))
        return fail(CDI_E_BUFFER, "workspace NULL or not 256-byte aligned");
    const int64_t nvox = geom_nvox(geom);
    if (n_fluid <= 0 || n_fluid > nvox) return fail(CDI_E_INVALID, "bad n_fluid");
    // the primitive count only sizes the tail of the voxel workspace
    int64_t nprims = 0;
    if (geom->kind == CDI_DISKS) {
        std::vector<geomgen_prim> pr;
        if ((rc = make_prims(geom, pr, nullptr)) != CDI_OK) return rc;
        nprims = (int64_t)pr.size();
    } else if (geom->kind == CDI_SPHERES) {
        nprims = geomgen_sphere_count(geom->nx, geom->ny, geom->nz, geom->buffer_x, geom->porosity,
                                      geom->r_min, geom->r_max);
    } else if (geom->kind == CDI_FIBRES) {
        std::vector<geomgen_fibre> fb;
        if ((rc = make_fibres(geom, fb)) != CDI_OK) return rc;
        nprims = (int64_t)fb.size();
    }
    VoxLayout V = vox_layout(vox_ws, geom, nprims);
    if (vox_ws_bytes < V.bytes) return fail(CDI_E_BUFFER, "vox_ws too small");
    const int st_kind = params->precision;
    const int64_t P = (n_fluid + kTile - 1) / kTile * kTile;
    // per-node arrays are addressed with 32-bit byte offsets (16-byte moments)
    // (the two planes of a direction and its opposite from one base: 2P elements)
    if (P * (st_kind == kF32 ? 8 : moment_buffers(st_kind) ? 16 : 4) > 4294967295LL)
        return fail(CDI_E_INVALID,
                    "too many fluid nodes for one instance (limit 2^29 FP32, 2^30 FP16, 2^28 with moment buffers)");
    NodeLayout N = node_layout(node_ws, geom->dim, st_kind, params->streaming == CDI_STREAM_PULL, P,
                               (int64_t)geom->ny * (geom->dim == 2 ? 1 : geom->nz), diag_doubles(geom, P),
                               geom->nx);
    if (node_ws_bytes < N.bytes) return fail(CDI_E_BUFFER, "node_ws too small: %llu < %llu",
                                             (unsigned long long)node_ws_bytes, (unsigned long long)N.bytes);
    if (params->np_x_bc != CDI_NPX_PERIODIC && params->np_x_bc != CDI_NPX_CLOSED && geom->nx < 2)
        return fail(CDI_E_INVALID, "nx too small");

    cdi_solver *s = new (std::nothrow) cdi_solver();
    if (!s) return fail(CDI_E_INVALID, "out of host memory");
    s->geom = *geom;
    s->geom.user_labels = nullptr;
    s->params = *params;
    s->dim = geom->dim;
    s->Q = geom->dim == 2 ? 9 : 19;
    s->st = st_kind;
    s->mb = moment_buffers(st_kind);
    s->pull = params->streaming == CDI_STREAM_PULL && st_kind != kMom;
    s->inout = params->drive == CDI_INLET_OUTLET;
    s->nvox = nvox;
    s->nf = n_fluid;
    s->P = (int)P;
    s->ntiles = (int)(P / kTile);
    s->stream = (hipStream_t)stream;
    if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
    s->vox = V;
    s->node = N;
    s->porosity = (double)n_fluid / (double)nvox;
    s->ka = params->no_adsorption ? 0.0  // a blocking electrode
            : params->Ka > 0      ? params->Ka
                                  : (4.28e-3 / 1.03e-2) * params->u_in / s->porosity;
    for (int k = 0; k < 2; ++k) s->keff[k] = s->ka * params->D[k] / (params->D[k] + 0.5 * s->ka);

    Grid &g = s->g;
    g.nx = geom->nx;
    g.ny = geom->ny;
    g.nz = geom->dim == 2 ? 1 : geom->nz;
    g.n_f = (int)n_fluid;
    g.P = (int)P;
    g.periodic_x = params->drive == CDI_BODY_FORCE;
    g.inout = params->drive == CDI_INLET_OUTLET;
    g.bk = V.bk;
    g.fluid = V.ifluid;
    g.map = V.imap;
    g.sched = nullptr;
    g.nbr = nullptr;
    g.lds_pad = 0;
    g.stage_odd = stage_odd_for(0, s->ntiles);
    Phys &p = s->p;
    p.omega = (float)(1.0 / params->tau);
    p.fcoef = (float)(1.0 - 0.5 / params->tau);
    for (int a = 0; a < 3; ++a) p.F[a] = (float)params->body_force[a];
    p.forced = params->drive == CDI_BODY_FORCE;
    p.linear_eq = params->equilibrium == CDI_EQ_LINEAR;
    for (int k = 0; k < 2; ++k) {
        p.D[k] = (float)params->D[k];
        p.invD[k] = (float)(1.0 / params->D[k]);
        p.z[k] = (float)params->z[k];
        p.keff[k] = (float)s->keff[k];
    }
    p.c0 = (float)params->c0;
    p.c_out = (float)params->c_out;
    p.u_in = (float)params->u_in;
    p.rho_out = (float)params->rho_out;
    p.dpsi_dx = (float)(params->dpsi_vt / geom->nx);
    p.npx = params->np_x_bc;
    p.dt = (float)(1.0 / params->np_substeps);
    p.psi = params->psi_field ? N.psi : nullptr;  // filled below in internal order
    p.hs = kHalfScale;
    p.hs_inv = 1.f / kHalfScale;

    hipStream_t st = s->stream;
    int err = CDI_OK;
    auto chk = [&](hipError_t e) {
        if (e != hipSuccess && err == CDI_OK) err = fail(CDI_E_DEVICE, "init: %s", hipGetErrorString(e));
    };
    // rest state: f - w_i = 0 (FP32) / zero deviations and zero moments (FP16, moments)
    if (s->mb) {
        if (s->st == kF16) chk(launch_fill_u32((uint32_t *)N.f, 0u, (int64_t)s->Q * P / 2, st));
        if (s->st == kF16 && s->pull) chk(launch_fill_u32((uint32_t *)N.f2, 0u, (int64_t)s->Q * P / 2, st));
        chk(launch_fill_f32((float *)N.M[0], 0.f, 4 * P, st));
        chk(launch_fill_f32((float *)N.M[1], 0.f, 4 * P, st));
    } else if (s->st == kH16) {
        chk(launch_fill_u32((uint32_t *)N.f, 0u, (int64_t)s->Q * P / 2, st));
        if (s->pull) chk(launch_fill_u32((uint32_t *)N.f2, 0u, (int64_t)s->Q * P / 2, st));
    } else {
        chk(launch_fill_f32((float *)N.f, 0.f, (int64_t)s->Q * P, st));
        if (s->pull) chk(launch_fill_f32((float *)N.f2, 0.f, (int64_t)s->Q * P, st));
    }
    chk(launch_fill_f32(N.j[0], 0.f, (int64_t)s->dim * P, st));
    chk(launch_fill_f32(N.j[1], 0.f, (int64_t)s->dim * P, st));
    chk(launch_fill_f32(N.ubuf, 0.f, (int64_t)(s->dim + 1) * P, st));
    if (N.rref[0]) {  // rest state: no reference deviation yet
        chk(launch_fill_f32(N.rref[0], 0.f, geom->nx, st));
        chk(launch_fill_f32(N.rref[1], 0.f, geom->nx, st));
    }
    if (params->psi_field)
        chk(launch_permute(params->psi_field, N.psi, V.lex2int, (int)n_fluid, (int)P, 1, 0, st));
    chk(launch_fill_f32(N.C[0], (float)params->c0, 2 * P, st));
    chk(launch_fill_f32(N.C[1], (float)params->c0, 2 * P, st));
    chk(launch_fill_u32((uint32_t *)N.Clo[0], 0u, P, st));
    chk(launch_fill_u32((uint32_t *)N.Clo[1], 0u, P, st));
    chk(launch_fill_f64(N.acc, 0.0, 8ll * s->ntiles, st));
    chk(launch_fill_f64(N.resid, 0.0, 2ll * s->ntiles, st));
    chk(launch_build_nbr(s->dim, g, N.nbr, st));
    // the ion-carrying steps read their neighbours from the list by default
    g.nbr = N.nbr;
    s->tuning.nbr_list = 1;
    if (err == CDI_OK) err = build_schedule(s, 0, 0);  // bricks already give locality
    if (err != CDI_OK) {
        delete s;
        return err;
    }
    *out = s;
    g_err[0] = 0;
    return CDI_OK;
}

int cdi_destroy(cdi_solver *s)
{
    delete s;
    return CDI_OK;
}

int cdi_get_info(const cdi_solver *s, cdi_solver_info *out)
{
    if (!s || !out) return fail(CDI_E_INVALID, "NULL argument");
    out->n_vox = s->nvox;
    out->n_fluid = s->nf;
    out->dim = s->dim;
    out->q = s->Q;
    out->nx = s->g.nx;
    out->ny = s->g.ny;
    out->nz = s->g.nz;
    out->precision = s->params.precision;
    out->flow_steps = s->flow_steps;
    out->np_steps = s->np_steps;
    out->ka = s->ka;
    out->keff[0] = s->keff[0];
    out->keff[1] = s->keff[1];
    out->porosity = s->porosity;
    return CDI_OK;
}

int cdi_flow_steps(cdi_solver *s, int64_t n)
{
    if (!s || n < 0) return fail(CDI_E_INVALID, "bad arguments");
    for (int64_t k = 0; k < n; ++k) {
        int rc = step_once(s, 1, 0, 0);
        if (rc) return rc;
    }
    if (n > 0) s->jstate = J_INVALID;
    return CDI_OK;
}

int cdi_flow_step_to_steady(cdi_solver *s, double tol, int64_t max_steps, int32_t check_every,
                            int64_t *steps_out, double *residual_out)
{
    if (!s || max_steps < 0 || check_every < 2) return fail(CDI_E_INVALID, "bad arguments");
    const int K = check_every;
    double r = INFINITY, best = INFINITY;
    int since_best = 0;
    int status = CDI_E_NOT_CONVERGED;
    int64_t t = 0;
    for (; t < max_steps; ++t) {
        int flags = 0;
        if (!s->mb && t % K == K - 1) flags |= kStoreU;
        const bool check = t > 0 && t % K == 0;
        if (check) flags |= kResid;
        int rc = step_once(s, 1, 0, flags);
        if (rc) return rc;
        if ((flags & kStoreU) && s->node.rref[0]) {
            // FP32: renew the plane references from this state's rho - 1 (stored
            // with u); the next step reads with the old table and writes with the new
            HIPCHK(launch_plane_means(s->g, s->node.ubuf + (size_t)s->dim * s->P, s->node.rref[s->rcur ^ 1],
                                      s->stream));
            s->rpend = 1;
            s->rlive = 1;
        }
        if (check) {
            HIPCHK(launch_reduce_tiles(s->node.resid, s->ntiles, 2, 2, s->node.red, s->stream));
            double h[2];
            if ((rc = d2h(s, h, s->node.red, 16)) != CDI_OK) return rc;
            r = std::sqrt(h[0]) / std::sqrt(h[1]);
            if (!std::isfinite(r)) {
                status = fail(CDI_E_DIVERGED, "residual is not finite");
                ++t;
                break;
            }
            if (r <= tol) {
                status = CDI_OK;
                ++t;
                break;
            }
            if (r < best) {
                best = r;
                since_best = 0;
            } else if (++since_best >= 10) {
                status = CDI_STAGNATED;
                ++t;
                break;
            }
        }
    }
    s->jstate = J_INVALID;
    if (steps_out) *steps_out = t;
    if (residual_out) *residual_out = r;
    if (status == CDI_E_NOT_CONVERGED) fail(CDI_E_NOT_CONVERGED, "max_steps reached, residual %g", r);
    return status;
}

// fused steps between two checks of the positivity bound within one call
constexpr int64_t kFusedRecheck = 256;

int cdi_np_step(cdi_solver *s, int64_t nsteps, int32_t fused_flow)
{
    if (!s || nsteps < 0) return fail(CDI_E_INVALID, "bad arguments");
    if (fused_flow && s->params.np_substeps != 1) return fail(CDI_E_INVALID, "fused steps need np_substeps = 1");
    if (nsteps == 0) return CDI_OK;
    double worst = 0;
    int rc = check_stability(s, &worst);
    if (rc) return rc;
    if (!(worst <= 1.0))
        return fail(CDI_E_UNSTABLE, "positivity bound violated: dt * sum(outflow coefficients) = %g > 1", worst);
    for (int64_t k = 0; k < nsteps; ++k) {
        if (fused_flow && k > 0 && k % kFusedRecheck == 0) {
            // the flow keeps changing under fused steps: the bound is taken again
            s->jstate = s->mb ? J_IN_M : J_VALID;
            if ((rc = check_stability(s, &worst)) != CDI_OK) return rc;
            if (!(worst <= 1.0))
                return fail(CDI_E_UNSTABLE, "positivity bound violated after %lld fused steps: %g > 1",
                            (long long)k, worst);
        }
        if (fused_flow) {
            const int flags = (s->mb && k > 0) ? kJFromM : 0;
            if ((rc = step_once(s, 1, 1, flags)) != CDI_OK) return rc;
        } else {
            for (int m = 0; m < s->params.np_substeps; ++m)
                if ((rc = step_once(s, 0, 1, 0)) != CDI_OK) return rc;
        }
        s->np_steps++;
    }
    if (fused_flow) s->jstate = s->mb ? J_IN_M : J_VALID;
    return CDI_OK;
}

int cdi_adsorbed_total(cdi_solver *s, double out[2])
{
    if (!s || !out) return fail(CDI_E_INVALID, "NULL argument");
    HIPCHK(launch_reduce_tiles(s->node.acc, s->ntiles, 8, 2, s->node.red, s->stream));
    return d2h(s, out, s->node.red, 16);
}

int cdi_mass_balance(cdi_solver *s, double out[8])
{
    if (!s || !out) return fail(CDI_E_INVALID, "NULL argument");
    HIPCHK(launch_reduce_tiles(s->node.acc, s->ntiles, 8, 6, s->node.red, s->stream));
    HIPCHK(launch_mass(s->g, s->node.C[s->ccur], s->node.Clo[s->ccur], s->node.part, s->node.red + 8, s->stream));
    double h[10];
    int rc = d2h(s, h, s->node.red, 80);
    if (rc) return rc;
    for (int sp = 0; sp < 2; ++sp) {
        out[4 * sp + 0] = h[8 + sp];
        out[4 * sp + 1] = h[0 + sp];
        out[4 * sp + 2] = h[2 + sp];
        out[4 * sp + 3] = h[4 + sp];
    }
    return CDI_OK;
}

int cdi_copy_labels(cdi_solver *s, uint8_t *labels)
{
    if (!s || !labels) return fail(CDI_E_INVALID, "NULL argument");
    return d2h(s, labels, s->vox.labels, (uint64_t)s->nvox);
}

int cdi_copy_fluid_index(cdi_solver *s, int32_t *map, int32_t *fluid)
{
    if (!s) return fail(CDI_E_INVALID, "NULL argument");
    int rc = CDI_OK;
    if (map && (rc = d2h(s, map, s->vox.map, 4ull * s->nvox)) != CDI_OK) return rc;
    if (fluid && (rc = d2h(s, fluid, s->vox.fluid, 4ull * s->nf)) != CDI_OK) return rc;
    return CDI_OK;
}

int cdi_copy_velocity(cdi_solver *s, float *u)
{
    if (!s || !u) return fail(CDI_E_INVALID, "NULL argument");
    HIPCHK(launch_moments(s->dim, s->st, stream_arg(s), s->flow_steps > 0, s->g, s->p, cur_pops(s),
                          s->mb ? s->node.M[s->mcur] : nullptr, cur_rref(s), nullptr, s->node.tmp, nullptr, s->stream));
    return planes_d2h(s, u, s->node.tmp, s->dim);
}

int cdi_copy_density(cdi_solver *s, float *rho)
{
    if (!s || !rho) return fail(CDI_E_INVALID, "NULL argument");
    HIPCHK(launch_moments(s->dim, s->st, stream_arg(s), s->flow_steps > 0, s->g, s->p, cur_pops(s),
                          s->mb ? s->node.M[s->mcur] : nullptr, cur_rref(s), s->node.tmp, nullptr, nullptr, s->stream));
    return planes_d2h(s, rho, s->node.tmp, 1);
}

int cdi_copy_np_velocity(cdi_solver *s, float *j)
{
    if (!s || !j) return fail(CDI_E_INVALID, "NULL argument");
    int rc = ensure_j(s);
    if (rc) return rc;
    return planes_d2h(s, j, s->node.j[s->jcur], s->dim);
}

int cdi_set_np_velocity(cdi_solver *s, const float *j)
{
    if (!s || !j) return fail(CDI_E_INVALID, "NULL argument");
    int rc = planes_h2d(s, s->node.j[s->jcur], j, s->dim);
    if (rc) return rc;
    s->jstate = J_VALID;
    return CDI_OK;
}

int cdi_copy_concentration(cdi_solver *s, float *c)
{
    if (!s || !c) return fail(CDI_E_INVALID, "NULL argument");
    return planes_d2h(s, c, s->node.C[s->ccur], 2);
}

int cdi_set_concentration(cdi_solver *s, const float *c)
{
    if (!s || !c) return fail(CDI_E_INVALID, "NULL argument");
    int rc = planes_h2d(s, s->node.C[s->ccur], c, 2);
    if (rc) return rc;
    HIPCHK(launch_fill_u32((uint32_t *)s->node.Clo[s->ccur], 0u, s->P, s->stream));  // no remainders
    return CDI_OK;
}

// ------------------------------------------------------------ electric potential

namespace {

struct PotLayout {
    double *x, *r, *p, *p2, *q, *part, *state;
    float *xf, *rf, *pf, *pf2, *qf;
    uint8_t *dg;
    uint64_t bytes;
};

PotLayout pot_layout(void *ws, int P)
{
    Carver c(ws);
    PotLayout L;
    L.x = c.take<double>(8ull * P);
    L.r = c.take<double>(8ull * P);
    L.p = c.take<double>(8ull * P);
    L.p2 = c.take<double>(8ull * P);
    L.q = c.take<double>(8ull * P);
    L.xf = c.take<float>(4ull * P);
    L.rf = c.take<float>(4ull * P);
    L.pf = c.take<float>(4ull * P);
    L.pf2 = c.take<float>(4ull * P);
    L.qf = c.take<float>(4ull * P);
    L.dg = c.take<uint8_t>((uint64_t)P);
    L.part = c.take<double>(8ull * pot_part_doubles());
    L.state = c.take<double>(8ull * kStSlots);
    L.bytes = c.off;
    return L;
}

int check_potential(const cdi_solver *s, const cdi_potential *pc)
{
    if (!pc) return fail(CDI_E_INVALID, "potential settings are NULL");
    for (int e = 0; e < 2; ++e)
        if (pc->x_bc[e] < CDI_PSIX_DIRICHLET || pc->x_bc[e] > CDI_PSIX_PERIODIC)
            return fail(CDI_E_INVALID, "bad x_bc[%d]", e);
    if ((pc->x_bc[0] == CDI_PSIX_PERIODIC) != (pc->x_bc[1] == CDI_PSIX_PERIODIC))
        return fail(CDI_E_INVALID, "a periodic potential needs both x ends periodic");
    if (!(pc->tol >= 0) || pc->max_iter < 0 || pc->check_every < 0)
        return fail(CDI_E_INVALID, "bad tol, max_iter or check_every");
    if (!std::isfinite(pc->psi_electrode) || !std::isfinite(pc->psi_x[0]) || !std::isfinite(pc->psi_x[1]) ||
        !std::isfinite(pc->kappa2) || pc->kappa2 < 0)
        return fail(CDI_E_INVALID, "non-finite potential values or negative kappa2");
    if (8ull * s->P > 4294967295ull)
        return fail(CDI_E_INVALID, "too many fluid nodes for the potential solve (limit 2^29)");
    return CDI_OK;
}

int solve_potential(cdi_solver *s, const cdi_potential *pc, void *ws, uint64_t ws_bytes,
                    cdi_potential_result *out)
{
    int rc = check_potential(s, pc);
    if (rc) return rc;
    if (!ws || ((uintptr_t)ws % kAlign)) return fail(CDI_E_BUFFER, "workspace NULL or not 256-byte aligned");
    const PotLayout W = pot_layout(ws, s->P);
    if (ws_bytes < W.bytes) return fail(CDI_E_BUFFER, "potential workspace too small: %llu < %llu",
                                        (unsigned long long)ws_bytes, (unsigned long long)W.bytes);
    PotArgs a{};
    a.g = s->g;
    a.xbc[0] = pc->x_bc[0];
    a.xbc[1] = pc->x_bc[1];
    a.psi_e = pc->psi_electrode;
    a.psi_x[0] = pc->psi_x[0];
    a.psi_x[1] = pc->psi_x[1];
    a.src = pc->kappa2 / (2.0 * s->params.c0);
    a.z[0] = (float)s->params.z[0];
    a.z[1] = (float)s->params.z[1];
    a.C = s->node.C[s->ccur];
    a.psi0 = pc->warm_start ? s->p.psi : nullptr;
    a.x = W.x;
    a.r = W.r;
    a.p = W.p;
    a.p2 = W.p2;
    a.q = W.q;
    a.xf = W.xf;
    a.rf = W.rf;
    a.pf = W.pf;
    a.pf2 = W.pf2;
    a.qf = W.qf;
    // the neighbour list (built at init, one gather round trip fewer than the
    // map lookup; measured 6% faster per iteration on the 512^3 electrode)
    // follows the lattice's x ends: usable when the potential treats them alike
    const bool px = pc->x_bc[0] == CDI_PSIX_PERIODIC;
    a.nbr = px == (s->g.periodic_x != 0) ? s->node.nbr : nullptr;
    a.dg = W.dg;
    a.part = W.part;
    a.state = W.state;
    int G = 0;
    HIPCHK(pot_workgroups(s->dim, s->ntiles, a.nbr != nullptr, &G));
    HIPCHK(launch_pot_setup(s->dim, a, G, pc->tol, s->stream));
    double st[kStSlots];
    if ((rc = d2h(s, st, W.state, sizeof st)) != CDI_OK) return rc;
    if (st[kStNdir] == 0)
        return fail(CDI_E_INVALID, "no Dirichlet face (electrode or x end): the potential is not determined");
    int iters = 0, iters64 = 0, rounds = 0;
    if (st[kStBb] == 0) {  // b = 0: the solution is zero
        HIPCHK(launch_fill_f32(s->node.psi, 0.f, s->P, s->stream));
        st[kStDone] = kDoneConverged;
        st[kStRr] = 0;
    } else {
        // Mixed-precision refinement: each round forms the FP64 residual of x,
        // solves for the correction by CG on FP32 vectors (half the bytes of
        // an FP64 iteration) and adds it in FP64, until the FP64 residual
        // meets tol. A round that gains less than kPotRefineMinGain (the FP32
        // correction has reached its accuracy) hands over to CG on the FP64
        // vectors from the current x (pc->fp64: from the start). `iters`
        // counts CG iterations of both.
        const int chunk = pc->check_every > 0 ? pc->check_every : 32;
        bool f64 = pc->fp64 != 0;
        double prev = INFINITY;
        for (;;) {
            HIPCHK(launch_pot_refine(s->dim, a, G, pc->tol, f64 ? 0.0 : kPotInnerTol, f64, s->stream));
            if ((rc = d2h(s, st, W.state, sizeof st)) != CDI_OK) return rc;
            if (st[kStDone] != 0 || iters >= pc->max_iter) break;
            if (!f64 && st[kStRr] * kPotRefineMinGain * kPotRefineMinGain > prev) {
                f64 = true;
                HIPCHK(launch_pot_refine(s->dim, a, G, pc->tol, 0.0, true, s->stream));
                if ((rc = d2h(s, st, W.state, sizeof st)) != CDI_OK) return rc;
            }
            prev = st[kStRr];
            if (!f64) ++rounds;
            int kin = 0;
            while (st[kStDone] == 0 && iters < pc->max_iter) {
                const int n = std::min(chunk, pc->max_iter - iters);
                for (int k = kin; k < kin + n; ++k) HIPCHK(launch_pot_iter(s->dim, a, G, k, !f64, s->stream));
                HIPCHK(launch_pot_check(a, G, kin + n, s->stream));  // the next iteration's stop test
                if ((rc = d2h(s, st, W.state, sizeof st)) != CDI_OK) return rc;
                const int kend = st[kStDone] != 0 ? (int)st[kStIters] : kin + n;
                iters += kend - kin;
                if (f64) iters64 += kend - kin;
                kin = kend;
            }
            const bool bad = st[kStDone] == kDoneDiverged || st[kStDone] == kDoneBreakdown;
            if (f64) break;
            if (bad) {  // an FP32 correction that broke down is dropped; FP64 CG takes over
                prev = 0.0;
                continue;
            }
            HIPCHK(launch_pot_correct(a, s->stream));
        }
        if (st[kStDone] == kDoneDiverged || st[kStDone] == kDoneBreakdown)
            return fail(CDI_E_DIVERGED, "potential solve %s after %d iterations",
                        st[kStDone] == kDoneDiverged ? "diverged" : "broke down", iters);
        HIPCHK(launch_pot_store(a, s->node.psi, s->stream));
    }
    s->p.psi = s->node.psi;
    if (out) {
        out->iterations = iters;
        out->fp32_rounds = rounds;
        out->fp64_iterations = iters64;
        out->residual = st[kStBb] > 0 ? std::sqrt(st[kStRr] / st[kStBb]) : 0.0;
    }
    if (st[kStDone] == 0)
        return fail(CDI_E_NOT_CONVERGED, "potential solve: %d iterations, relative residual %g", iters,
                    std::sqrt(st[kStRr] / st[kStBb]));
    return CDI_OK;
}

}  // namespace

int cdi_potential_bytes(const cdi_solver *s, uint64_t *bytes)
{
    if (!s || !bytes) return fail(CDI_E_INVALID, "NULL argument");
    *bytes = pot_layout(nullptr, s->P).bytes;
    return CDI_OK;
}

int cdi_solve_potential(cdi_solver *s, const cdi_potential *pot, void *ws, uint64_t ws_bytes,
                        cdi_potential_result *out)
{
    if (!s) return fail(CDI_E_INVALID, "NULL solver");
    return solve_potential(s, pot, ws, ws_bytes, out);
}

}  // extern "C"

// ---------------------------------------------------------------- a solve without a caller workspace

// The workspace of cdi_solve_potential_noalloc: a file-scope device array,
// one copy per GPU the library runs on, held until the process ends. Host
// code never passes the array's name to a kernel or a copy (on the host it
// is a stand-in, not a device address): it looks up each device's address
// once, with that device current, and uses that.
static constexpr uint64_t kNoAllocScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (looked up on first use).
int scratch_on(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(CDI_E_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        if (cur != dev) HIPCHK(hipSetDevice(dev));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) HIPCHK(hipSetDevice(cur));
        if (e != hipSuccess || !ptr)
            return fail(CDI_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CDI_OK;
}

}  // namespace

extern "C" {

int cdi_solve_potential_noalloc(cdi_solver *s, const cdi_potential *pot, cdi_potential_result *out)
{
    if (!s) return fail(CDI_E_INVALID, "NULL solver");
    const uint64_t need = pot_layout(nullptr, s->P).bytes;
    if (need > kNoAllocScratchBytes)
        return fail(CDI_E_BUFFER, "potential solve needs %llu bytes of scratch, the library's holds %llu "
                                  "(use cdi_solve_potential with a workspace)",
                    (unsigned long long)need, (unsigned long long)kNoAllocScratchBytes);
    void *ws = nullptr;
    int rc = scratch_on(s->device, &ws);
    if (rc) return rc;
    // the solve initialises every workspace value it reads (setup kernel)
    return solve_potential(s, pot, ws, kNoAllocScratchBytes, out);
}

int cdi_np_step_coupled(cdi_solver *s, int64_t nsteps, int32_t fused_flow, const cdi_potential *pot,
                        int32_t every, void *ws, uint64_t ws_bytes)
{
    if (!s || nsteps < 0 || every < 1) return fail(CDI_E_INVALID, "bad arguments");
    for (int64_t k = 0; k < nsteps; k += every) {
        int rc = solve_potential(s, pot, ws, ws_bytes, nullptr);
        if (rc) return rc;
        if ((rc = cdi_np_step(s, std::min<int64_t>(every, nsteps - k), fused_flow)) != CDI_OK) return rc;
    }
    return CDI_OK;
}

int cdi_copy_potential(cdi_solver *s, float *psi)
{
    if (!s || !psi) return fail(CDI_E_INVALID, "NULL argument");
    if (s->p.psi) return planes_d2h(s, psi, s->node.psi, 1);
    // the ramp of the x coordinate
    std::vector<int32_t> fluid((size_t)s->nf);
    int rc = d2h(s, fluid.data(), s->vox.fluid, 4ull * s->nf);
    if (rc) return rc;
    for (int64_t n = 0; n < s->nf; ++n) {
        const int x = (int)(fluid[(size_t)n] % s->g.nx);
        psi[n] = (float)(s->params.dpsi_vt * (1.0 - (x + 0.5) / s->g.nx));
    }
    return CDI_OK;
}

// ------------------------------------------------------------ implicit ion transport

namespace {

struct NpsLayout {
    double *x, *r, *rh, *pv, *v, *sv, *t, *part, *state;
    float *dg;
    uint64_t bytes;
};

NpsLayout nps_layout(void *ws, int P)
{
    Carver c(ws);
    NpsLayout L;
    L.x = c.take<double>(16ull * P);
    L.r = c.take<double>(16ull * P);
    L.rh = c.take<double>(16ull * P);
    L.pv = c.take<double>(16ull * P);
    L.v = c.take<double>(16ull * P);
    L.sv = c.take<double>(16ull * P);
    L.t = c.take<double>(16ull * P);
    L.dg = c.take<float>(8ull * P);
    L.part = c.take<double>(8ull * nps_part_doubles());
    L.state = c.take<double>(8ull * kNsSlots);
    L.bytes = c.off;
    return L;
}

// One solve of (idt I + A) C' = idt C + b from C' = C; installs the result
// into the current concentrations unless it diverged.
int np_solve(cdi_solver *s, double idt, double tol, int32_t max_iter, void *ws, uint64_t ws_bytes, int *iters)
{
    if (!(tol >= 0) || max_iter < 0) return fail(CDI_E_INVALID, "bad tol or max_iter");
    if (!ws || ((uintptr_t)ws % kAlign)) return fail(CDI_E_BUFFER, "workspace NULL or not 256-byte aligned");
    if (16ull * s->P > 4294967295ull) return fail(CDI_E_INVALID, "too many fluid nodes for the ion solve (limit 2^28)");
    const NpsLayout W = nps_layout(ws, s->P);
    if (ws_bytes < W.bytes) return fail(CDI_E_BUFFER, "ion-solve workspace too small: %llu < %llu",
                                        (unsigned long long)ws_bytes, (unsigned long long)W.bytes);
    int rc = ensure_j(s);
    if (rc) return rc;
    NpsArgs a{};
    a.g = s->g;
    a.p = s->p;
    a.C = s->node.C[s->ccur];
    a.j = s->node.j[s->jcur];
    a.idt = idt;
    a.x = W.x;
    a.r = W.r;
    a.rh = W.rh;
    a.pv = W.pv;
    a.v = W.v;
    a.sv = W.sv;
    a.t = W.t;
    a.dg = W.dg;
    a.part = W.part;
    a.state = W.state;
    int G = 0;
    HIPCHK(nps_workgroups(s->dim, s->ntiles, &G));
    HIPCHK(launch_nps_setup(s->dim, a, G, tol, s->stream));
    double st[kNsSlots];
    if ((rc = d2h(s, st, W.state, sizeof st)) != CDI_OK) return rc;
    int k = 0;
    while (st[kNsDone] == 0 && k < max_iter) {
        const int n = std::min(32, max_iter - k);
        for (int q = k; q < k + n; ++q) HIPCHK(launch_nps_iter(s->dim, a, G, q, s->stream));
        k += n;
        HIPCHK(launch_nps_check(a, G, k, s->stream));
        if ((rc = d2h(s, st, W.state, sizeof st)) != CDI_OK) return rc;
    }
    *iters = (int)std::max(st[kNsIters], st[kNsIters + 1]);
    if (st[kNsDone] == 2.0) return fail(CDI_E_DIVERGED, "ion solve diverged or broke down after %d iterations", k);
    HIPCHK(launch_nps_store(a, s->node.C[s->ccur], s->node.Clo[s->ccur], s->stream));
    if (st[kNsDone] == 0)
        return fail(CDI_E_NOT_CONVERGED, "ion solve: %d iterations, relative residuals %g, %g", k,
                    std::sqrt(st[kNsRr] / std::max(st[kNsBb], 1e-300)),
                    std::sqrt(st[kNsRr + 1] / std::max(st[kNsBb + 1], 1e-300)));
    return CDI_OK;
}

}  // namespace

int cdi_np_solve_bytes(const cdi_solver *s, uint64_t *bytes)
{
    if (!s || !bytes) return fail(CDI_E_INVALID, "NULL argument");
    *bytes = nps_layout(nullptr, s->P).bytes;
    return CDI_OK;
}

int cdi_np_steady(cdi_solver *s, double tol, int32_t max_iter, void *ws, uint64_t ws_bytes, int32_t *iterations)
{
    if (!s) return fail(CDI_E_INVALID, "NULL solver");
    int it = 0;
    const int rc = np_solve(s, 0.0, tol, max_iter, ws, ws_bytes, &it);
    if (iterations) *iterations = it;
    return rc;
}

int cdi_np_implicit(cdi_solver *s, double dt, int64_t nsteps, double tol, int32_t max_iter, void *ws,
                    uint64_t ws_bytes, int32_t *iterations)
{
    if (!s || !(dt > 0) || nsteps < 0) return fail(CDI_E_INVALID, "bad arguments");
    int64_t total = 0;
    for (int64_t k = 0; k < nsteps; ++k) {
        int it = 0;
        const int rc = np_solve(s, 1.0 / dt, tol, max_iter, ws, ws_bytes, &it);
        total += it;
        if (rc) {
            if (iterations) *iterations = (int32_t)std::min<int64_t>(total, INT32_MAX);
            return rc;
        }
        // the new state's fluxes over dt enter the accumulators
        HIPCHK(launch_nps_rates(s->dim, s->g, s->p, s->node.C[s->ccur], s->node.j[s->jcur], dt, s->node.acc,
                                nullptr, nullptr, s->stream));
        s->np_steps++;
    }
    if (iterations) *iterations = (int32_t)std::min<int64_t>(total, INT32_MAX);
    return CDI_OK;
}

int cdi_np_rates(cdi_solver *s, double out[6])
{
    if (!s || !out) return fail(CDI_E_INVALID, "NULL argument");
    int rc = ensure_j(s);
    if (rc) return rc;
    HIPCHK(launch_nps_rates(s->dim, s->g, s->p, s->node.C[s->ccur], s->node.j[s->jcur], 1.0, nullptr,
                            s->node.diag, s->node.red, s->stream));
    double h[6];  // accumulator order: A_na, A_cl, In_na, In_cl, Out_na, Out_cl
    if ((rc = d2h(s, h, s->node.red, sizeof h)) != CDI_OK) return rc;
    for (int sp = 0; sp < 2; ++sp)
        for (int k = 0; k < 3; ++k) out[3 * sp + k] = h[2 * k + sp];
    return CDI_OK;
}

// ------------------------------------------------------------ diagnostics (Sec. 4)

int cdi_diagnostics(cdi_solver *s, cdi_diag *out)
{
    if (!s || !out) return fail(CDI_E_INVALID, "NULL argument");
    // u of the current populations into tmp (d planes), then the tile sums
    HIPCHK(launch_moments(s->dim, s->st, stream_arg(s), s->flow_steps > 0, s->g, s->p, cur_pops(s),
                          s->mb ? s->node.M[s->mcur] : nullptr, cur_rref(s), nullptr, s->node.tmp, nullptr, s->stream));
    HIPCHK(launch_diag(s->dim, s->g, s->node.tmp, s->node.nbr, s->node.diag, s->node.red, s->stream));
    double h[3];
    int rc = d2h(s, h, s->node.red, sizeof h);
    if (rc) return rc;
    out->n_surface = (int64_t)h[1];
    out->n_inlet = (int64_t)h[2];
    out->specific_surface = h[1] / (double)s->nvox;
    out->l_c = h[1] > 0 ? M_PI / out->specific_surface : INFINITY;
    out->U = h[0] / (double)s->nf;
    for (int k = 0; k < 2; ++k) {
        out->Pe[k] = out->U * out->l_c / s->params.D[k];
        out->Da[k] = s->ka * out->l_c / s->params.D[k];
    }
    return CDI_OK;
}

int cdi_profile_x(cdi_solver *s, double *out)
{
    if (!s || !out) return fail(CDI_E_INVALID, "NULL argument");
    const int nx = s->g.nx;
    double *res = s->node.diag + 3ll * nx * profile_chunks(s->g);
    HIPCHK(launch_profile_x(s->g, s->node.C[s->ccur], s->node.diag, res, s->stream));
    return d2h(s, out, res, 24ull * nx);
}

int cdi_salt_removal(const cdi_solver *s, const double bal0[8], const double bal1[8], int64_t nsteps,
                     int64_t n_inlet, double U, double out[4])
{
    if (!s || !bal0 || !bal1 || !out || nsteps <= 0 || n_inlet <= 0)
        return fail(CDI_E_INVALID, "bad arguments");
    const double c_in = s->params.c0;
    const double inflow = s->params.u_in * (double)n_inlet * (double)nsteps;  // volume that entered
    if (!(inflow > 0)) return fail(CDI_E_INVALID, "no inflow (u_in <= 0)");
    for (int k = 0; k < 2; ++k) {
        const double c_out = (bal1[4 * k + 3] - bal0[4 * k + 3]) / inflow;  // flux-weighted outlet concentration
        out[k] = (c_in - c_out) / c_in;
    }
    out[2] = 0.5 * (out[0] + out[1]);
    const double area = (double)s->g.ny * (double)s->g.nz;
    out[3] = U * area * out[2] * (double)nsteps / (double)s->nf;
    return CDI_OK;
}

int cdi_snapshot_bytes(cdi_solver *s, uint64_t *bytes)
{
    if (!s || !bytes) return fail(CDI_E_INVALID, "NULL argument");
    *bytes = sizeof(SnapHeader) + s->node.state_bytes;
    return CDI_OK;
}

int cdi_snapshot(cdi_solver *s, void *host, uint64_t bytes)
{
    if (!s || !host) return fail(CDI_E_INVALID, "NULL argument");
    if (bytes < sizeof(SnapHeader) + s->node.state_bytes) return fail(CDI_E_BUFFER, "snapshot buffer too small");
    SnapHeader h{kSnapMagic, s->node.state_bytes, s->parity, s->mcur, s->jcur, s->ccur, s->jstate, s->fcur,
                 s->p.psi != nullptr, s->rcur | (s->rpend << 1) | (s->rlive << 2), s->flow_steps, s->np_steps,
                 s->nf};
    std::memcpy(host, &h, sizeof h);
    return d2h(s, (uint8_t *)host + sizeof h, s->node.base, s->node.state_bytes);
}

int cdi_restore(cdi_solver *s, const void *host, uint64_t bytes)
{
    if (!s || !host) return fail(CDI_E_INVALID, "NULL argument");
    SnapHeader h;
    if (bytes < sizeof h) return fail(CDI_E_BUFFER, "snapshot too small");
    std::memcpy(&h, host, sizeof h);
    if (h.magic != kSnapMagic || h.bytes != s->node.state_bytes || h.nf != s->nf ||
        bytes < sizeof h + h.bytes)
        return fail(CDI_E_INVALID, "snapshot does not belong to this solver layout");
    int rc = h2d(s, s->node.base, (const uint8_t *)host + sizeof h, s->node.state_bytes);
    if (rc) return rc;
    s->parity = h.parity;
    s->fcur = h.fcur;
    s->mcur = h.mcur;
    s->jcur = h.jcur;
    s->ccur = h.ccur;
    s->jstate = h.jstate;
    s->rcur = h.rstate & 1;
    s->rpend = (h.rstate >> 1) & 1;
    s->rlive = (h.rstate >> 2) & 1;
    s->flow_steps = h.flow_steps;
    s->np_steps = h.np_steps;
    s->p.psi = h.psi_on ? s->node.psi : nullptr;
    return CDI_OK;
}

int cdi_set_tuning(cdi_solver *s, const cdi_tuning *t)
{
    if (!s || !t || t->blocks_per_cu < 0 || t->band_rows < 0 || t->columns < 0 || t->columns > 2 ||
        t->nbr_list < 0 || t->nbr_list > 1 || t->stage_odd < 0 || t->stage_odd > 2)
        return fail(CDI_E_INVALID, "bad tuning");
    int pad = 0;
    int rc = occupancy_pad(t->blocks_per_cu, &pad);
    if (rc) return rc;
    if (t->band_rows != s->tuning.band_rows || t->columns != s->tuning.columns ||
        ((t->band_rows > 0 || t->columns) && !s->g.sched))
        if ((rc = build_schedule(s, t->band_rows, t->columns)) != CDI_OK) return rc;
    s->g.lds_pad = pad;
    s->g.nbr = t->nbr_list ? s->node.nbr : nullptr;
    s->g.stage_odd = stage_odd_for(t->stage_odd, s->ntiles);
    s->tuning.stage_odd = t->stage_odd;
    s->tuning.nbr_list = t->nbr_list;
    s->tuning.blocks_per_cu = t->blocks_per_cu;
    return CDI_OK;
}

int cdi_get_tuning(const cdi_solver *s, cdi_tuning *t)
{
    if (!s || !t) return fail(CDI_E_INVALID, "NULL argument");
    *t = s->tuning;
    return CDI_OK;
}

int cdi_autotune(cdi_solver *s, int32_t steps, int32_t fused_flow, cdi_tuning *chosen, double *ms_per_step)
{
    if (!s || steps < 2) return fail(CDI_E_INVALID, "autotune needs a solver and steps >= 2");
    if (steps & 1) ++steps;  // whole AA step pairs
    uint64_t nb = 0;
    int rc = cdi_snapshot_bytes(s, &nb);
    if (rc) return rc;
    std::vector<uint8_t> snap(nb);
    if ((rc = cdi_snapshot(s, snap.data(), nb)) != CDI_OK) return rc;
    const cdi_tuning start = s->tuning;
    std::vector<cdi_tuning> cands;
    const int occ[] = {0, 2, 3, 4, 6};
    const int bands[] = {0, 8, 16, 32};
    for (int nl : {0, 1})
        for (int k : occ) {
            for (int r : bands)
                if (s->dim == 3 || r == 0) cands.push_back(cdi_tuning{k, r, 0, nl, 0});
            if (s->dim == 3) {
                cands.push_back(cdi_tuning{k, 0, 1, nl, 0});
                cands.push_back(cdi_tuning{k, 0, 2, nl, 0});
            }
        }
    // staged and unstaged odd steps, for the plain order and the default list
    for (int st : {1, 2}) cands.push_back(cdi_tuning{0, 0, 0, 1, st});
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    cdi_tuning best = start;
    float best_ms = INFINITY;
    for (const cdi_tuning &c : cands) {
        if (cdi_set_tuning(s, &c) != CDI_OK) continue;  // e.g. LDS cap not allowed here
        if ((rc = cdi_restore(s, snap.data(), nb)) != CDI_OK) break;
        // one untimed pair, then the timed steps
        rc = fused_flow ? cdi_np_step(s, 2, 1) : cdi_flow_steps(s, 2);
        if (rc) break;
        HIPCHK(hipEventRecord(e0, s->stream));
        rc = fused_flow ? cdi_np_step(s, steps, 1) : cdi_flow_steps(s, steps);
        if (rc) break;
        HIPCHK(hipEventRecord(e1, s->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int rc2 = cdi_set_tuning(s, &best);
    int rc3 = cdi_restore(s, snap.data(), nb);
    if (rc) return rc;
    if (rc2) return rc2;
    if (rc3) return rc3;
    if (chosen) *chosen = best;
    if (ms_per_step) *ms_per_step = best_ms / steps;
    return CDI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batches

namespace {

// Descriptor slots per batch: 0 first step, 1 odd leftover, 2-3 the two
// residual steps, 4-5 the step pair replayed from the captured graph. A call
// synchronises before rewriting any slot, so no slot is rewritten while a
// kernel of an earlier call may still read it.
constexpr int kSlots = 6;

}  // namespace

struct cdi_batch {
    std::vector<cdi_solver *> m;
    std::vector<int> tile_begin;
    int n = 0, dim = 0, st = 0, total_tiles = 0, cus = 0;
    int cap_n = 0, cap_tiles = 0;  // capacity of the workspace and staging (members, tiles)
    int workgroups_req = 0, blocks_per_cu = 0, lds_pad = 0;
    hipStream_t stream = nullptr;
    BatchInst *dinst = nullptr;  // device, kSlots * cap_n
    int2 *dtiles = nullptr;      // device, kSlots * cap_tiles (instance, tile), grouped by step class
    double *dred = nullptr;      // device, 2 per member slot
    BatchInst *hstage = nullptr; // pinned host, kSlots * cap_n
    int2 *htiles = nullptr;      // pinned host, kSlots * cap_tiles
    double *hworst = nullptr;    // pinned host, cap_n: the members' positivity bounds
    int cls_begin[kSlots][kClasses + 1] = {};
    std::vector<int> resid_valid;
    hipGraphExec_t exec = nullptr;
    std::vector<int> exec_sig;   // launch shape the graph was captured with
    hipEvent_t done = nullptr;
};

namespace {

uint64_t batch_layout(int n, int total_tiles, BatchInst **dinst, int2 **dtiles, double **dred, void *ws)
{
    Carver c(ws);
    BatchInst *a = c.take<BatchInst>(sizeof(BatchInst) * (uint64_t)kSlots * n);
    int2 *b = c.take<int2>(8ull * (uint64_t)kSlots * total_tiles);
    double *d = c.take<double>(16ull * n);
    if (dinst) *dinst = a;
    if (dtiles) *dtiles = b;
    if (dred) *dred = d;
    return c.off;
}

// Persistent grid size of a class launch over `count` tiles.
// Workgroups of a step class's launch over count tiles: the requested grid,
// else one per tile (what the autotuner picks at scale: on the 64 uneven
// cubes, 49.5M fluid nodes, a persistent grid of 8 per CU made the batched
// FP32 solves 1.5x slower than the solves one after the other).
int batch_workgroups(const cdi_batch *b, int count)
{
    int wg = b->workgroups_req > 0 ? b->workgroups_req : count;
    if (wg > count) wg = count;
    return wg < 1 ? 1 : wg;
}

int step_class(int mode, int odd)
{
    switch (mode) {
    case kModeFlow: return odd == kPull ? kClassFlowPull : odd ? kClassFlowOdd : kClassFlowEven;
    case kModeFused: return odd == kPull ? kClassFusedPull : odd ? kClassFusedOdd : kClassFusedEven;
    case kModeIons: return kClassIons;
    default: return -1;
    }
}

// Flags of member k's step number `idx` of an advance of `nsteps` steps.
int batch_flags(const cdi_solver *s, int mode, int64_t idx, int64_t nsteps, bool want_resid)
{
    int flags = 0;
    if (mode == kModeFlow && want_resid) {
        if (idx == nsteps - 2 && !s->mb) flags |= kStoreU;
        if (idx == nsteps - 1) flags |= kResid;
    }
    if (mode == kModeFused && s->mb && idx > 0) flags |= kJFromM;
    return flags;
}

// Descriptors of one step and its (instance, tile) list grouped by step class.
void fill_slot(cdi_batch *bt, int slot, const int32_t *modes, int64_t idx, int64_t nsteps, bool want_resid)
{
    BatchInst *h = bt->hstage + (size_t)slot * bt->cap_n;
    int count[kClasses] = {};
    for (int k = 0; k < bt->n; ++k) {
        const cdi_solver *s = bt->m[k];
        BatchInst &I = h[k];
        I.g = s->g;
        I.p = s->p;
        I.b = make_bufs(s, batch_flags(s, modes[k], idx, nsteps, want_resid));
        const int c = step_class(modes[k], stream_arg(s));
        if (c >= 0) count[c] += s->ntiles;
    }
    int *beg = bt->cls_begin[slot];
    beg[0] = 0;
    for (int c = 0; c < kClasses; ++c) beg[c + 1] = beg[c] + count[c];
    int pos[kClasses];
    for (int c = 0; c < kClasses; ++c) pos[c] = beg[c];
    int2 *t = bt->htiles + (size_t)slot * bt->cap_tiles;
    for (int k = 0; k < bt->n; ++k) {
        const int c = step_class(modes[k], stream_arg(bt->m[k]));
        if (c < 0) continue;
        for (int q = 0; q < bt->m[k]->ntiles; ++q) t[pos[c]++] = make_int2(k, q);
    }
}

void advance_members(cdi_batch *bt, const int32_t *modes)
{
    for (int k = 0; k < bt->n; ++k) {
        cdi_solver *s = bt->m[k];
        switch (modes[k]) {
        case kModeFlow: advance_state(s, 1, 0); break;
        case kModeIons: advance_state(s, 0, 1); s->np_steps++; break;
        case kModeFused: advance_state(s, 1, 1); s->np_steps++; break;
        default: break;
        }
    }
}

int upload_slot(cdi_batch *bt, int slot)
{
    const size_t bytes = sizeof(BatchInst) * (size_t)bt->n;
    HIPCHK(hipMemcpyAsync(bt->dinst + (size_t)slot * bt->cap_n, bt->hstage + (size_t)slot * bt->cap_n, bytes,
                          hipMemcpyHostToDevice, bt->stream));
    const size_t nt = (size_t)bt->cls_begin[slot][kClasses];
    if (nt)
        HIPCHK(hipMemcpyAsync(bt->dtiles + (size_t)slot * bt->cap_tiles,
                              bt->htiles + (size_t)slot * bt->cap_tiles, 8 * nt, hipMemcpyHostToDevice,
                              bt->stream));
    return CDI_OK;
}

int launch_slot(cdi_batch *bt, int slot)
{
    const int *beg = bt->cls_begin[slot];
    for (int c = 0; c < kClasses; ++c) {
        const int count = beg[c + 1] - beg[c];
        if (count <= 0) continue;
        HIPCHK(launch_batch(bt->dim, bt->st, c, bt->dinst + (size_t)slot * bt->cap_n,
                            bt->dtiles + (size_t)slot * bt->cap_tiles + beg[c], count,
                            batch_workgroups(bt, count), bt->lds_pad, bt->stream));
    }
    return CDI_OK;
}

// Launch shape of the step pair in slots 4 and 5.
std::vector<int> pair_signature(const cdi_batch *bt)
{
    std::vector<int> sig{bt->workgroups_req, bt->lds_pad};
    for (int slot = 4; slot <= 5; ++slot)
        for (int c = 0; c <= kClasses; ++c) sig.push_back(bt->cls_begin[slot][c]);
    return sig;
}

int eager_step(cdi_batch *bt, int slot, const int32_t *modes, int64_t idx, int64_t nsteps, bool want_resid)
{
    fill_slot(bt, slot, modes, idx, nsteps, want_resid);
    int rc = upload_slot(bt, slot);
    if (rc) return rc;
    if ((rc = launch_slot(bt, slot)) != CDI_OK) return rc;
    advance_members(bt, modes);
    return CDI_OK;
}

// Graph of one step pair (slots 4 and 5); rebuilt when the launch shape changes.
int ensure_graph(cdi_batch *bt)
{
    const std::vector<int> sig = pair_signature(bt);
    if (bt->exec && bt->exec_sig == sig) return CDI_OK;
    if (bt->exec) {
        (void)hipGraphExecDestroy(bt->exec);
        bt->exec = nullptr;
    }
    if (!bt->stream) return CDI_E_INVALID;  // the default stream cannot be captured
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_slot(bt, 4);
    if (rc == CDI_OK) rc = launch_slot(bt, 5);
    const hipError_t e = hipStreamEndCapture(bt->stream, &graph);
    if (rc != CDI_OK) return rc;
    if (e != hipSuccess) return fail(CDI_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&bt->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
        bt->exec = nullptr;
        return fail(CDI_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e2));
    }
    bt->exec_sig = sig;
    return CDI_OK;
}

}  // namespace

extern "C" {

int cdi_batch_bytes(cdi_solver *const *members, int32_t n, uint64_t *bytes)
{
    if (!members || n <= 0 || !bytes) return fail(CDI_E_INVALID, "bad batch arguments");
    int total = 0;
    for (int k = 0; k < n; ++k) {
        if (!members[k]) return fail(CDI_E_INVALID, "member %d is NULL", k);
        total += members[k]->ntiles;
    }
    *bytes = batch_layout(n, total, nullptr, nullptr, nullptr, nullptr);
    return CDI_OK;
}

}  // extern "C"

namespace {

// Tiles a batch of capacity max_fluid fluid nodes over max_members members can hold.
int64_t capacity_tiles(int32_t max_members, int64_t max_fluid)
{
    return (max_fluid + kTile - 1) / kTile + max_members;
}

// A batch with room for cap_n members and cap_tiles tiles in ws, holding members[0..n).
int batch_new(cdi_solver *const *members, int32_t n, int cap_n, int64_t cap_tiles, void *ws, uint64_t ws_bytes,
              void *stream, cdi_batch **out)
{
    if (!out || !ws || ((uintptr_t)ws % kAlign)) return fail(CDI_E_BUFFER, "batch workspace NULL or misaligned");
    if (cap_n <= 0 || cap_tiles <= 0 || cap_tiles > 0x3fffffff) return fail(CDI_E_INVALID, "bad batch capacity");
    const uint64_t need = batch_layout(cap_n, (int)cap_tiles, nullptr, nullptr, nullptr, nullptr);
    if (ws_bytes < need) return fail(CDI_E_BUFFER, "batch workspace too small: %llu < %llu",
                                     (unsigned long long)ws_bytes, (unsigned long long)need);
    for (int k = 1; k < n; ++k)
        if (members[k]->dim != members[0]->dim || members[k]->st != members[0]->st)
            return fail(CDI_E_INVALID, "batch members must share dimension and precision");
    cdi_batch *bt = new (std::nothrow) cdi_batch();
    if (!bt) return fail(CDI_E_INVALID, "out of host memory");
    bt->m.assign(members, members + n);
    bt->n = n;
    bt->dim = n > 0 ? members[0]->dim : -1;
    bt->st = n > 0 ? members[0]->st : -1;
    bt->cap_n = cap_n;
    bt->cap_tiles = (int)cap_tiles;
    bt->stream = (hipStream_t)stream;
    for (int k = 0; k < n; ++k) {
        bt->tile_begin.push_back(bt->total_tiles);
        bt->total_tiles += members[k]->ntiles;
    }
    batch_layout(cap_n, bt->cap_tiles, &bt->dinst, &bt->dtiles, &bt->dred, ws);
    bt->resid_valid.assign(n, 0);
    int dev = 0;
    auto cleanup = [&](int code) {
        if (bt->hstage) (void)hipHostFree(bt->hstage);
        if (bt->htiles) (void)hipHostFree(bt->htiles);
        if (bt->hworst) (void)hipHostFree(bt->hworst);
        if (bt->done) (void)hipEventDestroy(bt->done);
        delete bt;
        return code;
    };
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&bt->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return cleanup(fail(CDI_E_DEVICE, "device query failed"));
    if (hipHostMalloc((void **)&bt->hstage, sizeof(BatchInst) * (size_t)kSlots * cap_n, hipHostMallocDefault) !=
        hipSuccess)
        return cleanup(fail(CDI_E_DEVICE, "pinned staging allocation failed"));
    if (hipHostMalloc((void **)&bt->htiles, 8ull * kSlots * (size_t)bt->cap_tiles, hipHostMallocDefault) !=
        hipSuccess)
        return cleanup(fail(CDI_E_DEVICE, "pinned staging allocation failed"));
    if (hipHostMalloc((void **)&bt->hworst, 8ull * cap_n, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(CDI_E_DEVICE, "pinned staging allocation failed"));
    if (hipEventCreateWithFlags(&bt->done, hipEventDisableTiming) != hipSuccess)
        return cleanup(fail(CDI_E_DEVICE, "event creation failed"));
    *out = bt;
    return CDI_OK;
}

}  // namespace

extern "C" {

int cdi_batch_create(cdi_solver *const *members, int32_t n, void *ws, uint64_t ws_bytes, void *stream,
                     cdi_batch **out)
{
    uint64_t need = 0;
    int rc = cdi_batch_bytes(members, n, &need);
    if (rc) return rc;
    int64_t tiles = 0;
    for (int k = 0; k < n; ++k) tiles += members[k]->ntiles;
    return batch_new(members, n, n, tiles, ws, ws_bytes, stream, out);
}

int cdi_batch_capacity_bytes(int32_t max_members, int64_t max_fluid, uint64_t *bytes)
{
    if (max_members <= 0 || max_fluid <= 0 || !bytes) return fail(CDI_E_INVALID, "bad batch capacity");
    const int64_t tiles = capacity_tiles(max_members, max_fluid);
    if (tiles > 0x3fffffff) return fail(CDI_E_INVALID, "batch capacity too large");
    *bytes = batch_layout(max_members, (int)tiles, nullptr, nullptr, nullptr, nullptr);
    return CDI_OK;
}

int cdi_batch_create_empty(int32_t max_members, int64_t max_fluid, void *ws, uint64_t ws_bytes, void *stream,
                           cdi_batch **out)
{
    if (max_members <= 0 || max_fluid <= 0) return fail(CDI_E_INVALID, "bad batch capacity");
    return batch_new(nullptr, 0, max_members, capacity_tiles(max_members, max_fluid), ws, ws_bytes, stream, out);
}

int cdi_batch_admit(cdi_batch *bt, cdi_solver *member)
{
    if (!bt || !member) return fail(CDI_E_INVALID, "NULL argument");
    for (const cdi_solver *m : bt->m)
        if (m == member) return fail(CDI_E_INVALID, "solver is already a member");
    if (bt->n > 0 && (member->dim != bt->dim || member->st != bt->st))
        return fail(CDI_E_INVALID, "batch members must share dimension and precision");
    if (bt->n + 1 > bt->cap_n || (int64_t)bt->total_tiles + member->ntiles > bt->cap_tiles)
        return fail(CDI_E_BUFFER, "batch full: %d of %d members, %d + %d of %d tiles", bt->n, bt->cap_n,
                    bt->total_tiles, member->ntiles, bt->cap_tiles);
    if (bt->n == 0) {
        bt->dim = member->dim;
        bt->st = member->st;
    }
    bt->m.push_back(member);
    bt->tile_begin.push_back(bt->total_tiles);
    bt->total_tiles += member->ntiles;
    bt->resid_valid.push_back(0);
    bt->n++;
    return CDI_OK;
}

int cdi_batch_retire(cdi_batch *bt, cdi_solver *member)
{
    if (!bt || !member) return fail(CDI_E_INVALID, "NULL argument");
    int k = 0;
    while (k < bt->n && bt->m[k] != member) ++k;
    if (k == bt->n) return fail(CDI_E_INVALID, "solver is not a member");
    // nothing batched may still be reading the member's descriptors or state
    if (bt->stream) HIPCHK(hipStreamSynchronize(bt->stream));
    bt->m.erase(bt->m.begin() + k);
    bt->resid_valid.erase(bt->resid_valid.begin() + k);
    bt->n--;
    bt->tile_begin.clear();
    bt->total_tiles = 0;
    for (int q = 0; q < bt->n; ++q) {
        bt->tile_begin.push_back(bt->total_tiles);
        bt->total_tiles += bt->m[q]->ntiles;
    }
    return CDI_OK;
}

int cdi_batch_members(const cdi_batch *bt, int32_t *n)
{
    if (!bt || !n) return fail(CDI_E_INVALID, "NULL argument");
    *n = bt->n;
    return CDI_OK;
}

int cdi_batch_destroy(cdi_batch *bt)
{
    if (!bt) return CDI_OK;
    if (bt->stream) (void)hipStreamSynchronize(bt->stream);
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->hstage) (void)hipHostFree(bt->hstage);
    if (bt->htiles) (void)hipHostFree(bt->htiles);
    if (bt->hworst) (void)hipHostFree(bt->hworst);
    if (bt->done) (void)hipEventDestroy(bt->done);
    delete bt;
    return CDI_OK;
}

int cdi_batch_set_launch(cdi_batch *bt, int32_t workgroups, int32_t blocks_per_cu)
{
    if (!bt || workgroups < 0 || blocks_per_cu < 0) return fail(CDI_E_INVALID, "bad launch shape");
    int pad = 0;
    int rc = occupancy_pad(blocks_per_cu, &pad);
    if (rc) return rc;
    bt->workgroups_req = workgroups;
    bt->blocks_per_cu = blocks_per_cu;
    bt->lds_pad = pad;
    if (bt->exec) {
        (void)hipStreamSynchronize(bt->stream);
        (void)hipGraphExecDestroy(bt->exec);
        bt->exec = nullptr;
        bt->exec_sig.clear();
    }
    return CDI_OK;
}

int cdi_batch_get_launch(const cdi_batch *bt, int32_t *workgroups, int32_t *blocks_per_cu)
{
    if (!bt) return fail(CDI_E_INVALID, "NULL batch");
    if (workgroups) *workgroups = batch_workgroups(bt, bt->total_tiles);
    if (blocks_per_cu) *blocks_per_cu = bt->blocks_per_cu;
    return CDI_OK;
}

int cdi_batch_advance(cdi_batch *bt, int64_t nsteps, const int32_t *modes)
{
    if (!bt || nsteps < 0) return fail(CDI_E_INVALID, "bad arguments");
    if (nsteps == 0 || bt->n == 0) return CDI_OK;
    if (!modes) return fail(CDI_E_INVALID, "modes is NULL");
    bool any_flow = false, any_fused = false, need_first = false;
    for (int k = 0; k < bt->n; ++k) {
        const int md = modes[k];
        cdi_solver *s = bt->m[k];
        if (md < kModeIdle || md > kModeFused) return fail(CDI_E_INVALID, "bad mode for member %d", k);
        if (md == kModeFused) any_fused = true;
        if ((md == kModeIons || md == kModeFused) && s->params.np_substeps != 1)
            return fail(CDI_E_INVALID, "member %d: batched ion steps need np_substeps = 1", k);
        if (md == kModeFlow) any_flow = true;
        if ((md == kModeFlow || md == kModeFused) && s->flow_steps == 0) need_first = true;
        if (md == kModeFused && s->mb) need_first = true;
        // a pending renewal of the plane references applies to one step only
        if ((md == kModeFlow || md == kModeFused) && s->rpend) need_first = true;
    }
    if (any_fused && nsteps > kFusedRecheck) {
        // the flow keeps changing under fused steps: as cdi_np_step, the
        // positivity bound is taken again every kFusedRecheck steps (each
        // chunk checks it first). The last chunk keeps at least two steps, so
        // flow members end with their residual as from one call; the steps
        // themselves do not depend on the chunking.
        int64_t left = nsteps;
        while (left > 0) {
            int64_t c = left > kFusedRecheck ? kFusedRecheck : left;
            if (left - c == 1) --c;
            const int rc = cdi_batch_advance(bt, c, modes);
            if (rc != CDI_OK) return rc;
            left -= c;
        }
        return CDI_OK;
    }
    // order after the members' own streams
    for (int k = 0; k < bt->n; ++k) HIPCHK(hipStreamSynchronize(bt->m[k]->stream));
    HIPCHK(hipStreamSynchronize(bt->stream));
    // positivity of the ion updates, as cdi_np_step (the flux field is made
    // valid on the member's stream): every member's check is queued on its
    // stream first and all are read after one wait per member, instead of a
    // round trip to the host per member
    bool any_ions = false;
    for (int k = 0; k < bt->n; ++k) {
        if (modes[k] != kModeIons && modes[k] != kModeFused) continue;
        cdi_solver *s = bt->m[k];
        int rc = ensure_j(s);
        if (rc) return rc;
        HIPCHK(launch_stability(s->dim, s->g, s->p, s->node.j[s->jcur], s->node.part, s->node.red, s->stream));
        HIPCHK(hipMemcpyAsync(bt->hworst + k, s->node.red, 8, hipMemcpyDeviceToHost, s->stream));
        any_ions = true;
    }
    if (any_ions) {
        for (int k = 0; k < bt->n; ++k)
            if (modes[k] == kModeIons || modes[k] == kModeFused) HIPCHK(hipStreamSynchronize(bt->m[k]->stream));
        for (int k = 0; k < bt->n; ++k)
            if ((modes[k] == kModeIons || modes[k] == kModeFused) && !(bt->hworst[k] <= 1.0))
                return fail(CDI_E_UNSTABLE, "member %d: positivity bound violated (%g > 1)", k, bt->hworst[k]);
    }
    const bool want_resid = any_flow && nsteps >= 2;
    const int64_t suffix = want_resid ? 2 : 0;
    int64_t idx = 0;
    int rc = CDI_OK;
    if (need_first && nsteps - suffix >= 1) {
        if ((rc = eager_step(bt, 0, modes, idx, nsteps, want_resid)) != CDI_OK) return rc;
        ++idx;
    }
    const int64_t mid = nsteps - suffix - idx;
    const int64_t pairs = mid / 2;
    if (pairs > 0) {
        // descriptors of the two steps of a pair: the state now and one step on
        fill_slot(bt, 4, modes, idx, nsteps, want_resid);
        std::vector<cdi_solver> saved;
        saved.reserve(bt->n);
        for (int k = 0; k < bt->n; ++k) saved.push_back(*bt->m[k]);
        advance_members(bt, modes);
        fill_slot(bt, 5, modes, idx + 1, nsteps, want_resid);
        for (int k = 0; k < bt->n; ++k) *bt->m[k] = saved[k];
        if ((rc = upload_slot(bt, 4)) != CDI_OK) return rc;
        if ((rc = upload_slot(bt, 5)) != CDI_OK) return rc;
        if (bt->stream && ensure_graph(bt) == CDI_OK) {
            for (int64_t q = 0; q < pairs; ++q) HIPCHK(hipGraphLaunch(bt->exec, bt->stream));
        } else {  // default stream (not capturable): the same pair, launched directly
            for (int64_t q = 0; q < pairs; ++q) {
                if ((rc = launch_slot(bt, 4)) != CDI_OK) return rc;
                if ((rc = launch_slot(bt, 5)) != CDI_OK) return rc;
            }
        }
        for (int64_t q = 0; q < 2 * pairs; ++q) advance_members(bt, modes);
        idx += 2 * pairs;
    }
    // an odd leftover, then the residual steps
    while (idx < nsteps) {
        const int slot = (idx == nsteps - 2 && suffix) ? 2 : (idx == nsteps - 1 && suffix) ? 3 : 1;
        if (slot == 1 && idx != nsteps - suffix - 1) return fail(CDI_E_INVALID, "internal step accounting");
        if ((rc = eager_step(bt, slot, modes, idx, nsteps, want_resid)) != CDI_OK) return rc;
        ++idx;
    }
    for (int k = 0; k < bt->n; ++k) {
        cdi_solver *s = bt->m[k];
        bt->resid_valid[k] = 0;
        if (modes[k] == kModeFlow) {
            s->jstate = J_INVALID;
            if (want_resid) {
                HIPCHK(launch_reduce_tiles(s->node.resid, s->ntiles, 2, 2, bt->dred + 2 * k, bt->stream));
                bt->resid_valid[k] = 1;
            }
        } else if (modes[k] == kModeFused) {
            s->jstate = s->mb ? J_IN_M : J_VALID;
        }
    }
    // the members' streams wait for the batch
    HIPCHK(hipEventRecord(bt->done, bt->stream));
    for (int k = 0; k < bt->n; ++k)
        if (bt->m[k]->stream != bt->stream) HIPCHK(hipStreamWaitEvent(bt->m[k]->stream, bt->done, 0));
    return CDI_OK;
}

int cdi_batch_residuals(cdi_batch *bt, double *r)
{
    if (!bt || !r) return fail(CDI_E_INVALID, "NULL argument");
    std::vector<double> h(2 * (size_t)bt->n);
    HIPCHK(hipMemcpyAsync(h.data(), bt->dred, 16ull * bt->n, hipMemcpyDeviceToHost, bt->stream));
    HIPCHK(hipStreamSynchronize(bt->stream));
    for (int k = 0; k < bt->n; ++k)
        r[k] = bt->resid_valid[k] ? std::sqrt(h[2 * k]) / std::sqrt(h[2 * k + 1]) : NAN;
    return CDI_OK;
}

int cdi_batch_autotune(cdi_batch *bt, int32_t steps, const int32_t *modes, int32_t *workgroups,
                       double *ms_per_step)
{
    if (!bt || !modes || steps < 2) return fail(CDI_E_INVALID, "bad arguments");
    std::vector<std::vector<uint8_t>> snaps(bt->n);
    int rc = CDI_OK;
    for (int k = 0; k < bt->n; ++k) {
        uint64_t nb = 0;
        if ((rc = cdi_snapshot_bytes(bt->m[k], &nb)) != CDI_OK) return rc;
        snaps[k].resize(nb);
        if ((rc = cdi_snapshot(bt->m[k], snaps[k].data(), nb)) != CDI_OK) return rc;
    }
    auto restore_all = [&]() {
        for (int k = 0; k < bt->n; ++k) {
            int r2 = cdi_restore(bt->m[k], snaps[k].data(), snaps[k].size());
            if (r2) return r2;
        }
        return (int)CDI_OK;
    };
    const int start_wg = bt->workgroups_req, start_occ = bt->blocks_per_cu;
    std::vector<int> cands;
    for (int mult : {2, 3, 4, 5, 6, 8, 12, 16}) cands.push_back(mult * bt->cus);
    cands.push_back(bt->total_tiles);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int best = start_wg;
    float best_ms = INFINITY;
    for (int wg : cands) {
        if (wg > bt->total_tiles) continue;
        if ((rc = cdi_batch_set_launch(bt, wg, start_occ)) != CDI_OK) break;
        if ((rc = restore_all()) != CDI_OK) break;
        if ((rc = cdi_batch_advance(bt, 2, modes)) != CDI_OK) break;  // builds the graph
        if ((rc = cdi_batch_advance(bt, 2, modes)) != CDI_OK) break;
        HIPCHK(hipStreamSynchronize(bt->stream));
        HIPCHK(hipEventRecord(e0, bt->stream));
        if ((rc = cdi_batch_advance(bt, steps, modes)) != CDI_OK) break;
        HIPCHK(hipEventRecord(e1, bt->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = wg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int rc2 = cdi_batch_set_launch(bt, best, start_occ);
    const int rc3 = restore_all();
    for (int k = 0; k < bt->n; ++k) bt->resid_valid[k] = 0;
    if (rc) return rc;
    if (rc2) return rc2;
    if (rc3) return rc3;
    if (workgroups) *workgroups = best;
    if (ms_per_step) *ms_per_step = best_ms / steps;
    return CDI_OK;
}

}  // extern "C"
