// cdi_internal.h -- lattice tables, kernel argument blocks and launcher
// declarations shared by the HIP translation units of libcdi.
//
// Data layout in device memory (N_f fluid nodes, stride P = N_f rounded up to
// a whole number of 256-node tiles):
//   populations  Q x P values in blocks of 64 nodes (block k: the Q
//                directions of nodes 64k .. 64k + 63, 64 values each), FP32
//                f - w_i(1 + R[x]) or FP16 scaled values; none with moment
//                storage
//   moments      FP16 and moment storage: float4 (rho - 1, ux, uy, uz) per
//                node, double buffered (the moments of the previous step
//                belong to the emitters of the populations now stored)
//   jbuf         advecting mass flux j = rho u for the ions, d planes of P,
//                double buffered (fused steps read one and write the other)
//   conc         2 species x P, double buffered (Jacobi update)
//   acc          per tile 8 doubles: A_na, A_cl, In_na, In_cl, Out_na, Out_cl
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace cdi {

constexpr int kTile = 256;  // fluid nodes per tile (= threads per block)

// D2Q9; directions 1..4 are the faces +x, -x, +y, -y.
struct D2Q9 {
    static constexpr int D = 2, Q = 9;
    static constexpr int ex[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int ey[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
    static constexpr float w[9] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                                   1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
};

// D3Q19; directions 1..6 are the faces +x, -x, +y, -y, +z, -z.
struct D3Q19 {
    static constexpr int D = 3, Q = 19;
    static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr float w[19] = {1.f / 3,  1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18,
                                    1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                                    1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
};

// map values of non-fluid voxels
constexpr int kElectrode = -1;
constexpr int kInert = -2;
constexpr int kOutside = -3;  // beyond an open x end

// Nernst-Planck x-end treatments (same numbering as the public enum)
constexpr int kNpxInletOutlet = 0, kNpxPeriodic = 1, kNpxClosed = 2, kNpxDirichlet = 3;

// step flags
constexpr int kStoreU = 1;    // write u of the incoming state to ubuf
constexpr int kResid = 2;     // accumulate |u - ubuf|^2 and |u|^2 per tile
constexpr int kJFromM = 4;    // FP16/moment fused: ions read j from the moments buffer
constexpr int kNee = 8;       // the stored state carries inlet/outlet extrapolation
                              // (every state after the first step)

// Internal node order: fluid nodes are numbered brick by brick (bricks of
// 2^bsx x 2^bsy x 2^bsz voxels, bricks in x-fastest order, voxels inside a
// brick x-fastest), so that a workgroup's nodes and most of their lattice
// neighbours share a small block of memory. The public numbering (fields
// handed to the caller, the fluid index map) stays lexicographic.
struct Bricks {
    int bsx, bsy, bsz;  // log2 of the brick edge lengths
    int nbx, nby, nbz;  // bricks along each axis (padded)
    int cbx, cby;       // bits of x and y in a packed node coordinate
};

// Packed node coordinates: x | y << cbx | z << (cbx + cby), 32 bits.
__host__ __device__ inline uint32_t pack_xyz(const Bricks &k, int x, int y, int z)
{
    return (uint32_t)x | ((uint32_t)y << k.cbx) | ((uint32_t)z << (k.cbx + k.cby));
}

__host__ __device__ inline int64_t brick_index(const Bricks &k, int x, int y, int z)
{
    const int64_t b = ((int64_t)(z >> k.bsz) * k.nby + (y >> k.bsy)) * k.nbx + (x >> k.bsx);
    const int l = ((((z & ((1 << k.bsz) - 1)) << k.bsy) | (y & ((1 << k.bsy) - 1))) << k.bsx) |
                  (x & ((1 << k.bsx) - 1));
    return (b << (k.bsx + k.bsy + k.bsz)) | l;
}

struct Grid {
    int nx, ny, nz;
    int n_f;         // fluid nodes
    int P;           // plane stride (multiple of kTile)
    int periodic_x;  // LBM periodic in x (body-force drive)
    int inout;       // inlet/outlet planes at x = 0 and x = nx - 1
    Bricks bk;
    const uint32_t *fluid;  // internal node -> packed (x, y, z)
    const int *map;         // brick-ordered voxel -> internal node, or kElectrode / kInert
    // Tile schedule: XCD-local position -> tile. Tiles are ordered by
    // (band of rows, z) so the planes above and below a tile were visited
    // shortly before by the same XCD and are still in its L2.
    const int *sched;
    // Optional neighbour list: map value of the neighbour of node n along
    // direction i in nbr[(i - 1) * P + n] (i = 1 .. Q-1), so that a step reads
    // it with the node's other data instead of after its coordinates.
    const int *nbr;
    // dynamic LDS reserved per step workgroup: caps the workgroups resident
    // per CU (and so the working set the L2 must hold); 0 = no cap
    int lds_pad;
    // odd AA steps of the storages that allow it stage the tile's population
    // slots in LDS (set by the host from the tuning and the tile count)
    int stage_odd;
};

struct Phys {
    float omega;       // 1 / tau
    float fcoef;       // 1 - 1/(2 tau), Guo source prefactor
    float F[3];        // body-force density
    int forced;
    int linear_eq;
    // Nernst-Planck
    float D[2], invD[2], z[2], keff[2];
    float c0, c_out, u_in;
    float rho_out;     // outlet density of the flow
    float dpsi_dx;     // ramp drop per cell (dpsi / nx)
    int npx;
    float dt;
    const float *psi;  // optional field (fluid order), else ramp
    // FP16 deviation scale
    float hs, hs_inv;
};

// Buffers of one step; multi-plane fields are P apart (structure of arrays).
struct Bufs {
    void *f;        // populations: the array read (and, AA streaming, written)
    void *f2;       // pull streaming: the array written
    const float4 *Min;
    float4 *Mout;
    const float *jin;
    float *jout;
    const float *Cin;
    float *Cout;
    const __half2 *Clin;  // the concentrations' FP16 remainders (see lo_encode), per node
    __half2 *Clout;
    double *acc;
    double *resid;
    float *ubuf;    // FP32 storage: u (d planes) and rho - 1 (plane d) of the state, on kStoreU
    // FP32 storage: reference density deviation per x plane of the values read
    // and of the values written (see PlaneRef); nullptr: zero
    const float *rin;
    const float *rout;
    int flags;
};

// Storage of the lattice state (values of cdi_params.precision): FP32
// populations and FP16 populations (both relative to the plane references,
// the FP16 ones scaled; the ions' flux in its own buffer), FP16 deviations
// from the emitter's equilibrium with FP32 moment buffers, moments only.
constexpr int kF32 = 0, kF16 = 1, kMom = 2, kH16 = 3;
template <int ST>
constexpr bool kPlain = ST == kF32 || ST == kH16;  // populations relative to the plane references
template <int ST>
constexpr bool kHalfPop = ST == kF16 || ST == kH16;  // populations stored in FP16

// One instance of a batched launch.
constexpr int kModeIdle = 0, kModeFlow = 1, kModeIons = 2, kModeFused = 3;
struct BatchInst {
    Grid g;
    Phys p;
    Bufs b;
};
// Step classes of a batched step (kernel variants): LBM only or fused, by AA
// parity, and ions only.
constexpr int kClassFlowEven = 0, kClassFlowOdd = 1, kClassFusedEven = 2, kClassFusedOdd = 3,
              kClassIons = 4, kClassFlowPull = 5, kClassFusedPull = 6, kClasses = 7;

// Value of the kernels' parity argument for pull streaming (AA uses 0 / 1).
constexpr int kPull = 2;

// ------------------------------------------------------------ launchers
// Every launcher enqueues on `stream` and returns hipGetLastError().
hipError_t launch_init_labels(uint8_t *labels, int nx, int ny, int nz, int walls2d, hipStream_t s);
hipError_t launch_voxelize(uint8_t *labels, const int64_t *prims, int64_t nprims, int dim, int nx,
                           int ny, int nz, int walls_y, int buffer_x, hipStream_t s);
hipError_t launch_compact(const uint8_t *labels, int64_t nvox, int *map, int *fluid, int *blk,
                          int64_t *nfluid, hipStream_t s);
int64_t compact_blocks(int64_t nvox);
// Internal (brick-ordered) numbering of the fluid voxels: imap over the
// brick enumeration, ifluid[node] = lexicographic voxel, and lex2int[k] =
// internal node of lexicographic fluid node k (needs the lexicographic map).
hipError_t launch_compact_bricks(const uint8_t *labels, const int *lexmap, int nx, int ny, int nz,
                                 const Bricks &bk, int *imap, uint32_t *ifluid, int *lex2int, int *blk,
                                 int64_t *nfluid, hipStream_t s);
int64_t brick_enum_size(const Bricks &bk);
// Reorder d planes between the internal (stride P) and lexicographic (stride
// n_f) node orders. to_lex: dst[c*n_f + k] = src[c*P + lex2int[k]]; else the
// inverse scatter.
hipError_t launch_permute(const float *src, float *dst, const int *lex2int, int n_f, int P, int d,
                          int to_lex, hipStream_t s);

// Streaming kernels of known traffic over bytes (a multiple of 16): copy,
// XOR checksum of every 8 KiB block of src into dst (16 bytes per block),
// fill with a 32-bit value.
constexpr int kStreamCopy = 0, kStreamRead = 1, kStreamFill = 2;
constexpr uint64_t kStreamReadBlock = 8192;
hipError_t launch_stream(int mode, void *dst, const void *src, uint64_t bytes, uint32_t value, hipStream_t s);

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);

// One LBM and/or Nernst-Planck step over all fluid nodes.
//   dim 2/3, st = kF32/kF16/kMom, odd = AA parity of the stored state or
//   kPull, lbm/np switches.
hipError_t launch_step(int dim, int st, int odd, int lbm, int np, const Grid &g, const Phys &p,
                       const Bufs &b, hipStream_t s);
// One step of the instances of one step class in one persistent launch of
// `workgroups` workgroups over the class's (instance, tile) list (inst and
// tiles in device memory).
hipError_t launch_batch(int dim, int st, int cls, const BatchInst *inst, const int2 *tiles, int ntiles,
                        int workgroups, int lds_pad, hipStream_t s);
// Moments of the stored state: rho (nullable), u (nullable, d planes),
// j (nullable, d planes); rref: the FP32 plane references of the state
// (nullptr: zero).
hipError_t launch_moments(int dim, int st, int odd, int nee, const Grid &g, const Phys &p,
                          const void *f, const float4 *M, const float *rref, float *rho, float *u, float *j,
                          hipStream_t s);
// Plane references: rref[x] = mean of drho (rho - 1 of the fluid nodes, one
// plane of P values in node order) over the fluid voxels of plane x, 0 where
// the plane holds none; FP64 sums in a fixed order (one workgroup per plane).
hipError_t launch_plane_means(const Grid &g, const float *drho, float *rref, hipStream_t s);
// Packed coordinates of the first node of every tile (host-side tile schedule).
hipError_t launch_tile_heads(const Grid &g, uint32_t *heads, hipStream_t s);
// Neighbour list of every fluid node (see Grid::nbr), Q-1 planes of P.
hipError_t launch_build_nbr(int dim, const Grid &g, int *nbr, hipStream_t s);
// j = (1 + drho) u from the moments buffer (FP16 and moment storage).
hipError_t launch_j_from_m(int dim, const Grid &g, const float4 *M, float *j, hipStream_t s);
// Deterministic single-block sums: out[k] = sum_t in[t*stride + k], k < width.
hipError_t launch_reduce_tiles(const double *in, int ntiles, int stride, int width, double *out,
                               hipStream_t s);
// FP64 sum of each concentration field with its remainders (solute mass): out[0..1].
hipError_t launch_mass(const Grid &g, const float *C, const __half2 *Clo, double *part, double *out, hipStream_t s);
// max over nodes/species of dt * (sum of outflow coefficients); out[0].
hipError_t launch_stability(int dim, const Grid &g, const Phys &p, const float *j, double *part,
                            double *out, hipStream_t s);

}  // namespace cdi
