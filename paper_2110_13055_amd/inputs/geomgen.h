/*
 * geomgen.h -- seeded synthetic electrode geometry (input generator).
 *
 * The paper builds its porous electrodes from voxel images (Sec. 2, MAC grid:
 * one grid block per image voxel; Sec. 4 SEM image; Sec. 5 random fibres).
 * The images themselves are not available, so workloads are synthetic: a
 * seeded list of solid primitives (disks in 2D, spheres or straight fibres
 * in 3D) with the porosity and grain sizes of the paper's electrodes.
 *
 * This module only draws primitives. It holds none of the transport or flow
 * arithmetic. Both the GPU library and the CPU reference implementation
 * compile their own copy of it, so that both start from identical
 * primitive lists; each then voxelises the primitives independently.
 *
 * Units: every length is an integer in 1/256 lattice units, so the inside
 * test "voxel centre within radius" is exact integer arithmetic.
 *
 * RNG: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014). One draw is one 64-bit
 * output. A uniform integer on [lo, hi] is lo + (x mod (hi - lo + 1)).
 * Draw order per primitive: radius, cx, cy, (cz).
 */
#ifndef CDI_GEOMGEN_H
#define CDI_GEOMGEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One primitive: radius and centre, all in 1/256 lattice units. cz = 0 in 2D. */
typedef struct {
    int64_t r, cx, cy, cz;
} geomgen_prim;

/* Status codes (0 = OK). */
#define GEOMGEN_OK 0
#define GEOMGEN_E_INVALID (-1)
#define GEOMGEN_E_JAMMED (-2)   /* RSA could not reach the porosity */
#define GEOMGEN_E_NOMEM (-3)

/* Advance a SplitMix64 state and return the next output. */
uint64_t geomgen_splitmix64(uint64_t *state);

/* Uniform integer on [lo, hi] from one draw (lo <= hi). */
int64_t geomgen_uniform_int(uint64_t *state, int64_t lo, int64_t hi);

/*
 * 2D non-overlapping disks by random sequential addition.
 *   nx, ny        lattice size (x = flow axis)
 *   buffer_x      number of always-fluid planes at each x end
 *   walls_y       1: rows 0 and ny-1 are inert walls (not counted as pore)
 *                 0: y is periodic (disks wrap in y)
 *   porosity      stop as soon as fluid voxels / (nx*ny) <= porosity
 *   r_min, r_max  radius range in lattice units
 *   min_gap       minimum surface-to-surface gap in lattice units (> 0)
 * A candidate is accepted iff its centre distance to every accepted disk is
 * >= r1 + r2 + gap. Fails with GEOMGEN_E_JAMMED after 10^6 consecutive
 * rejections. *out is malloc'd (caller frees with geomgen_free).
 * *n_fluid receives the exact fluid-voxel count of the final geometry.
 */
int geomgen_disks(int nx, int ny, int buffer_x, int walls_y, uint64_t seed,
                  double porosity, double r_min, double r_max, double min_gap,
                  geomgen_prim **out, int64_t *n_out, int64_t *n_fluid);

/*
 * 3D overlapping spheres (Boolean model), periodic in y and z, clipped in x to
 * the interior slab [buffer_x, nx - buffer_x). The count is
 *   n = round(-ln(phi_int) * V_int / E[V]),  E[V] = (4 pi / 3) E[r^3],
 * with r uniform on [r_min, r_max] and phi_int the interior porosity that
 * yields the requested overall porosity once the fluid buffers are included.
 */
int geomgen_spheres(int nx, int ny, int nz, int buffer_x, uint64_t seed,
                    double porosity, double r_min, double r_max,
                    geomgen_prim **out, int64_t *n_out);

/* Number of spheres geomgen_spheres would draw (no allocation). */
int64_t geomgen_sphere_count(int nx, int ny, int nz, int buffer_x,
                             double porosity, double r_min, double r_max);

/*
 * One straight fibre (Sec. 5): radius r and a point o of its core line in
 * 1/256 lattice units, and the core line's direction d as an integer vector
 * (any length; |d_i| <= 1024). The fibre is every voxel whose centre lies
 * within r of the infinite core line, inside the interior slab.
 */
typedef struct {
    int64_t r, ox, oy, oz, dx, dy, dz, pad;
} geomgen_fibre;

/*
 * 3D overlapping straight fibres (Sec. 5: a random core orientation through a
 * random point, extended to the domain faces, voxels within the radius solid,
 * free overlap). Draws per fibre: radius (uniform on [r_min, r_max] in 1/256
 * units), origin (ox, oy, oz uniform in the interior slab box
 * [buffer_x, nx - buffer_x) x [0, ny) x [0, nz)), then direction attempts of
 * three draws (a, b, c) uniform on [-1024, 1024] until 0 < a^2 + b^2 + c^2 <=
 * 1024^2 (a point uniform in the ball: an isotropic direction, integers
 * only). Fibres are added until the Boolean-model pore fraction of the slab,
 * exp(-sum_k v_k / V_int), is <= phi_int (the interior porosity that gives the
 * requested overall porosity with the fluid buffers), where v_k = pi r_k^2
 * L_k and L_k is the length of fibre k's core line inside the slab box.
 * Fibres do not wrap. Limits: nx, ny, nz <= 1024, r_max <= 64 (the exact
 * inside test then fits int64). *out is malloc'd (geomgen_free).
 */
int geomgen_fibres(int nx, int ny, int nz, int buffer_x, uint64_t seed,
                   double porosity, double r_min, double r_max,
                   geomgen_fibre **out, int64_t *n_out);

void geomgen_free(void *p);

#ifdef __cplusplus
}
#endif
#endif
