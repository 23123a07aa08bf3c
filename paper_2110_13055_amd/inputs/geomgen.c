/*
 * geomgen.c -- seeded synthetic electrode primitives. See geomgen.h.
 *
 * The porous electrodes of the paper are voxel images (Sec. 2: each grid
 * block is one image voxel). This file draws the primitive lists that stand
 * in for those images. It contains no flow or transport arithmetic.
 */
#include "geomgen.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

uint64_t geomgen_splitmix64(uint64_t *state)
{
    /* SplitMix64, Steele, Lea & Flood (2014), constants as published. */
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int64_t geomgen_uniform_int(uint64_t *state, int64_t lo, int64_t hi)
{
    uint64_t span = (uint64_t)(hi - lo) + 1u;
    uint64_t x = geomgen_splitmix64(state);
    return lo + (int64_t)(x % span);
}

void geomgen_free(void *p) { free(p); }

static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

static int64_t wrap(int64_t i, int64_t n)
{
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

/* Stamp one disk into the counting bitmap; returns the number of voxels that
 * turned from pore to solid. Used only for the RSA stop rule. */
static int64_t stamp_disk(uint8_t *solid, int nx, int ny, int walls_y, const geomgen_prim *p)
{
    int64_t added = 0;
    int64_t i0 = floor_div(p->cx - p->r, 256) - 1, i1 = floor_div(p->cx + p->r, 256) + 1;
    int64_t j0 = floor_div(p->cy - p->r, 256) - 1, j1 = floor_div(p->cy + p->r, 256) + 1;
    for (int64_t j = j0; j <= j1; ++j) {
        int64_t jj;
        if (walls_y) {
            if (j < 1 || j > ny - 2) continue;
            jj = j;
        } else {
            jj = wrap(j, ny);
        }
        int64_t dy = 128 * (2 * j + 1) - p->cy;
        for (int64_t i = i0; i <= i1; ++i) {
            if (i < 0 || i >= nx) continue;
            int64_t dx = 128 * (2 * i + 1) - p->cx;
            if (dx * dx + dy * dy <= p->r * p->r) {
                uint8_t *s = &solid[jj * nx + i];
                if (!*s) {
                    *s = 1;
                    ++added;
                }
            }
        }
    }
    return added;
}

int geomgen_disks(int nx, int ny, int buffer_x, int walls_y, uint64_t seed,
                  double porosity, double r_min, double r_max, double min_gap,
                  geomgen_prim **out, int64_t *n_out, int64_t *n_fluid)
{
    if (!out || !n_out || nx < 4 || ny < 3 || buffer_x < 0 || r_min <= 0 || r_max < r_min ||
        min_gap < 0 || porosity <= 0 || porosity > 1)
        return GEOMGEN_E_INVALID;
    const int64_t rlo = llround(r_min * 256.0), rhi = llround(r_max * 256.0);
    const int64_t gap = llround(min_gap * 256.0);
    const int64_t xmin = 256 * (int64_t)buffer_x, xmax = 256 * (int64_t)(nx - buffer_x);
    if (xmax - xmin < 2 * rhi) return GEOMGEN_E_INVALID;
    if (!walls_y && 2 * rhi + 3 * 256 > 256 * (int64_t)ny) return GEOMGEN_E_INVALID;

    const int64_t nvox = (int64_t)nx * ny;
    int64_t fluid = nvox - (walls_y ? 2 * (int64_t)nx : 0);
    uint8_t *solid = (uint8_t *)calloc((size_t)nvox, 1);
    int64_t cap = 64, n = 0;
    geomgen_prim *prims = (geomgen_prim *)malloc(sizeof(geomgen_prim) * (size_t)cap);
    if (!solid || !prims) {
        free(solid);
        free(prims);
        return GEOMGEN_E_NOMEM;
    }
    uint64_t st = seed;
    int64_t rejects = 0;
    const int64_t Ly = 256 * (int64_t)ny;
    while ((double)fluid > porosity * (double)nvox) {
        geomgen_prim c;
        c.r = geomgen_uniform_int(&st, rlo, rhi);
        c.cx = geomgen_uniform_int(&st, xmin + c.r, xmax - c.r);
        c.cy = geomgen_uniform_int(&st, 0, Ly - 1);
        c.cz = 0;
        int ok = 1;
        for (int64_t k = 0; k < n && ok; ++k) {
            int64_t dx = c.cx - prims[k].cx, dy = c.cy - prims[k].cy;
            if (!walls_y) {
                if (dy > Ly / 2) dy -= Ly;
                if (dy < -Ly / 2) dy += Ly;
            }
            int64_t s = c.r + prims[k].r + gap;
            if (dx * dx + dy * dy < s * s) ok = 0;
        }
        if (!ok) {
            if (++rejects > 1000000) {
                free(solid);
                free(prims);
                return GEOMGEN_E_JAMMED;
            }
            continue;
        }
        rejects = 0;
        if (n == cap) {
            cap *= 2;
            geomgen_prim *np = (geomgen_prim *)realloc(prims, sizeof(geomgen_prim) * (size_t)cap);
            if (!np) {
                free(solid);
                free(prims);
                return GEOMGEN_E_NOMEM;
            }
            prims = np;
        }
        prims[n++] = c;
        fluid -= stamp_disk(solid, nx, ny, walls_y, &c);
    }
    free(solid);
    *out = prims;
    *n_out = n;
    if (n_fluid) *n_fluid = fluid;
    return GEOMGEN_OK;
}

static int sphere_setup(int nx, int ny, int nz, int buffer_x, double porosity, double r_min,
                        double r_max, double *n_expected)
{
    if (nx < 2 * buffer_x + 1 || ny < 1 || nz < 1 || buffer_x < 0 || r_min <= 0 ||
        r_max < r_min || porosity <= 0 || porosity >= 1)
        return GEOMGEN_E_INVALID;
    if (2 * r_max + 3 > ny || 2 * r_max + 3 > nz) return GEOMGEN_E_INVALID;
    const double nvox = (double)nx * ny * nz;
    const double nbuf = 2.0 * buffer_x * (double)ny * nz;
    const double nint = nvox - nbuf;
    const double phi_int = (porosity * nvox - nbuf) / nint;
    if (!(phi_int > 0.0 && phi_int < 1.0)) return GEOMGEN_E_INVALID;
    const double a = r_min, b = r_max;
    /* E[r^3] for r uniform on [a, b]; the degenerate a == b case is a^3. */
    const double er3 = (b > a) ? (b * b * b * b - a * a * a * a) / (4.0 * (b - a)) : a * a * a;
    const double pi = 3.14159265358979323846;
    const double ev = (4.0 * pi / 3.0) * er3;
    *n_expected = -log(phi_int) * nint / ev;
    return GEOMGEN_OK;
}

int64_t geomgen_sphere_count(int nx, int ny, int nz, int buffer_x, double porosity,
                             double r_min, double r_max)
{
    double ne;
    if (sphere_setup(nx, ny, nz, buffer_x, porosity, r_min, r_max, &ne) != GEOMGEN_OK) return -1;
    return (int64_t)llround(ne);
}

int geomgen_spheres(int nx, int ny, int nz, int buffer_x, uint64_t seed,
                    double porosity, double r_min, double r_max,
                    geomgen_prim **out, int64_t *n_out)
{
    if (!out || !n_out) return GEOMGEN_E_INVALID;
    double ne;
    int rc = sphere_setup(nx, ny, nz, buffer_x, porosity, r_min, r_max, &ne);
    if (rc != GEOMGEN_OK) return rc;
    const int64_t n = (int64_t)llround(ne);
    geomgen_prim *prims = (geomgen_prim *)malloc(sizeof(geomgen_prim) * (size_t)(n > 0 ? n : 1));
    if (!prims) return GEOMGEN_E_NOMEM;
    const int64_t rlo = llround(r_min * 256.0), rhi = llround(r_max * 256.0);
    const int64_t xmin = 256 * (int64_t)buffer_x, xmax = 256 * (int64_t)(nx - buffer_x);
    uint64_t st = seed;
    for (int64_t k = 0; k < n; ++k) {
        prims[k].r = geomgen_uniform_int(&st, rlo, rhi);
        prims[k].cx = geomgen_uniform_int(&st, xmin, xmax - 1);
        prims[k].cy = geomgen_uniform_int(&st, 0, 256 * (int64_t)ny - 1);
        prims[k].cz = geomgen_uniform_int(&st, 0, 256 * (int64_t)nz - 1);
    }
    *out = prims;
    *n_out = n;
    return GEOMGEN_OK;
}

/* Length (lattice units) of the line o + t d inside the box lo <= p <= hi
 * (1/256 units), by the slab method. */
static double chord_length(const int64_t o[3], const int64_t d[3], const int64_t lo[3],
                           const int64_t hi[3])
{
    double tlo = -INFINITY, thi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0) continue; /* the origin lies inside the slab of this axis */
        double t1 = (double)(lo[a] - o[a]) / (double)d[a];
        double t2 = (double)(hi[a] - o[a]) / (double)d[a];
        if (t1 > t2) {
            const double t = t1;
            t1 = t2;
            t2 = t;
        }
        if (t1 > tlo) tlo = t1;
        if (t2 < thi) thi = t2;
    }
    if (!(thi > tlo)) return 0.0;
    const double dn = sqrt((double)(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
    return (thi - tlo) * dn / 256.0;
}

int geomgen_fibres(int nx, int ny, int nz, int buffer_x, uint64_t seed,
                   double porosity, double r_min, double r_max,
                   geomgen_fibre **out, int64_t *n_out)
{
    if (!out || !n_out) return GEOMGEN_E_INVALID;
    if (nx < 2 * buffer_x + 1 || ny < 1 || nz < 1 || buffer_x < 0 || nx > 1024 || ny > 1024 ||
        nz > 1024 || r_min <= 0 || r_max < r_min || r_max > 64 || porosity <= 0 || porosity >= 1)
        return GEOMGEN_E_INVALID;
    const double nvox = (double)nx * ny * nz;
    const double nbuf = 2.0 * buffer_x * (double)ny * nz;
    const double nint = nvox - nbuf;
    const double phi_int = (porosity * nvox - nbuf) / nint;
    if (!(phi_int > 0.0 && phi_int < 1.0)) return GEOMGEN_E_INVALID;
    const double target = -log(phi_int) * nint; /* sum of v_k that reaches phi_int */
    const double pi = 3.14159265358979323846;
    const int64_t rlo = llround(r_min * 256.0), rhi = llround(r_max * 256.0);
    const int64_t lo[3] = {256 * (int64_t)buffer_x, 0, 0};
    const int64_t hi[3] = {256 * (int64_t)(nx - buffer_x), 256 * (int64_t)ny, 256 * (int64_t)nz};
    int64_t cap = 1024, n = 0;
    geomgen_fibre *f = (geomgen_fibre *)malloc(sizeof(geomgen_fibre) * (size_t)cap);
    if (!f) return GEOMGEN_E_NOMEM;
    uint64_t st = seed;
    double covered = 0.0;
    while (covered < target) {
        if (n == cap) {
            if (cap >= (int64_t)1 << 24) {
                free(f);
                return GEOMGEN_E_INVALID;
            }
            geomgen_fibre *g = (geomgen_fibre *)realloc(f, sizeof(geomgen_fibre) * (size_t)(2 * cap));
            if (!g) {
                free(f);
                return GEOMGEN_E_NOMEM;
            }
            f = g;
            cap *= 2;
        }
        geomgen_fibre *p = &f[n];
        p->r = geomgen_uniform_int(&st, rlo, rhi);
        p->ox = geomgen_uniform_int(&st, lo[0], hi[0] - 1);
        p->oy = geomgen_uniform_int(&st, lo[1], hi[1] - 1);
        p->oz = geomgen_uniform_int(&st, lo[2], hi[2] - 1);
        for (;;) {
            const int64_t a = geomgen_uniform_int(&st, -1024, 1024);
            const int64_t b = geomgen_uniform_int(&st, -1024, 1024);
            const int64_t c = geomgen_uniform_int(&st, -1024, 1024);
            const int64_t q = a * a + b * b + c * c;
            if (q > 0 && q <= 1024 * 1024) {
                p->dx = a;
                p->dy = b;
                p->dz = c;
                break;
            }
        }
        p->pad = 0;
        const int64_t o[3] = {p->ox, p->oy, p->oz}, d[3] = {p->dx, p->dy, p->dz};
        const double r = (double)p->r / 256.0;
        covered += pi * r * r * chord_length(o, d, lo, hi);
        ++n;
    }
    *out = f;
    *n_out = n;
    return GEOMGEN_OK;
}
