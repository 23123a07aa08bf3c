/*
 * cdi_oracle.c -- plain FP64 CPU reference of the pore-scale CDI model.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the GPU library. See cdi_oracle.h.
 *
 * Everything here runs on the dense voxel grid with plain loops, two lattices
 * (push scheme) and double precision. The loops over cells are split into
 * fixed chunks so that every sum is taken in the same order whatever the
 * thread count.
 */
#include "cdi_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CHUNK 4096

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Geometry (Sec. 2: every grid block is one voxel of the electrode image).  */
/* ------------------------------------------------------------------------ */

static int64_t fdiv(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

static int64_t wrapi(int64_t i, int64_t n)
{
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

int oracle_voxelize(int dim, int nx, int ny, int nz, int walls_y, int buffer_x,
                    const int64_t *prims, int64_t nprims, uint8_t *labels)
{
    if (dim == 2) nz = 1;
    const int64_t nvox = (int64_t)nx * ny * nz;
    for (int64_t v = 0; v < nvox; ++v) labels[v] = 0;
    if (dim == 2 && walls_y) {
        for (int x = 0; x < nx; ++x) {
            labels[x] = 2;
            labels[(int64_t)(ny - 1) * nx + x] = 2;
        }
    }
    /* Voxel (i,j,k) has its centre at (i+1/2, j+1/2, k+1/2); in 1/256 units
     * that is 128*(2i+1). A voxel is solid iff some primitive contains its
     * centre (distance <= radius), tested in exact integer arithmetic. */
    for (int64_t p = 0; p < nprims; ++p) {
        const int64_t r = prims[4 * p], cx = prims[4 * p + 1], cy = prims[4 * p + 2],
                      cz = prims[4 * p + 3];
        const int64_t i0 = fdiv(cx - r, 256) - 1, i1 = fdiv(cx + r, 256) + 1;
        const int64_t j0 = fdiv(cy - r, 256) - 1, j1 = fdiv(cy + r, 256) + 1;
        int64_t k0 = 0, k1 = 0;
        if (dim == 3) {
            k0 = fdiv(cz - r, 256) - 1;
            k1 = fdiv(cz + r, 256) + 1;
        }
        for (int64_t k = k0; k <= k1; ++k) {
            const int64_t dz = (dim == 3) ? 128 * (2 * k + 1) - cz : 0;
            const int64_t kk = (dim == 3) ? wrapi(k, nz) : 0;
            for (int64_t j = j0; j <= j1; ++j) {
                int64_t jj;
                if (dim == 2 && walls_y) {
                    if (j < 0 || j >= ny) continue;
                    jj = j;
                } else {
                    jj = wrapi(j, ny);
                }
                const int64_t dy = 128 * (2 * j + 1) - cy;
                for (int64_t i = i0; i <= i1; ++i) {
                    if (i < buffer_x || i >= nx - buffer_x) continue;
                    const int64_t dx = 128 * (2 * i + 1) - cx;
                    if (dx * dx + dy * dy + dz * dz <= r * r) {
                        uint8_t *l = &labels[(kk * ny + jj) * nx + i];
                        if (*l != 2) *l = 1;
                    }
                }
            }
        }
    }
    return ORACLE_OK;
}

/* Straight fibres (Sec. 5): a voxel of the interior slab is electrode iff
 * its centre c lies within r of some fibre's infinite core line o + t d, i.e.
 * |(c - o) x d|^2 <= r^2 |d|^2, in exact integer arithmetic (1/256 units).
 * Every voxel is tested against every fibre. */
int oracle_voxelize_fibres(int nx, int ny, int nz, int buffer_x, const int64_t *fibres, int64_t nfib,
                           uint8_t *labels)
{
    const int64_t nvox = (int64_t)nx * ny * nz;
    for (int64_t v = 0; v < nvox; ++v) labels[v] = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < nz; ++k) {
        for (int j = 0; j < ny; ++j) {
            for (int i = buffer_x; i < nx - buffer_x; ++i) {
                const int64_t c[3] = {128 * (2 * (int64_t)i + 1), 128 * (2 * (int64_t)j + 1),
                                      128 * (2 * (int64_t)k + 1)};
                for (int64_t f = 0; f < nfib; ++f) {
                    const int64_t *F = fibres + 8 * f;
                    const int64_t vx = c[0] - F[1], vy = c[1] - F[2], vz = c[2] - F[3];
                    const int64_t dx = F[4], dy = F[5], dz = F[6];
                    const int64_t ax = vy * dz - vz * dy, ay = vz * dx - vx * dz, az = vx * dy - vy * dx;
                    if (ax * ax + ay * ay + az * az <= F[0] * F[0] * (dx * dx + dy * dy + dz * dz)) {
                        labels[((int64_t)k * ny + j) * nx + i] = 1;
                        break;
                    }
                }
            }
        }
    }
    return ORACLE_OK;
}

int64_t oracle_compact(const uint8_t *labels, int64_t nvox, int32_t *map, int32_t *fluid)
{
    int64_t n = 0;
    for (int64_t v = 0; v < nvox; ++v) {
        if (labels[v] == 0) {
            if (map) map[v] = (int32_t)n;
            if (fluid) fluid[n] = (int32_t)v;
            ++n;
        } else if (map) {
            map[v] = labels[v] == 1 ? -1 : -2;
        }
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Lattices (LBM paragraph: D2Q9 and D3Q19, nu = (tau - 1/2)/3).             */
/* ------------------------------------------------------------------------ */

static const int E2[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                             {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W2[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int E3[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W3[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

struct oracle_solver {
    oracle_cfg cfg;
    int Q;
    int e[19][3];
    double w[19];
    int opp[19];
    int64_t nvox, nf;
    uint8_t *labels;
    int32_t *map, *fluid;
    double *f, *fn;     /* Q x nvox */
    double *u;          /* 3 x nvox: advecting velocity of Nernst-Planck (mass flux j) */
    double *unew;       /* 3 x nvox scratch */
    double *uprev;      /* 3 x nvox residual scratch */
    double *C, *Cn;     /* 2 x nvox */
    double *psi;        /* nvox */
    int psi_is_field;
    int u_valid;
    double ka, keff[2];
    double acc[2][3];   /* A, In, Out */
    int64_t flow_steps, np_steps;
};

int64_t oracle_num_fluid(const oracle_solver *s) { return s->nf; }
double oracle_ka(const oracle_solver *s) { return s->ka; }
int64_t oracle_flow_step_count(const oracle_solver *s) { return s->flow_steps; }
int64_t oracle_np_step_count(const oracle_solver *s) { return s->np_steps; }

static void vox_xyz(const oracle_solver *s, int64_t v, int *x, int *y, int *z)
{
    const oracle_cfg *c = &s->cfg;
    *x = (int)(v % c->nx);
    *y = (int)((v / c->nx) % c->ny);
    *z = (int)(v / ((int64_t)c->nx * c->ny));
}

/* Equilibrium of the BGK model, Eq. (8): the standard second-order
 * polynomial in u (quadratic), or its Stokes-limit linear part. */
static double feq(const oracle_solver *s, int i, double rho, const double u[3])
{
    const double eu = s->e[i][0] * u[0] + s->e[i][1] * u[1] + s->e[i][2] * u[2];
    if (s->cfg.equilibrium == ORACLE_EQ_LINEAR) return s->w[i] * rho * (1.0 + 3.0 * eu);
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return s->w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

/* rho = sum f, u = (sum e f + F/2) / rho (Guo et al. 2002 forcing adds F/2;
 * F = 0 without a body force). */
static void moments(const oracle_solver *s, const double *f, int64_t v, int with_force,
                    double *rho, double u[3])
{
    double r = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < s->Q; ++i) {
        const double fi = f[(int64_t)i * s->nvox + v];
        r += fi;
        j[0] += s->e[i][0] * fi;
        j[1] += s->e[i][1] * fi;
        j[2] += s->e[i][2] * fi;
    }
    if (with_force && s->cfg.drive == ORACLE_DRIVE_BODY_FORCE) {
        for (int a = 0; a < 3; ++a) j[a] += 0.5 * s->cfg.force[a];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
}

/* Neighbour voxel of v along offset (dx,dy,dz): y and z wrap; x wraps only
 * when periodic_x, otherwise -1 is returned for a step out of the domain. */
static int64_t neighbour(const oracle_solver *s, int64_t v, int dx, int dy, int dz, int periodic_x)
{
    const oracle_cfg *c = &s->cfg;
    int x, y, z;
    vox_xyz(s, v, &x, &y, &z);
    int xn = x + dx;
    if (xn < 0 || xn >= c->nx) {
        if (!periodic_x) return -1;
        xn = (int)wrapi(xn, c->nx);
    }
    const int yn = (int)wrapi(y + dy, c->ny);
    const int zn = (int)wrapi(z + dz, c->nz);
    return ((int64_t)zn * c->ny + yn) * c->nx + xn;
}

oracle_solver *oracle_create(const oracle_cfg *cfg, const uint8_t *labels, const double *psi_fluid)
{
    if (!cfg || !labels) return NULL;
    if (!(cfg->dim == 2 || cfg->dim == 3) || cfg->nx < 4 || cfg->ny < 1 || cfg->nz < 1) return NULL;
    if (!(cfg->tau > 0.5) || cfg->np_substeps < 1) return NULL;
    oracle_solver *s = (oracle_solver *)calloc(1, sizeof(oracle_solver));
    if (!s) return NULL;
    s->cfg = *cfg;
    if (cfg->dim == 2) s->cfg.nz = 1;
    const oracle_cfg *c = &s->cfg;
    s->Q = cfg->dim == 2 ? 9 : 19;
    for (int i = 0; i < s->Q; ++i) {
        for (int a = 0; a < 3; ++a) s->e[i][a] = cfg->dim == 2 ? E2[i][a] : E3[i][a];
        s->w[i] = cfg->dim == 2 ? W2[i] : W3[i];
    }
    for (int i = 0; i < s->Q; ++i)
        for (int k = 0; k < s->Q; ++k)
            if (s->e[k][0] == -s->e[i][0] && s->e[k][1] == -s->e[i][1] && s->e[k][2] == -s->e[i][2])
                s->opp[i] = k;
    s->nvox = (int64_t)c->nx * c->ny * c->nz;
    const int64_t nv = s->nvox;
    s->labels = (uint8_t *)malloc((size_t)nv);
    s->map = (int32_t *)malloc(sizeof(int32_t) * (size_t)nv);
    s->fluid = (int32_t *)malloc(sizeof(int32_t) * (size_t)nv);
    s->f = (double *)calloc((size_t)(s->Q * nv), sizeof(double));
    s->fn = (double *)calloc((size_t)(s->Q * nv), sizeof(double));
    s->u = (double *)calloc((size_t)(3 * nv), sizeof(double));
    s->unew = (double *)calloc((size_t)(3 * nv), sizeof(double));
    s->uprev = (double *)calloc((size_t)(3 * nv), sizeof(double));
    s->C = (double *)calloc((size_t)(2 * nv), sizeof(double));
    s->Cn = (double *)calloc((size_t)(2 * nv), sizeof(double));
    s->psi = (double *)calloc((size_t)nv, sizeof(double));
    if (!s->labels || !s->map || !s->fluid || !s->f || !s->fn || !s->u || !s->unew || !s->uprev ||
        !s->C || !s->Cn || !s->psi) {
        oracle_destroy(s);
        return NULL;
    }
    memcpy(s->labels, labels, (size_t)nv);
    s->nf = oracle_compact(s->labels, nv, s->map, s->fluid);

    /* Initial state: fluid at rest (rho = 1, u = 0), C = c0 everywhere
     * ("initially saturated"). */
    for (int64_t v = 0; v < nv; ++v) {
        if (s->labels[v] != 0) continue;
        for (int i = 0; i < s->Q; ++i) s->f[(int64_t)i * nv + v] = s->w[i];
        s->C[v] = cfg->c0;
        s->C[nv + v] = cfg->c0;
    }
    /* Potential: prescribed field, or a linear ramp high at the inlet. */
    if (psi_fluid) {
        s->psi_is_field = 1;
        for (int64_t n = 0; n < s->nf; ++n) s->psi[s->fluid[n]] = psi_fluid[n];
    } else {
        for (int64_t v = 0; v < nv; ++v) {
            int x, y, z;
            vox_xyz(s, v, &x, &y, &z);
            s->psi[v] = cfg->dpsi * (1.0 - (x + 0.5) / c->nx);
        }
    }
    /* Adsorption constant: given; <= 0 selects the paper's Da/Pe ratio of its
     * base case (Da = 4.28e-3 at Pe = 1.03e-2) times the mean pore velocity
     * u_in/phi; none with no_adsorption (a blocking electrode, as the charged
     * wall of the electromigration check of Sec. 3). */
    const double phi = (double)s->nf / (double)nv;
    s->ka = cfg->no_adsorption ? 0.0 : cfg->Ka > 0 ? cfg->Ka : (4.28e-3 / 1.03e-2) * cfg->u_in / phi;
    /* Robin law D dC/dn = Ka C (Eq. 6) across half a cell: the wall value is
     * eliminated, giving the face flux k_eff * C_P. */
    for (int sp = 0; sp < 2; ++sp) s->keff[sp] = s->ka * cfg->D[sp] / (cfg->D[sp] + 0.5 * s->ka);
    return s;
}

void oracle_destroy(oracle_solver *s)
{
    if (!s) return;
    free(s->labels);
    free(s->map);
    free(s->fluid);
    free(s->f);
    free(s->fn);
    free(s->u);
    free(s->unew);
    free(s->uprev);
    free(s->C);
    free(s->Cn);
    free(s->psi);
    free(s);
}

/* ------------------------------------------------------------------------ */
/* LBM step: Eq. (7) with the BGK collision of Eq. (8).                      */
/* ------------------------------------------------------------------------ */

static void lbm_step(oracle_solver *s)
{
    const oracle_cfg *c = &s->cfg;
    const int64_t nv = s->nvox;
    const int Q = s->Q;
    const int periodic_x = c->drive == ORACLE_DRIVE_BODY_FORCE;
    const double tau = c->tau;
    const double *F = c->force;
    const int forced = c->drive == ORACLE_DRIVE_BODY_FORCE;

#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        double rho, u[3];
        moments(s, s->f, v, 1, &rho, u);
        for (int i = 0; i < Q; ++i) {
            const double fi = s->f[(int64_t)i * nv + v];
            double fs = fi - (fi - feq(s, i, rho, u)) / tau;
            if (forced) {
                /* Guo, Zheng & Shi (2002) source term. */
                const double eu = s->e[i][0] * u[0] + s->e[i][1] * u[1] + s->e[i][2] * u[2];
                double src = 0;
                for (int a = 0; a < 3; ++a)
                    src += (3.0 * (s->e[i][a] - u[a]) + 9.0 * eu * s->e[i][a]) * F[a];
                fs += (1.0 - 0.5 / tau) * s->w[i] * src;
            }
            /* Stream to x + e_i; a solid target reflects the population back
             * into the opposite direction of this node (half-way bounce-back,
             * the no-flow rule at solid-fluid interfaces). */
            const int64_t t = neighbour(s, v, s->e[i][0], s->e[i][1], s->e[i][2], periodic_x);
            if (t < 0) continue; /* leaves through an open x end */
            if (s->labels[t] != 0)
                s->fn[(int64_t)s->opp[i] * nv + v] = fs;
            else
                s->fn[(int64_t)i * nv + t] = fs;
        }
    }

    if (c->drive == ORACLE_DRIVE_INLET_OUTLET) {
        /* Non-equilibrium extrapolation (Guo, Zheng & Shi 2002) on the planes
         * x = 0 (velocity u_in) and x = nx-1 (density rho_out), from the
         * neighbour one plane inside, after streaming. */
        for (int side = 0; side < 2; ++side) {
            const int xb = side == 0 ? 0 : c->nx - 1;
            const int xn = side == 0 ? 1 : c->nx - 2;
            for (int z = 0; z < c->nz; ++z)
                for (int y = 0; y < c->ny; ++y) {
                    const int64_t vb = ((int64_t)z * c->ny + y) * c->nx + xb;
                    const int64_t vn = ((int64_t)z * c->ny + y) * c->nx + xn;
                    if (s->labels[vb] != 0 || s->labels[vn] != 0) continue;
                    double rn, un[3];
                    moments(s, s->fn, vn, 0, &rn, un);
                    double rb, ub[3];
                    if (side == 0) {
                        rb = rn;
                        ub[0] = c->u_in;
                        ub[1] = 0;
                        ub[2] = 0;
                    } else {
                        rb = c->rho_out;
                        ub[0] = un[0];
                        ub[1] = un[1];
                        ub[2] = un[2];
                    }
                    for (int i = 0; i < Q; ++i) {
                        const double fneq = s->fn[(int64_t)i * nv + vn] - feq(s, i, rn, un);
                        s->fn[(int64_t)i * nv + vb] = feq(s, i, rb, ub) + fneq;
                    }
                }
        }
    }
    double *t = s->f;
    s->f = s->fn;
    s->fn = t;
    s->flow_steps++;
}

void oracle_flow_steps(oracle_solver *s, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) lbm_step(s);
    s->u_valid = 0;
}

static void velocity_field(const oracle_solver *s, double *u3)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        double rho, u[3];
        moments(s, s->f, v, 1, &rho, u);
        for (int a = 0; a < 3; ++a) u3[(int64_t)a * s->nvox + v] = u[a];
    }
}

/* Mass flux j = rho u = sum e f (+ F/2) of the current populations: the
 * velocity that advects the ions (rho_0 = 1). At steady state the LBM's
 * continuity equation makes j, not u = j / rho, divergence-free. */
static void flux_field(const oracle_solver *s, double *j3)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        double rho, u[3];
        moments(s, s->f, v, 1, &rho, u);
        for (int a = 0; a < 3; ++a) j3[(int64_t)a * s->nvox + v] = rho * u[a];
    }
}

/* Fixed-chunk FP64 sums of |u - uprev|^2 and |u|^2 over fluid nodes. */
static double residual(const oracle_solver *s, const double *u, const double *up)
{
    const int64_t nchunks = (s->nf + CHUNK - 1) / CHUNK;
    double *part = (double *)calloc((size_t)(2 * (nchunks > 0 ? nchunks : 1)), sizeof(double));
    const int d = s->cfg.dim;
#pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        double a = 0, b = 0;
        const int64_t n1 = (ch + 1) * CHUNK < s->nf ? (ch + 1) * CHUNK : s->nf;
        for (int64_t n = ch * CHUNK; n < n1; ++n) {
            const int64_t v = s->fluid[n];
            for (int k = 0; k < d; ++k) {
                const double du = u[(int64_t)k * s->nvox + v] - up[(int64_t)k * s->nvox + v];
                a += du * du;
                b += u[(int64_t)k * s->nvox + v] * u[(int64_t)k * s->nvox + v];
            }
        }
        part[2 * ch] = a;
        part[2 * ch + 1] = b;
    }
    double num = 0, den = 0;
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        num += part[2 * ch];
        den += part[2 * ch + 1];
    }
    free(part);
    return sqrt(num) / sqrt(den);
}

int oracle_flow_to_steady(oracle_solver *s, double tol, int64_t max_steps, int check_every,
                          int64_t *steps_out, double *residual_out)
{
    /* Step t (0-based within this call) moves the state from f^t to f^{t+1}
     * and sees u^t = velocity of f^t. Step t = K-1 (mod K) records u^t; step
     * t = 0 (mod K), t > 0, evaluates r = |u^t - u^{t-1}| / |u^t|. The call
     * stops after that step if r <= tol. */
    if (check_every < 2 || max_steps < 0) return ORACLE_E_INVALID;
    const int K = check_every;
    double r = INFINITY;
    int rc = ORACLE_E_NOT_CONVERGED;
    int64_t t = 0;
    for (; t < max_steps; ++t) {
        int stop = 0;
        if (t % K == K - 1) velocity_field(s, s->uprev);
        if (t > 0 && t % K == 0) {
            velocity_field(s, s->unew);
            r = residual(s, s->unew, s->uprev);
            if (!isfinite(r)) {
                rc = ORACLE_E_DIVERGED;
                lbm_step(s);
                ++t;
                break;
            }
            if (r <= tol) stop = 1;
        }
        lbm_step(s);
        if (stop) {
            rc = ORACLE_OK;
            ++t;
            break;
        }
    }
    s->u_valid = 0;
    if (steps_out) *steps_out = t;
    if (residual_out) *residual_out = r;
    return rc;
}

void oracle_get_velocity(const oracle_solver *s, double *u)
{
    for (int64_t n = 0; n < s->nf; ++n) {
        double rho, uu[3];
        moments(s, s->f, s->fluid[n], 1, &rho, uu);
        for (int a = 0; a < s->cfg.dim; ++a) u[(int64_t)a * s->nf + n] = uu[a];
    }
}

void oracle_get_density(const oracle_solver *s, double *rho)
{
    for (int64_t n = 0; n < s->nf; ++n) {
        double uu[3];
        moments(s, s->f, s->fluid[n], 1, &rho[n], uu);
    }
}

void oracle_get_populations(const oracle_solver *s, double *f)
{
    for (int i = 0; i < s->Q; ++i)
        for (int64_t n = 0; n < s->nf; ++n) f[(int64_t)i * s->nf + n] = s->f[(int64_t)i * s->nvox + s->fluid[n]];
}

void oracle_init_equilibrium(oracle_solver *s, const double *rho, const double *u)
{
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        const double r = rho ? rho[n] : 1.0;
        double uu[3] = {0, 0, 0};
        for (int a = 0; a < s->cfg.dim; ++a) uu[a] = u ? u[(int64_t)a * s->nf + n] : 0.0;
        for (int i = 0; i < s->Q; ++i) s->f[(int64_t)i * s->nvox + v] = feq(s, i, r, uu);
    }
    s->u_valid = 0;
}

void oracle_freeze_velocity(oracle_solver *s)
{
    flux_field(s, s->u);
    s->u_valid = 1;
}

void oracle_set_velocity(oracle_solver *s, const double *u)
{
    memset(s->u, 0, sizeof(double) * (size_t)(3 * s->nvox));
    for (int a = 0; a < s->cfg.dim; ++a)
        for (int64_t n = 0; n < s->nf; ++n) s->u[(int64_t)a * s->nvox + s->fluid[n]] = u[(int64_t)a * s->nf + n];
    s->u_valid = 1;
}

void oracle_get_np_velocity(const oracle_solver *s, double *u)
{
    for (int a = 0; a < s->cfg.dim; ++a)
        for (int64_t n = 0; n < s->nf; ++n) u[(int64_t)a * s->nf + n] = s->u[(int64_t)a * s->nvox + s->fluid[n]];
}

/* ------------------------------------------------------------------------ */
/* Nernst-Planck, Eq. (3), finite volumes on the fluid voxels.               */
/* ------------------------------------------------------------------------ */

/* Bernoulli function B(x) = x / (e^x - 1), B(0) = 1. */
static double bern(double x)
{
    if (x == 0.0) return 1.0;
    return x / expm1(x);
}

/* Scharfetter-Gummel flux from P to N across a unit face: w is the normal
 * drift velocity (advection plus migration), D the diffusivity. This is the
 * exact flux of the 1D steady constant-coefficient equation between the two
 * cell centres. */
static double sg_flux(double D, double w, double cp, double cn)
{
    const double pe = w / D;
    return D * (bern(-pe) * cp - bern(pe) * cn);
}

static double ramp_psi(const oracle_solver *s, int x)
{
    return s->cfg.dpsi * (1.0 - (x + 0.5) / s->cfg.nx);
}

/* Per-cell update for species sp. Writes the outflow sum (per unit time) and
 * the per-category fluxes. If diag is non-NULL it receives the sum of the
 * coefficients multiplying C_P (positivity bound). */
static double cell_outflow(const oracle_solver *s, int64_t v, int sp, const double *C,
                           double *fa, double *fin, double *fout, double *diag)
{
    const oracle_cfg *c = &s->cfg;
    const int d = c->dim;
    const double D = c->D[sp];
    const double z = (double)c->z[sp];
    const double cp = C[(int64_t)sp * s->nvox + v];
    const double psip = s->psi[v];
    int x, y, zc;
    vox_xyz(s, v, &x, &y, &zc);
    double out = 0, dg = 0;
    *fa = 0;
    *fin = 0;
    *fout = 0;
    for (int axis = 0; axis < d; ++axis) {
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            int off[3] = {0, 0, 0};
            off[axis] = sgn;
            if (axis == 0 && (x + sgn < 0 || x + sgn >= c->nx) && c->np_x_bc != ORACLE_NPX_PERIODIC) {
                if (c->np_x_bc == ORACLE_NPX_CLOSED) continue;
                const int inlet = (x + sgn < 0);
                if (inlet) {
                    /* Dirichlet ghost at the feed concentration c0 one cell
                     * upstream, entering with the plug velocity u_in. */
                    const double psig = s->psi_is_field ? psip : ramp_psi(s, -1);
                    const double w = -c->u_in - z * D * (psig - psip); /* outward normal -x */
                    const double F = sg_flux(D, w, cp, c->c0);
                    out += F;
                    *fin += -F;
                    dg += D * bern(-w / D);
                } else if (c->np_x_bc == ORACLE_NPX_DIRICHLET) {
                    const double psig = s->psi_is_field ? psip : ramp_psi(s, c->nx);
                    const double w = s->u[v] - z * D * (psig - psip);
                    const double F = sg_flux(D, w, cp, c->c_out);
                    out += F;
                    *fout += F;
                    dg += D * bern(-w / D);
                } else {
                    /* Open outlet: no diffusive flux (zero gradient); the
                     * normal drift carries C_P out, or carries feed solution
                     * c0 in where it points into the domain. */
                    const double psig = s->psi_is_field ? psip : ramp_psi(s, c->nx);
                    const double w = s->u[v] - z * D * (psig - psip);
                    const double F = (w > 0 ? w : 0.0) * cp + (w < 0 ? w : 0.0) * c->c0;
                    out += F;
                    *fout += F;
                    dg += (w > 0 ? w : 0.0);
                }
                continue;
            }
            const int64_t vn = neighbour(s, v, off[0], off[1], off[2], 1);
            const uint8_t L = s->labels[vn];
            if (L == 1) {
                /* adsorbing electrode face, Eq. (6) */
                const double F = s->keff[sp] * cp;
                out += F;
                *fa += F;
                dg += s->keff[sp];
            } else if (L == 0) {
                const double un = 0.5 * (s->u[(int64_t)axis * s->nvox + v] + s->u[(int64_t)axis * s->nvox + vn]) * sgn;
                /* The applied ramp is a uniform field: across the seam of
                 * periodic ions its step is the same as on every x face (the
                 * stored ramp values would jump by the whole drop there). */
                const int seam = axis == 0 && (x + sgn < 0 || x + sgn >= c->nx);
                const double dpsi = (seam && !s->psi_is_field) ? -sgn * c->dpsi / c->nx : s->psi[vn] - psip;
                const double w = un - z * D * dpsi;
                out += sg_flux(D, w, cp, C[(int64_t)sp * s->nvox + vn]);
                dg += D * bern(-w / D);
            }
            /* L == 2: inert wall, no flux */
        }
    }
    if (diag) *diag = dg;
    return out;
}

double oracle_np_stability(const oracle_solver *s)
{
    const double dt = 1.0 / s->cfg.np_substeps;
    double worst = 0;
    for (int64_t n = 0; n < s->nf; ++n) {
        for (int sp = 0; sp < 2; ++sp) {
            double a, b, c, dg;
            cell_outflow(s, s->fluid[n], sp, s->C, &a, &b, &c, &dg);
            if (dt * dg > worst) worst = dt * dg;
        }
    }
    return worst;
}

static void np_substep(oracle_solver *s, double dt)
{
    const int64_t nchunks = (s->nf + CHUNK - 1) / CHUNK;
    double *part = (double *)calloc((size_t)(6 * (nchunks > 0 ? nchunks : 1)), sizeof(double));
    const int64_t nv = s->nvox;
#pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        double p[6] = {0, 0, 0, 0, 0, 0};
        const int64_t n1 = (ch + 1) * CHUNK < s->nf ? (ch + 1) * CHUNK : s->nf;
        for (int64_t n = ch * CHUNK; n < n1; ++n) {
            const int64_t v = s->fluid[n];
            for (int sp = 0; sp < 2; ++sp) {
                double fa, fi, fo;
                const double out = cell_outflow(s, v, sp, s->C, &fa, &fi, &fo, NULL);
                /* forward Euler, all faces from C^n */
                s->Cn[(int64_t)sp * nv + v] = s->C[(int64_t)sp * nv + v] - dt * out;
                p[3 * sp + 0] += dt * fa;
                p[3 * sp + 1] += dt * fi;
                p[3 * sp + 2] += dt * fo;
            }
        }
        for (int k = 0; k < 6; ++k) part[6 * ch + k] = p[k];
    }
    for (int64_t ch = 0; ch < nchunks; ++ch)
        for (int sp = 0; sp < 2; ++sp)
            for (int k = 0; k < 3; ++k) s->acc[sp][k] += part[6 * ch + 3 * sp + k];
    free(part);
    double *t = s->C;
    s->C = s->Cn;
    s->Cn = t;
}

int oracle_np_steps(oracle_solver *s, int64_t n, int fused)
{
    if (!s->u_valid) oracle_freeze_velocity(s);
    if (oracle_np_stability(s) > 1.0) return ORACLE_E_UNSTABLE;
    const double dt = 1.0 / s->cfg.np_substeps;
    for (int64_t k = 0; k < n; ++k) {
        if (fused) flux_field(s, s->unew); /* j^n of the state this step starts from */
        for (int m = 0; m < s->cfg.np_substeps; ++m) np_substep(s, dt);
        if (fused) {
            lbm_step(s);
            double *t = s->u;
            s->u = s->unew;
            s->unew = t;
        }
        s->np_steps++;
    }
    return ORACLE_OK;
}

void oracle_get_conc(const oracle_solver *s, double *c)
{
    for (int sp = 0; sp < 2; ++sp)
        for (int64_t n = 0; n < s->nf; ++n) c[(int64_t)sp * s->nf + n] = s->C[(int64_t)sp * s->nvox + s->fluid[n]];
}

void oracle_set_conc(oracle_solver *s, const double *c)
{
    for (int sp = 0; sp < 2; ++sp)
        for (int64_t n = 0; n < s->nf; ++n) s->C[(int64_t)sp * s->nvox + s->fluid[n]] = c[(int64_t)sp * s->nf + n];
}

void oracle_balance(const oracle_solver *s, double *out)
{
    for (int sp = 0; sp < 2; ++sp) {
        double m = 0;
        for (int64_t n = 0; n < s->nf; ++n) m += s->C[(int64_t)sp * s->nvox + s->fluid[n]];
        out[4 * sp + 0] = m;
        out[4 * sp + 1] = s->acc[sp][0];
        out[4 * sp + 2] = s->acc[sp][1];
        out[4 * sp + 3] = s->acc[sp][2];
    }
}

void oracle_adsorbed_total(const oracle_solver *s, double out[2])
{
    out[0] = s->acc[0][0];
    out[1] = s->acc[1][0];
}

/* ------------------------------------------------------------------------ */
/* Electric potential, Eq. (4)-(5), in thermal voltages psi~ = e psi / k_BT. */
/* ------------------------------------------------------------------------ */
/*
 * Finite volumes on the fluid voxels, one unknown per cell centre. The flux
 * of grad psi through a face between two fluid cells is psi_N - psi_P. At a
 * face shared with an electrode voxel the paper's Dirichlet condition holds
 * on the face itself, half a cell from the centre: flux 2 (psi_e - psi_P).
 * Inert walls carry no field (zero normal derivative). Each x end is either
 * a Dirichlet face (value psi_x[end], half a cell away), a zero-field face,
 * or periodic (both ends). With psi~ and the Debye length lambda_D of a
 * symmetric electrolyte at c0 (lambda_D^2 = eps_r eps_0 k_B T / (2 e F c0),
 * the length of Eq. (10)), Eq. (4) with the charge of Eq. (5) reads
 *   lap psi~ = -(kappa2 / (2 c0)) sum_i z_i C_i,  kappa2 = (h / lambda_D)^2,
 * so a cell balances sum(face fluxes) + (kappa2 / (2 c0)) sum_i z_i C_i = 0.
 * Written as A psi = b with A symmetric positive definite when at least one
 * Dirichlet face exists: A_PP = sum of face coefficients (1 per fluid face,
 * 2 per Dirichlet face), A_PN = -1, b_P = source + sum 2 psi_face. Solved by
 * conjugate gradients (Hestenes-Stiefel) with the diagonal as preconditioner.
 */
static int pot_face(const oracle_solver *s, const oracle_potential *pc, int64_t v, int axis, int sgn,
                    int64_t *vn, double *value)
{
    const oracle_cfg *c = &s->cfg;
    int x, y, z;
    vox_xyz(s, v, &x, &y, &z);
    int off[3] = {0, 0, 0};
    off[axis] = sgn;
    if (axis == 0 && (x + sgn < 0 || x + sgn >= c->nx) && pc->x_bc[0] != ORACLE_PSIX_PERIODIC) {
        const int end = x + sgn < 0 ? 0 : 1;
        if (pc->x_bc[end] == ORACLE_PSIX_NEUMANN) return 0;
        *value = pc->psi_x[end];
        return 2;
    }
    const int64_t n = neighbour(s, v, off[0], off[1], off[2], 1);
    if (s->labels[n] == 0) {
        *vn = n;
        return 1;
    }
    if (s->labels[n] == 1) {
        *value = pc->psi_electrode;
        return 2;
    }
    return 0; /* inert wall */
}

/* q = A p over the fluid cells (p, q: nvox arrays, fluid entries used). */
static void pot_apply(const oracle_solver *s, const oracle_potential *pc, const double *p, double *q)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        double acc = 0;
        for (int axis = 0; axis < s->cfg.dim; ++axis)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int64_t vn = -1;
                double val = 0;
                const int kind = pot_face(s, pc, v, axis, sgn, &vn, &val);
                if (kind == 1) acc += p[v] - p[vn];
                else if (kind == 2) acc += 2.0 * p[v];
            }
        q[v] = acc;
    }
}

/* Sum over fluid cells of a[v] * b[v] in fixed chunks (same order for any
 * thread count). */
static double pot_dot(const oracle_solver *s, const double *a, const double *b)
{
    const int64_t nchunks = (s->nf + CHUNK - 1) / CHUNK;
    double *part = (double *)calloc((size_t)(nchunks > 0 ? nchunks : 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int64_t n1 = (ch + 1) * CHUNK < s->nf ? (ch + 1) * CHUNK : s->nf;
        double t = 0;
        for (int64_t n = ch * CHUNK; n < n1; ++n) t += a[s->fluid[n]] * b[s->fluid[n]];
        part[ch] = t;
    }
    double t = 0;
    for (int64_t ch = 0; ch < nchunks; ++ch) t += part[ch];
    free(part);
    return t;
}

int oracle_solve_potential(oracle_solver *s, const oracle_potential *pc, int *iters, double *relres)
{
    if (!s || !pc || pc->max_iter < 0 || !(pc->tol >= 0)) return ORACLE_E_INVALID;
    if ((pc->x_bc[0] == ORACLE_PSIX_PERIODIC) != (pc->x_bc[1] == ORACLE_PSIX_PERIODIC))
        return ORACLE_E_INVALID;
    const oracle_cfg *c = &s->cfg;
    const int64_t nv = s->nvox;
    double *x = (double *)calloc((size_t)nv, sizeof(double));
    double *r = (double *)calloc((size_t)nv, sizeof(double));
    double *zv = (double *)calloc((size_t)nv, sizeof(double));
    double *p = (double *)calloc((size_t)nv, sizeof(double));
    double *q = (double *)calloc((size_t)nv, sizeof(double));
    double *dg = (double *)calloc((size_t)nv, sizeof(double));
    if (!x || !r || !zv || !p || !q || !dg) {
        free(x), free(r), free(zv), free(p), free(q), free(dg);
        return ORACLE_E_INVALID;
    }
    /* right-hand side and diagonal */
    int64_t n_dirichlet = 0;
    const double src = pc->kappa2 / (2.0 * c->c0);
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        double b = src * (c->z[0] * s->C[v] + c->z[1] * s->C[nv + v]);
        double d = 0;
        for (int axis = 0; axis < c->dim; ++axis)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int64_t vn = -1;
                double val = 0;
                const int kind = pot_face(s, pc, v, axis, sgn, &vn, &val);
                if (kind == 1) d += 1.0;
                else if (kind == 2) {
                    d += 2.0;
                    b += 2.0 * val;
                    ++n_dirichlet;
                }
            }
        r[v] = b; /* x0 = 0 */
        dg[v] = d;
    }
    int rc = ORACLE_OK;
    int k = 0;
    double rel = 0;
    if (n_dirichlet == 0) {
        rc = ORACLE_E_INVALID; /* the potential would be defined up to a constant only */
    } else {
        const double bnorm = sqrt(pot_dot(s, r, r));
        for (int64_t n = 0; n < s->nf; ++n) {
            const int64_t v = s->fluid[n];
            zv[v] = dg[v] > 0 ? r[v] / dg[v] : 0.0;
            p[v] = zv[v];
        }
        double rz = pot_dot(s, r, zv);
        double rr = bnorm * bnorm;
        rel = bnorm > 0 ? 1.0 : 0.0;
        while (bnorm > 0 && sqrt(rr) > pc->tol * bnorm) {
            if (k >= pc->max_iter) {
                rc = ORACLE_E_NOT_CONVERGED;
                break;
            }
            pot_apply(s, pc, p, q);
            const double alpha = rz / pot_dot(s, p, q);
            for (int64_t n = 0; n < s->nf; ++n) {
                const int64_t v = s->fluid[n];
                x[v] += alpha * p[v];
                r[v] -= alpha * q[v];
                zv[v] = dg[v] > 0 ? r[v] / dg[v] : 0.0;
            }
            const double rz_new = pot_dot(s, r, zv);
            rr = pot_dot(s, r, r);
            const double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t n = 0; n < s->nf; ++n) {
                const int64_t v = s->fluid[n];
                p[v] = zv[v] + beta * p[v];
            }
            ++k;
            if (!isfinite(rr)) {
                rc = ORACLE_E_DIVERGED;
                break;
            }
        }
        if (bnorm > 0) rel = sqrt(rr) / bnorm;
        if (rc == ORACLE_OK || rc == ORACLE_E_NOT_CONVERGED) {
            for (int64_t n = 0; n < s->nf; ++n) s->psi[s->fluid[n]] = x[s->fluid[n]];
            s->psi_is_field = 1;
        }
    }
    if (iters) *iters = k;
    if (relres) *relres = rel;
    free(x), free(r), free(zv), free(p), free(q), free(dg);
    return rc;
}

void oracle_get_potential(const oracle_solver *s, double *psi)
{
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        psi[n] = s->psi[v]; /* the ramp's values when no field was set or solved */
    }
}

/* Coupled Poisson-Nernst-Planck: before every `every`-th ion step the
 * potential is solved afresh from the concentrations the step starts from
 * (Eq. 4-5), then the step runs on it (Eq. 3): an explicit, lagged coupling. */
int oracle_np_steps_coupled(oracle_solver *s, int64_t n, int fused, const oracle_potential *pc, int every)
{
    if (!s || !pc || every < 1 || n < 0) return ORACLE_E_INVALID;
    for (int64_t k = 0; k < n; ++k) {
        if (k % every == 0) {
            const int rc = oracle_solve_potential(s, pc, NULL, NULL);
            if (rc != ORACLE_OK) return rc;
        }
        const int rc = oracle_np_steps(s, 1, fused);
        if (rc != ORACLE_OK) return rc;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics of Sec. 4: Pe, Da, l_c = pi / s, U, vertical averages.        */
/* ------------------------------------------------------------------------ */

void oracle_diagnostics(const oracle_solver *s, oracle_diag *out)
{
    const oracle_cfg *c = &s->cfg;
    const int periodic_x = c->drive == ORACLE_DRIVE_BODY_FORCE;
    int64_t faces = 0, inlet = 0;
    double usum = 0;
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        for (int axis = 0; axis < c->dim; ++axis)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                int off[3] = {0, 0, 0};
                off[axis] = sgn;
                const int64_t vn = neighbour(s, v, off[0], off[1], off[2], periodic_x);
                if (vn >= 0 && s->labels[vn] == 1) ++faces;
            }
        if (v % c->nx == 0) ++inlet;
        double rho, u[3];
        moments(s, s->f, v, 1, &rho, u);
        usum += u[0];
    }
    out->n_surface = faces;
    out->n_inlet = inlet;
    /* s: electrode surface per unit total volume (faces of unit area over N
     * voxels); l_c = pi / s */
    out->specific_surface = (double)faces / (double)s->nvox;
    out->l_c = faces > 0 ? 3.14159265358979323846 / out->specific_surface : INFINITY;
    /* U = sum_i u_i / (N phi): the streamwise velocity summed over all grid
     * blocks (zero in the solid) over the number of pore blocks */
    out->U = s->nf > 0 ? usum / (double)s->nf : 0.0;
    for (int sp = 0; sp < 2; ++sp) {
        out->Pe[sp] = out->U * out->l_c / c->D[sp];
        out->Da[sp] = s->ka * out->l_c / c->D[sp];
    }
}

void oracle_profile_x(const oracle_solver *s, double *out)
{
    const int nx = s->cfg.nx;
    for (int k = 0; k < 3 * nx; ++k) out[k] = 0;
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        const int x = (int)(v % nx);
        out[x] += s->C[v];
        out[nx + x] += s->C[s->nvox + v];
        out[2 * nx + x] += 1.0;
    }
    for (int x = 0; x < nx; ++x)
        if (out[2 * nx + x] > 0) {
            out[x] /= out[2 * nx + x];
            out[nx + x] /= out[2 * nx + x];
        }
}

/* Salt removal of Sec. 4.1 over a window of nsteps ion steps between two
 * balances: P_rm = (C_in - C_out) / C_in per species, C_in = c0 and C_out the
 * outflowing amount over the volume that entered, u_in n_inlet nsteps;
 * out[2] the mean of the two species; out[3] = U A P_rm dt / (V_t phi) with
 * A = ny nz and V_t phi = N_f. */
void oracle_salt_removal(const oracle_solver *s, const double *bal0, const double *bal1, int64_t nsteps,
                         int64_t n_inlet, double U, double out[4])
{
    const double volume = s->cfg.u_in * (double)n_inlet * (double)nsteps;
    for (int sp = 0; sp < 2; ++sp) {
        const double c_out = (bal1[4 * sp + 3] - bal0[4 * sp + 3]) / volume;
        out[sp] = (s->cfg.c0 - c_out) / s->cfg.c0;
    }
    out[2] = 0.5 * (out[0] + out[1]);
    out[3] = U * (double)s->cfg.ny * (double)s->cfg.nz * out[2] * (double)nsteps / (double)s->nf;
}

/* ------------------------------------------------------------------------ */
/* Implicit Nernst-Planck (the paper's time scheme, Sec. 2) and the steady   */
/* state.                                                                   */
/* ------------------------------------------------------------------------ */
/*
 * For frozen u and psi the outflow of a cell is affine in the concentrations
 * of its species: out(C) = A C - b, with b = -out(0) the ghost (inlet,
 * outlet) terms. A backward-Euler step solves (I/dt + A) C' = C/dt + b; the
 * steady state solves A C = b. Both by BiCGSTAB (van der Vorst 1992) with
 * the diagonal of the matrix as right preconditioner, per species.
 */
typedef struct {
    const oracle_solver *s;
    int sp;
    double idt;   /* 1/dt, 0 for the steady problem */
    double *W;    /* 2 x nvox scratch: the field of species sp goes in its slot */
} np_op;

/* y = (idt I + A) x over the fluid cells (nvox arrays) */
static void np_op_apply(np_op *op, const double *x, double *y)
{
    const oracle_solver *s = op->s;
    const int64_t nv = s->nvox;
    double *slot = op->W + (int64_t)op->sp * nv;
    for (int64_t n = 0; n < s->nf; ++n) slot[s->fluid[n]] = x[s->fluid[n]];
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        double fa, fi, fo;
        const double full = cell_outflow(s, v, op->sp, op->W, &fa, &fi, &fo, NULL);
        y[v] = full + op->idt * x[v];
    }
    /* remove the constant part: out(0) */
    for (int64_t n = 0; n < s->nf; ++n) slot[s->fluid[n]] = 0.0;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        double fa, fi, fo;
        y[v] -= cell_outflow(s, v, op->sp, op->W, &fa, &fi, &fo, NULL);
    }
}

/* diagonal of (idt I + A) and b = -out(0) */
static void np_op_diag_rhs(np_op *op, double *dg, double *b)
{
    const oracle_solver *s = op->s;
    double *slot = op->W + (int64_t)op->sp * s->nvox;
    for (int64_t n = 0; n < s->nf; ++n) slot[s->fluid[n]] = 0.0;
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t v = s->fluid[n];
        double fa, fi, fo, d;
        b[v] = -cell_outflow(s, v, op->sp, op->W, &fa, &fi, &fo, &d);
        dg[v] = d + op->idt;
    }
}

static double np_dot(const oracle_solver *s, const double *a, const double *b) { return pot_dot(s, a, b); }

/* Solve (idt I + A) x = rhs from the start x; returns iterations or -1. */
static int np_bicgstab(np_op *op, const double *rhs, double *x, double tol, int max_iter, double *relres)
{
    const oracle_solver *s = op->s;
    const int64_t nv = s->nvox;
    double *r = calloc((size_t)nv, sizeof(double)), *rh = calloc((size_t)nv, sizeof(double));
    double *p = calloc((size_t)nv, sizeof(double)), *v = calloc((size_t)nv, sizeof(double));
    double *y = calloc((size_t)nv, sizeof(double)), *z = calloc((size_t)nv, sizeof(double));
    double *t = calloc((size_t)nv, sizeof(double)), *sv = calloc((size_t)nv, sizeof(double));
    double *dg = calloc((size_t)nv, sizeof(double)), *bb = calloc((size_t)nv, sizeof(double));
    int it = -1;
    if (!r || !rh || !p || !v || !y || !z || !t || !sv || !dg || !bb) goto done;
    np_op_diag_rhs(op, dg, bb);
    np_op_apply(op, x, t);
    for (int64_t n = 0; n < s->nf; ++n) {
        const int64_t c = s->fluid[n];
        r[c] = rhs[c] - t[c];
        rh[c] = r[c];
    }
    const double bnorm = sqrt(np_dot(s, rhs, rhs));
    double rho = 1, alpha = 1, omega = 1;
    double rn = sqrt(np_dot(s, r, r));
    it = 0;
    while (bnorm > 0 && rn > tol * bnorm && it < max_iter) {
        const double rho1 = np_dot(s, rh, r);
        const double beta = (rho1 / rho) * (alpha / omega);
        rho = rho1;
        for (int64_t n = 0; n < s->nf; ++n) {
            const int64_t c = s->fluid[n];
            p[c] = r[c] + beta * (p[c] - omega * v[c]);
            y[c] = p[c] / dg[c];
        }
        np_op_apply(op, y, v);
        alpha = rho / np_dot(s, rh, v);
        for (int64_t n = 0; n < s->nf; ++n) {
            const int64_t c = s->fluid[n];
            sv[c] = r[c] - alpha * v[c];
            z[c] = sv[c] / dg[c];
        }
        np_op_apply(op, z, t);
        const double tt = np_dot(s, t, t);
        omega = tt > 0 ? np_dot(s, t, sv) / tt : 0.0;
        for (int64_t n = 0; n < s->nf; ++n) {
            const int64_t c = s->fluid[n];
            x[c] += alpha * y[c] + omega * z[c];
            r[c] = sv[c] - omega * t[c];
        }
        rn = sqrt(np_dot(s, r, r));
        ++it;
        if (!isfinite(rn) || omega == 0.0) {
            it = -1;
            break;
        }
    }
    if (relres) *relres = bnorm > 0 ? rn / bnorm : 0.0;
    if (it >= max_iter && rn > tol * bnorm) it = -2;
done:
    free(r), free(rh), free(p), free(v), free(y), free(z), free(t), free(sv), free(dg), free(bb);
    return it;
}

/* Right-hand side b of species sp (the ghost terms) into b. */
static void np_rhs(np_op *op, double *b)
{
    const oracle_solver *s = op->s;
    double *dg = calloc((size_t)s->nvox, sizeof(double));
    np_op_diag_rhs(op, dg, b);
    free(dg);
}

int oracle_np_steady(oracle_solver *s, double tol, int max_iter, int *iters)
{
    if (!s->u_valid) oracle_freeze_velocity(s);
    const int64_t nv = s->nvox;
    double *W = calloc((size_t)(2 * nv), sizeof(double)), *b = calloc((size_t)nv, sizeof(double));
    double *x = calloc((size_t)nv, sizeof(double));
    int rc = ORACLE_OK, tot = 0;
    for (int sp = 0; sp < 2 && rc == ORACLE_OK; ++sp) {
        np_op op = {s, sp, 0.0, W};
        np_rhs(&op, b);
        for (int64_t n = 0; n < s->nf; ++n) x[s->fluid[n]] = s->C[(int64_t)sp * nv + s->fluid[n]];
        const int it = np_bicgstab(&op, b, x, tol, max_iter, NULL);
        if (it < 0) rc = it == -2 ? ORACLE_E_NOT_CONVERGED : ORACLE_E_DIVERGED;
        else tot += it;
        if (rc == ORACLE_OK)
            for (int64_t n = 0; n < s->nf; ++n) s->C[(int64_t)sp * nv + s->fluid[n]] = x[s->fluid[n]];
    }
    if (iters) *iters = tot;
    free(W), free(b), free(x);
    return rc;
}

/* Per species: rates of adsorption, inflow and outflow of the current state
 * (out[3 sp + k], per unit time). */
void oracle_np_rates(const oracle_solver *s, double out[6])
{
    for (int sp = 0; sp < 2; ++sp) {
        double a = 0, in = 0, o = 0;
        for (int64_t n = 0; n < s->nf; ++n) {
            double fa, fi, fo;
            cell_outflow(s, s->fluid[n], sp, s->C, &fa, &fi, &fo, NULL);
            a += fa;
            in += fi;
            o += fo;
        }
        out[3 * sp] = a;
        out[3 * sp + 1] = in;
        out[3 * sp + 2] = o;
    }
}

int oracle_np_implicit(oracle_solver *s, double dt, int64_t nsteps, double tol, int max_iter, int *iters)
{
    if (!(dt > 0) || nsteps < 0) return ORACLE_E_INVALID;
    if (!s->u_valid) oracle_freeze_velocity(s);
    const int64_t nv = s->nvox;
    double *W = calloc((size_t)(2 * nv), sizeof(double)), *b = calloc((size_t)nv, sizeof(double));
    double *x = calloc((size_t)nv, sizeof(double)), *rhs = calloc((size_t)nv, sizeof(double));
    int rc = ORACLE_OK, tot = 0;
    for (int64_t k = 0; k < nsteps && rc == ORACLE_OK; ++k) {
        for (int sp = 0; sp < 2 && rc == ORACLE_OK; ++sp) {
            np_op op = {s, sp, 1.0 / dt, W};
            np_rhs(&op, b);
            for (int64_t n = 0; n < s->nf; ++n) {
                const int64_t c = s->fluid[n];
                x[c] = s->C[(int64_t)sp * nv + c];
                rhs[c] = x[c] / dt + b[c];
            }
            const int it = np_bicgstab(&op, rhs, x, tol, max_iter, NULL);
            if (it < 0) rc = it == -2 ? ORACLE_E_NOT_CONVERGED : ORACLE_E_DIVERGED;
            else tot += it;
            if (rc == ORACLE_OK)
                for (int64_t n = 0; n < s->nf; ++n) s->Cn[(int64_t)sp * nv + s->fluid[n]] = x[s->fluid[n]];
        }
        if (rc != ORACLE_OK) break;
        double *t = s->C;
        s->C = s->Cn;
        s->Cn = t;
        /* the fluxes of the new state over dt enter the accumulators */
        double rates[6];
        oracle_np_rates(s, rates);
        for (int sp = 0; sp < 2; ++sp)
            for (int q = 0; q < 3; ++q) s->acc[sp][q] += dt * rates[3 * sp + q];
        s->np_steps++;
    }
    if (iters) *iters = tot;
    free(W), free(b), free(x), free(rhs);
    return rc;
}
