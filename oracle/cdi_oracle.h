/*
 * cdi_oracle.h -- plain FP64 CPU reference of the pore-scale CDI model.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The GPU library never
 * links, includes or calls it, and it shares no code with the GPU library
 * (the seeded primitive generator, which holds no model arithmetic, is the
 * only module both compile).
 *
 * What it computes (Liu, Waugh, Komini Babu, Spendelow, Kang, 2021):
 *   - voxel labels from primitives, and the compacted fluid-node numbering
 *     (Sec. 2: one grid block per image voxel on a MAC grid);
 *   - lattice Boltzmann Stokes flow, Eq. (7)-(8), D2Q9 / D3Q19 BGK with the
 *     moments of the LBM paragraph (rho = sum f, u = sum e f / rho,
 *     nu = (tau - 1/2)/3), bounce-back at solid faces (no-flow paragraph);
 *   - the Nernst-Planck equation, Eq. (3), for Na+ and Cl- with a prescribed
 *     potential, and the adsorption law of Eq. (6) as a flux at electrode faces;
 *   - the potential itself from Poisson's equation, Eq. (4), with the charge
 *     of Eq. (5) and Dirichlet values on the electrode surface.
 * Everything is plain loops over the dense voxel grid in double precision,
 * using a two-lattice push scheme. Readings of what the paper leaves open
 * (time scheme, face fluxes, boundary treatments) are stated where used.
 */
#ifndef CDI_ORACLE_H
#define CDI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_DRIVE_INLET_OUTLET = 0, ORACLE_DRIVE_BODY_FORCE = 1 };
enum { ORACLE_EQ_QUADRATIC = 0, ORACLE_EQ_LINEAR = 1 };
/* Nernst-Planck treatment of the two x-end faces. */
enum {
    ORACLE_NPX_INLET_OUTLET = 0, /* Dirichlet c0 ghost at inlet, zero-gradient outlet */
    ORACLE_NPX_PERIODIC = 1,
    ORACLE_NPX_CLOSED = 2,       /* zero flux */
    ORACLE_NPX_DIRICHLET = 3     /* ghost c0 at inlet, ghost c_out at outlet */
};

typedef struct {
    int dim, nx, ny, nz;     /* lattice; x is the flow axis; nz = 1 in 2D */
    int drive;               /* ORACLE_DRIVE_* */
    int equilibrium;         /* ORACLE_EQ_* */
    double tau;              /* BGK relaxation time (> 1/2) */
    double u_in;             /* inlet plug velocity (lattice units) */
    double rho_out;          /* outlet density */
    double force[3];         /* body-force density (drive = BODY_FORCE) */
    double D[2];             /* diffusivities of Na+, Cl- (lattice units) */
    int z[2];                /* valences */
    double c0;               /* inlet / initial concentration */
    double c_out;            /* outlet ghost concentration (NPX_DIRICHLET only) */
    double Ka;               /* adsorption constant; <= 0: derive 0.4155*u_in/phi */
    double dpsi;             /* potential drop (thermal voltages) inlet minus outlet */
    int np_x_bc;             /* ORACLE_NPX_* */
    int np_substeps;         /* sub-steps per NP step (>= 1) */
    int no_adsorption;       /* 1: K_a = 0 (a blocking electrode) */
} oracle_cfg;

/* status codes */
#define ORACLE_OK 0
#define ORACLE_E_INVALID (-1)
#define ORACLE_E_UNSTABLE (-3)
#define ORACLE_E_NOT_CONVERGED (-4)
#define ORACLE_E_DIVERGED (-5)

/* ---- geometry (Sec. 2, MAC grid of voxels) ---- */

/* Voxelise primitives (r, cx, cy, cz in 1/256 lattice units, 4 int64 each).
 * labels: nx*ny*nz bytes, x fastest: 0 fluid, 1 adsorbing electrode, 2 inert.
 * dim 2: kind is disks; rows 0, ny-1 are inert walls if walls_y, otherwise
 * y is periodic. dim 3: spheres, periodic in y and z. Primitives are clipped
 * in x to [buffer_x, nx - buffer_x). */
int oracle_voxelize(int dim, int nx, int ny, int nz, int walls_y, int buffer_x,
                    const int64_t *prims, int64_t nprims, uint8_t *labels);

/* Voxelise straight fibres (8 int64 each: r, ox, oy, oz, dx, dy, dz, unused;
 * lengths in 1/256 lattice units, d an integer direction): a voxel with
 * buffer_x <= x < nx - buffer_x is electrode (1) iff its centre lies within r
 * of some fibre's infinite core line; no wrap. */
int oracle_voxelize_fibres(int nx, int ny, int nz, int buffer_x, const int64_t *fibres, int64_t nfib,
                           uint8_t *labels);

/* Rank fluid voxels in lexicographic (x fastest) order. map[v] = rank, or -1
 * for electrode, -2 for inert voxels. fluid[rank] = v. Returns N_f. */
int64_t oracle_compact(const uint8_t *labels, int64_t nvox, int32_t *map, int32_t *fluid);

/* ---- solver ---- */
typedef struct oracle_solver oracle_solver;

/* psi_fluid: optional prescribed potential (thermal voltages) per fluid node
 * in compacted order; NULL selects the linear ramp dpsi*(1 - (x+1/2)/nx). */
oracle_solver *oracle_create(const oracle_cfg *cfg, const uint8_t *labels, const double *psi_fluid);
void oracle_destroy(oracle_solver *s);
int64_t oracle_num_fluid(const oracle_solver *s);
double oracle_ka(const oracle_solver *s);       /* resolved Ka */

/* n LBM steps (collide, stream with bounce-back, inlet/outlet). */
void oracle_flow_steps(oracle_solver *s, int64_t n);
/* Step until r = |u^n - u^{n-1}| / |u^n| <= tol, evaluated every check_every
 * steps; u^n is the velocity of the state a step starts from. */
int oracle_flow_to_steady(oracle_solver *s, double tol, int64_t max_steps, int check_every,
                          int64_t *steps_out, double *residual_out);

/* Velocity / density of the current populations (compacted order, dim x N_f). */
void oracle_get_velocity(const oracle_solver *s, double *u);
void oracle_get_density(const oracle_solver *s, double *rho);
/* Populations f_i of the current state, Q x N_f. */
void oracle_get_populations(const oracle_solver *s, double *f);

/* Set every fluid node to f^eq(rho, u) (rho, u per fluid node; NULL = 1 / 0). */
void oracle_init_equilibrium(oracle_solver *s, const double *rho, const double *u);
/* Freeze the NP advecting velocity at the mass flux j = rho u of the current
 * populations (rho_0 = 1). */
void oracle_freeze_velocity(oracle_solver *s);
/* Prescribe the NP velocity (dim x N_f, compacted order). */
void oracle_set_velocity(oracle_solver *s, const double *u);
void oracle_get_np_velocity(const oracle_solver *s, double *u);

/* n Nernst-Planck steps. fused = 1 also advances the LBM each step and feeds
 * NP with the mass flux of the previous step. Returns ORACLE_E_UNSTABLE if
 * the positivity bound fails at the start. */
int oracle_np_steps(oracle_solver *s, int64_t n, int fused);
/* max over fluid cells of dt * (sum of outflow coefficients of C_P). */
double oracle_np_stability(const oracle_solver *s);

void oracle_get_conc(const oracle_solver *s, double *c);     /* 2 x N_f */
void oracle_set_conc(oracle_solver *s, const double *c);     /* 2 x N_f */
/* out[s*4 + k]: k = 0 mass sum C, 1 adsorbed A, 2 inflow In, 3 outflow Out */
void oracle_balance(const oracle_solver *s, double *out);
void oracle_adsorbed_total(const oracle_solver *s, double out[2]);
int64_t oracle_flow_step_count(const oracle_solver *s);
int64_t oracle_np_step_count(const oracle_solver *s);

/* ---- electric potential, Eq. (4)-(5) ---- */
/* x-end faces of the potential problem. */
enum { ORACLE_PSIX_DIRICHLET = 0, ORACLE_PSIX_NEUMANN = 1, ORACLE_PSIX_PERIODIC = 2 };

typedef struct {
    double psi_electrode;  /* psi~ on every electrode face (Dirichlet, half a cell away) */
    int x_bc[2];           /* ORACLE_PSIX_* of the x = 0 and x = nx faces (periodic: both) */
    double psi_x[2];       /* Dirichlet values of those faces */
    double kappa2;         /* (h / lambda_D)^2; the charge term is kappa2 / (2 c0) sum z_i C_i */
    double tol;            /* stop at |b - A psi|_2 <= tol |b|_2 */
    int max_iter;
} oracle_potential;

/* Solve the discrete Poisson problem for the current concentrations (kappa2
 * = 0: Laplace) by Jacobi-preconditioned conjugate gradients from zero and
 * make the result the potential of the Nernst-Planck steps. iters / relres
 * (nullable) receive the iterations and the final relative residual.
 * ORACLE_E_INVALID without any Dirichlet face (singular problem). */
int oracle_solve_potential(oracle_solver *s, const oracle_potential *pc, int *iters, double *relres);
/* n ion steps (fused as in oracle_np_steps), the potential solved afresh
 * from the current concentrations before every `every`-th step. */
int oracle_np_steps_coupled(oracle_solver *s, int64_t n, int fused, const oracle_potential *pc, int every);
/* Potential in use per fluid node (compacted order): the ramp, the given
 * field or the solved one. */
void oracle_get_potential(const oracle_solver *s, double *psi);

/* ---- diagnostics of Sec. 4 ---- */
typedef struct {
    int64_t n_surface;       /* fluid-electrode voxel faces */
    int64_t n_inlet;         /* fluid voxels of the x = 0 plane */
    double specific_surface; /* s = n_surface / N (per lattice unit) */
    double l_c;              /* pi / s */
    double U;                /* sum of u_x over the fluid / N_f (u of the current populations) */
    double Pe[2], Da[2];     /* U l_c / D_i, K_a l_c / D_i */
} oracle_diag;

void oracle_diagnostics(const oracle_solver *s, oracle_diag *out);
/* Vertically averaged concentrations: out[x], out[nx + x] = mean C of Na, Cl
 * over the fluid voxels of plane x; out[2 nx + x] = their number. */
void oracle_profile_x(const oracle_solver *s, double *out);

/* Salt removal and removed amount over a window between two oracle_balance
 * read-backs nsteps ion steps apart (see cdi_oracle.c). */
void oracle_salt_removal(const oracle_solver *s, const double *bal0, const double *bal1, int64_t nsteps,
                         int64_t n_inlet, double U, double out[4]);

/* ---- implicit ion transport (the paper's time scheme, Sec. 2) ---- */
/* Steady state of the ion equations on the frozen flow and current
 * potential (A C = b, BiCGSTAB to relative residual tol), from the current
 * concentrations. The accumulators are left as they are. */
int oracle_np_steady(oracle_solver *s, double tol, int max_iter, int *iters);
/* nsteps backward-Euler steps of length dt: (I/dt + A) C' = C/dt + b; the
 * new state's adsorption, inflow and outflow rates times dt enter the
 * accumulators (the scheme conserves M + A + Out - In exactly). */
int oracle_np_implicit(oracle_solver *s, double dt, int64_t nsteps, double tol, int max_iter, int *iters);
/* Adsorption, inflow and outflow rates of the current state per species:
 * out[3 sp + 0..2]. */
void oracle_np_rates(const oracle_solver *s, double out[6]);

/* Threads the OpenMP loops use (1 if built without OpenMP). */
int oracle_threads(void);
/* Threads for the following OpenMP loops (n > 0; no effect without OpenMP).
   Results do not depend on it: every reduction is chunked in a fixed order. */
void oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
