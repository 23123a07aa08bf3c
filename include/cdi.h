/*
 * cdi.h -- C ABI of the MI355X (gfx950) pore-scale capacitive-deionisation
 * solver: lattice Boltzmann Stokes flow coupled to an explicit finite-volume
 * Nernst-Planck update for Na+ and Cl- with surface adsorption.
 *
 * Model (Liu, Waugh, Komini Babu, Spendelow, Kang, 2021):
 *   - flow: Stokes equations, Eq. (1)-(2), solved by the lattice Boltzmann
 *     equation with BGK collision, Eq. (7)-(8); D2Q9 or D3Q19; moments
 *     rho = sum f, u = sum e f / rho; viscosity nu = (tau - 1/2)/3; no-flow
 *     by bounce-back at solid faces (Sec. 2);
 *   - ions: Nernst-Planck, Eq. (3), advection + diffusion + migration in a
 *     prescribed potential or the solution of Poisson's equation with its
 *     charge density, Eq. (4)-(5) (thermal voltages, psi~ = e psi / k_B T);
 *     explicit steps, or the implicit scheme of Sec. 2 (backward Euler and
 *     the steady state);
 *   - adsorption: linear law D dC/dn = K_a C at electrode faces, Eq. (6);
 *   - geometry: one lattice node per image voxel (Sec. 2, MAC grid).
 *
 * Conventions for every entry point:
 *   - x is the flow axis; voxel index v = x + nx*(y + ny*z), x fastest.
 *   - "device" pointers are HIP device allocations owned by the caller; the
 *     library never allocates, frees or resizes them. "host" pointers are
 *     ordinary host memory, read or written synchronously.
 *   - stream is a hipStream_t passed as void* (NULL = default stream). All
 *     device work of a solver is ordered on its stream.
 *   - Every call returns an int status: CDI_OK (0), a positive warning, or a
 *     negative CDI_E_* code; cdi_last_error() then describes the failure
 *     (thread-local string, valid until the next call on that thread).
 *     Nothing is thrown or aborted across the ABI.
 *   - A solver handle is not thread-safe: drive each one from one thread.
 */
#ifndef CDI_H
#define CDI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define CDI_OK 0
#define CDI_STAGNATED 1          /* flow stopped: residual stopped decreasing (FP32/FP16) */
#define CDI_E_INVALID (-1)       /* bad argument or configuration */
#define CDI_E_GEOMETRY (-2)      /* generator could not reach the porosity */
#define CDI_E_UNSTABLE (-3)      /* tau <= 1/2, or NP positivity bound violated */
#define CDI_E_NOT_CONVERGED (-4) /* max_steps reached; state remains valid */
#define CDI_E_DIVERGED (-5)      /* NaN/Inf residual */
#define CDI_E_DEVICE (-6)        /* HIP runtime error */
#define CDI_E_BUFFER (-7)        /* workspace too small or misaligned */

/* ---------------------------------------------------------------- enums */
enum { CDI_DISKS = 0, CDI_SPHERES = 1, CDI_USER_LABELS = 2, CDI_FIBRES = 3 };
enum { CDI_INLET_OUTLET = 0, CDI_BODY_FORCE = 1 };
enum { CDI_EQ_QUADRATIC = 0, CDI_EQ_LINEAR = 1 };
enum { CDI_NPX_INLET_OUTLET = 0, CDI_NPX_PERIODIC = 1, CDI_NPX_CLOSED = 2, CDI_NPX_DIRICHLET = 3 };
enum { CDI_FP32 = 0, CDI_FP16_DEV = 1, CDI_MOMENTS = 2, CDI_FP16 = 3 };
enum { CDI_STREAM_AA = 0, CDI_STREAM_PULL = 1 };

/*
 * Electrode geometry (Sec. 2: every grid block is one image voxel; Sec. 4-5:
 * porous carbon electrodes). Voxel labels: 0 pore (fluid), 1 adsorbing
 * electrode solid, 2 inert solid (channel wall).
 *   dim          2 (D2Q9, nz ignored = 1) or 3 (D3Q19)
 *   seed         SplitMix64 seed of the primitive generator
 *   kind         CDI_DISKS (2D, non-overlapping, random sequential addition),
 *                CDI_SPHERES (3D, overlapping, Boolean model, periodic y/z),
 *                CDI_USER_LABELS (labels copied from user_labels),
 *                CDI_FIBRES (3D straight overlapping fibres, Sec. 5: each a
 *                random core line through a random point, extended to the
 *                domain faces, every voxel within the radius solid; added
 *                until the Boolean-model porosity reaches the target; no
 *                wrap; edges <= 1024, r_max <= 64)
 *   porosity     target pore fraction over all voxels
 *   r_min,r_max  primitive radius range (lattice units; fibres: half the
 *                fibre diameter)
 *   min_gap      disks only: minimum surface gap (lattice units)
 *   walls_y      2D only: rows 0 and ny-1 are inert walls (else y periodic)
 *   buffer_x     always-fluid planes at each x end (>= 2 with inlet/outlet)
 *   user_labels  host, nx*ny*nz bytes, used for CDI_USER_LABELS only
 */
typedef struct {
    int32_t dim, nx, ny, nz;
    uint64_t seed;
    int32_t kind;
    double porosity, r_min, r_max, min_gap;
    int32_t walls_y;
    int32_t buffer_x;
    const uint8_t *user_labels;
} cdi_geometry;

/*
 * Physical and numerical parameters, lattice units (dx = dt = 1).
 *   tau          BGK relaxation time, Eq. (8); must exceed 1/2
 *   drive        CDI_INLET_OUTLET: plug velocity u_in at x = 0, density
 *                rho_out at x = nx-1 (non-equilibrium extrapolation);
 *                CDI_BODY_FORCE: periodic in x, driven by body_force
 *                (Guo forcing), the paper's pressure-gradient-as-body-force
 *   equilibrium  quadratic (default) or linear-in-u (Stokes limit)
 *   D[2], z[2]   diffusivity and valence of Na+ (index 0) and Cl- (index 1)
 *   c0           inlet and initial concentration ("initially saturated")
 *   c_out        outlet ghost concentration (CDI_NPX_DIRICHLET only)
 *   Ka           adsorption constant of Eq. (6); <= 0 selects
 *                Ka = (4.28e-3 / 1.03e-2) * u_in / porosity, the paper's
 *                Da/Pe ratio of its base case times the mean pore velocity
 *   dpsi_vt      potential drop inlet minus outlet in thermal voltages; the
 *                potential is the ramp dpsi_vt * (1 - (x + 1/2)/nx) until a
 *                field is given or solved (cdi_solve_potential)
 *   psi_field    device, N_f floats in fluid-node order, or NULL: a
 *                prescribed potential (thermal voltages) replacing the ramp,
 *                copied at initialisation. With a field, the x-end faces
 *                carry no migration (the ghost cell shares the cell's value)
 *   np_x_bc      treatment of the two x-end faces for Nernst-Planck
 *   np_substeps  Nernst-Planck sub-steps per step (dt = 1/np_substeps);
 *                fused steps need 1
 *   precision    CDI_FP32: populations stored in FP32 relative to the rest
 *                equilibrium of a reference density per x plane,
 *                f - w_i (1 + R[x]), with R[x] the plane mean of rho - 1,
 *                renewed at every residual check of cdi_flow_step_to_steady
 *                (zero until then): the stored values carry only the local
 *                fluctuations, which FP32 rounds finely;
 *                CDI_FP16: the same values stored in FP16 (times 2^12), all
 *                arithmetic FP32: half the population bytes, at an accuracy
 *                set by FP16's 11-bit significand;
 *                CDI_FP16_DEV: post-collision populations stored as FP16
 *                deviations from the local equilibrium, with the
 *                equilibrium's moments kept in FP32; all arithmetic FP32;
 *                CDI_MOMENTS: only the FP32 moments (rho - 1, u) are stored.
 *                Requires tau = 1 and no body force (else CDI_E_INVALID):
 *                then the BGK post-collision populations equal the local
 *                equilibrium (Eq. 8 with f* = f_eq), so the FP16 deviations
 *                are identically zero and this is CDI_FP16_DEV without them,
 *                bit for bit
 *   streaming    how populations move between steps (FP32 and FP16 storage;
 *                the results are identical):
 *                CDI_STREAM_AA: one array updated in place, alternating a
 *                step that reads and writes each node's own slots with one
 *                that reads and writes its neighbours' slots;
 *                CDI_STREAM_PULL: two arrays; every step gathers from the
 *                neighbours' slots of one and writes the node's own slots of
 *                the other (twice the population memory, no scattered stores)
 *   no_adsorption 1: K_a = 0 whatever Ka says (a blocking electrode, as the
 *                charged wall of the electromigration check, Sec. 3); 0: Ka
 */
typedef struct {
    double tau;
    int32_t drive;
    int32_t equilibrium;
    double u_in, rho_out;
    double body_force[3];
    double D[2];
    int32_t z[2];
    double c0, c_out, Ka, dpsi_vt;
    const float *psi_field;
    int32_t np_x_bc;
    int32_t np_substeps;
    int32_t precision;
    int32_t streaming;
    int32_t no_adsorption;
} cdi_params;

/* Sizes reported by cdi_plan. */
typedef struct {
    int64_t n_vox;          /* nx*ny*nz */
    int64_t n_prims;        /* primitives drawn by the generator */
    int64_t n_fluid_est;    /* target-porosity estimate of N_f (exact for disks) */
    uint64_t vox_bytes;     /* device workspace of cdi_build_geometry */
    uint64_t node_bytes_per_fluid; /* device workspace per fluid node (approximate) */
} cdi_plan_info;

typedef struct cdi_solver cdi_solver;

/* Solver facts after initialisation. */
typedef struct {
    int64_t n_vox, n_fluid;
    int32_t dim, q, nx, ny, nz;
    int32_t precision;
    int64_t flow_steps, np_steps;  /* steps taken so far */
    double ka, keff[2];            /* resolved Ka and k_eff per species */
    double porosity;               /* achieved N_f / N_vox */
} cdi_solver_info;

/* ------------------------------------------------------------ set-up */

/* Host only, no device work. Draws the seeded primitives (cheap) and reports
 * the voxel-level workspace size. INVALID on bad geometry, GEOMETRY when the
 * disk generator jams. */
int cdi_plan(const cdi_geometry *geom, const cdi_params *params, cdi_plan_info *out);

/* Host only, no device work: admission check of an inlet/outlet flow. The
 * lattice Boltzmann method is weakly compressible: the pressure drop that
 * drives the flow through the electrode is carried by density differences,
 * which must stay well below the rest density. Estimates the steady density
 * drop by Darcy's law over the electrode's length (nx - 2 buffer_x) with
 * the Kozeny-Carman permeability phi^3 / (5 s^2), s the fluid-solid surface
 * per volume (from the primitives' statistics, or counted on user labels),
 * drho = 3 nu u_in L / k; zero for the body-force drive. *drho_estimate
 * (nullable) receives it. Returns UNSTABLE when it exceeds max_drho (<= 0:
 * 0.5), else OK. */
int cdi_flow_check(const cdi_geometry *geom, const cdi_params *params, double max_drho, double *drho_estimate);

/* Voxelise the primitives and number the fluid voxels on the device (labels,
 * fluid index map, compacted fluid list), into vox_ws (device, >= vox_bytes,
 * 256-byte aligned). Synchronises once to return *n_fluid. Bit-identical to
 * a sequential lexicographic numbering. */
int cdi_build_geometry(const cdi_geometry *geom, void *vox_ws, uint64_t vox_ws_bytes,
                       void *stream, int64_t *n_fluid);

/* Device workspace needed by cdi_flow_init for n_fluid nodes. */
int cdi_node_bytes(const cdi_geometry *geom, const cdi_params *params, int64_t n_fluid,
                   uint64_t *bytes);

/* Initialise a solver on a built geometry: fluid at rest (rho = 1, u = 0),
 * C = c0, accumulators zero. vox_ws must hold the output of
 * cdi_build_geometry; node_ws (device, >= cdi_node_bytes, 256-byte aligned)
 * holds all per-node state. Both must outlive the solver. Asynchronous on
 * stream. UNSTABLE if tau <= 1/2. *out is library-owned: cdi_destroy it. */
int cdi_flow_init(const cdi_geometry *geom, const cdi_params *params, void *vox_ws,
                  uint64_t vox_ws_bytes, void *node_ws, uint64_t node_ws_bytes,
                  int64_t n_fluid, void *stream, cdi_solver **out);

int cdi_destroy(cdi_solver *s);
int cdi_get_info(const cdi_solver *s, cdi_solver_info *out);

/* ------------------------------------------------------------ time stepping */

/* n lattice Boltzmann steps (collide, stream, bounce-back, inlet/outlet).
 * Asynchronous. */
int cdi_flow_steps(cdi_solver *s, int64_t n);

/* Step the flow until r = |u^t - u^{t-1}|_2 / |u^t|_2 <= tol, where u^t is the
 * velocity of the state step t starts from (0-based within the call), and r
 * is evaluated (FP64) at t = check_every, 2*check_every, ... The call stops
 * after the step that evaluated r <= tol. Synchronises once per check.
 * Returns OK, STAGNATED (r failed to decrease over 10 consecutive checks),
 * NOT_CONVERGED (max_steps taken; state valid) or DIVERGED (r not finite).
 * steps_out / residual_out (host, nullable) receive the steps taken and the
 * last residual. */
int cdi_flow_step_to_steady(cdi_solver *s, double tol, int64_t max_steps, int32_t check_every,
                            int64_t *steps_out, double *residual_out);

/* nsteps Nernst-Planck steps, asynchronous. fused_flow = 0: the advecting
 * velocity is frozen at the mass flux j = rho u of the current populations
 * (or the field set by cdi_set_np_velocity). fused_flow = 1: every step also
 * advances the flow, and the ions see the mass flux of the previous step.
 * Checks the positivity bound dt * sum(outflow coefficients) <= 1 before the
 * first step (synchronising) and returns UNSTABLE without stepping if it
 * fails; with fused_flow, whose flow keeps changing, again every 256 steps
 * (UNSTABLE then after the steps already taken, state valid). */
int cdi_np_step(cdi_solver *s, int64_t nsteps, int32_t fused_flow);

/* Total adsorbed amount per species [Na, Cl] (lattice units: concentration x
 * voxel volume), FP64, since initialisation. Synchronises. */
int cdi_adsorbed_total(cdi_solver *s, double out[2]);

/* FP64 balance per species: out[4*s + k], k = 0 solute sum_C, 1 adsorbed A,
 * 2 inflow In, 3 outflow Out. M + A + Out - In is conserved. Synchronises. */
int cdi_mass_balance(cdi_solver *s, double out[8]);

/* ------------------------------------------------------------ state access
 * All copies are synchronous, into caller-owned host memory. Fields are in
 * fluid-node order, component-major (component c of node n at c*N_f + n). */
int cdi_copy_labels(cdi_solver *s, uint8_t *labels);                 /* N_vox */
int cdi_copy_fluid_index(cdi_solver *s, int32_t *map, int32_t *fluid); /* N_vox, N_f (nullable) */
int cdi_copy_velocity(cdi_solver *s, float *u);      /* dim x N_f, u of the current populations */
int cdi_copy_density(cdi_solver *s, float *rho);     /* N_f */
int cdi_copy_np_velocity(cdi_solver *s, float *j);   /* dim x N_f, advecting field in use */
int cdi_set_np_velocity(cdi_solver *s, const float *j); /* dim x N_f, prescribe (frozen) */
int cdi_copy_concentration(cdi_solver *s, float *c); /* 2 x N_f */
int cdi_set_concentration(cdi_solver *s, const float *c); /* 2 x N_f */

/* ------------------------------------------------------------ launch tuning
 * How the step kernel is scheduled on the GPU. Results are bitwise identical
 * for every tuning (each node's update and each tile's accumulator sum do
 * not depend on the schedule); only the speed changes. */
typedef struct {
    int32_t blocks_per_cu; /* cap on resident step workgroups per compute unit (0 = none) */
    int32_t band_rows;     /* 3D: rows per band of the tile schedule (0 = plain order) */
    int32_t columns;       /* 3D, 1: tiles of each group of 8 brick layers dealt round-robin over the
                              8 XCDs, so the 8 layers at one (x, y) are processed together (the
                              layers above and below a tile meet in the memory-side cache);
                              2: tiles in the Morton (Z-order) order of their bricks, each XCD
                              walking a contiguous run of the curve (a brick's neighbours along
                              every axis are mostly a few bricks away in that XCD's sweep);
                              either takes precedence over band_rows. 0: off */
    int32_t nbr_list;      /* 1 (the default): the ion-only steps and the fused steps with FP16 or moment
                              storage read each node's neighbours from a list built at init (4 (Q-1)
                              bytes per node of extra reads) instead of looking them up through the
                              voxel map after the node's coordinates (flow-only and fused FP32 steps
                              always look them up: measured no faster with the list); 0: map lookups
                              everywhere */
    int32_t stage_odd;     /* odd AA steps with FP32 or FP16 populations: each workgroup stages its
                              tile's population slots in LDS
                              (the slots whose reader is in the tile are then read and written there,
                              and the tile's own slots move as coalesced loads and stores). 0 (the
                              default): staged when the instance has at least CDI_STAGE_MIN_TILES
                              tiles of 256 fluid nodes (measured: FP32 steps 2-8 % faster from there
                              on; a smaller lattice's working set stays largely in the memory-side
                              cache, and there staging made the steps 5-13 % slower); 1: always;
                              2: never. Batched launches never stage */
} cdi_tuning;

#define CDI_STAGE_MIN_TILES 16384

int cdi_set_tuning(cdi_solver *s, const cdi_tuning *t);
int cdi_get_tuning(const cdi_solver *s, cdi_tuning *t);

/* Autotuner: snapshots the state to host memory, times each candidate tuning
 * over `steps` steps (fused_flow as in cdi_np_step) with HIP events on the
 * solver's stream, restores the state and keeps the fastest. chosen and
 * ms_per_step (host, nullable) receive the winner and its time per step.
 * Synchronises. */
int cdi_autotune(cdi_solver *s, int32_t steps, int32_t fused_flow, cdi_tuning *chosen,
                 double *ms_per_step);

/* ------------------------------------------------------------ batches
 * Many independent electrodes (uneven sizes, own parameters) advanced by one
 * launch per step class. Members must share the device, the stream, the
 * dimension and the storage precision. Each member's results are bitwise
 * identical to advancing that member alone with the same sequence of calls
 * (tile results do not depend on which workgroup computes them). */
typedef struct cdi_batch cdi_batch;

enum { CDI_MODE_IDLE = 0, CDI_MODE_FLOW = 1, CDI_MODE_IONS = 2, CDI_MODE_FUSED = 3 };

/* Device workspace a batch of these members needs. */
int cdi_batch_bytes(cdi_solver *const *members, int32_t n, uint64_t *bytes);

/* Group n solvers. ws: device, >= cdi_batch_bytes, 256-byte aligned; it and the
 * members must outlive the batch. stream: the stream batched work runs on (a
 * non-default stream enables HIP graph replay); the batch orders itself after
 * the members' streams on entry and the members' streams after it on exit.
 * The batch only borrows the members: they stay usable on their own between
 * batch calls. */
int cdi_batch_create(cdi_solver *const *members, int32_t n, void *ws, uint64_t ws_bytes, void *stream,
                     cdi_batch **out);
int cdi_batch_destroy(cdi_batch *b);

/* Batches whose membership changes while they run (continuous batching):
 * an empty batch with room for up to max_members members holding up to
 * max_fluid fluid nodes together; cdi_batch_capacity_bytes sizes its device
 * workspace ws (256-byte aligned, kept by the caller until destroy). Members
 * must still share the device, the dimension and the storage precision (set
 * by the first admitted). */
int cdi_batch_capacity_bytes(int32_t max_members, int64_t max_fluid, uint64_t *bytes);
int cdi_batch_create_empty(int32_t max_members, int64_t max_fluid, void *ws, uint64_t ws_bytes, void *stream,
                           cdi_batch **out);

/* Admit a solver as the last member (index cdi_batch_members - 1), with no new
 * workspace: BUFFER when the batch is full (members or fluid nodes beyond its
 * capacity), INVALID for a duplicate or a mismatched solver. Retire a member:
 * waits for the batch's queued work, then removes it (later members move up
 * one index; the solver itself is untouched and usable alone). The modes of
 * the next cdi_batch_advance follow the new member order. A membership
 * change keeps the captured step graph when the launch shape is unchanged
 * (it re-captures otherwise). Results stay bitwise those of each member
 * stepped alone. */
int cdi_batch_admit(cdi_batch *b, cdi_solver *member);
int cdi_batch_retire(cdi_batch *b, cdi_solver *member);
int cdi_batch_members(const cdi_batch *b, int32_t *n);

/* Advance every member by nsteps in its mode (host array modes[n]):
 *   FLOW  = cdi_flow_steps, IONS = cdi_np_step(fused 0), FUSED = cdi_np_step(fused 1),
 *   IDLE  = untouched.
 * Like cdi_np_step, IONS/FUSED members are checked for positivity first
 * (UNSTABLE names the first failing member and nothing is stepped) and, when
 * a member is FUSED, again at least every 256 steps (UNSTABLE then after the
 * steps already taken, state valid). Runs of
 * identical steps are replayed from a captured HIP graph. FLOW members also get
 * the residual of their last step (see cdi_batch_residuals) when nsteps >= 2.
 * Asynchronous except for the positivity check. */
int cdi_batch_advance(cdi_batch *b, int64_t nsteps, const int32_t *modes);

/* r[k] = |u^t - u^{t-1}| / |u^t| over the last two steps of the last advance
 * for FLOW members, NaN for the others. Synchronises. */
int cdi_batch_residuals(cdi_batch *b, double *r);

/* Grid size of the batched launches (0, the default: one workgroup per tile
 * of each step class; fewer make the workgroups persistent, each taking
 * every G-th tile of its XCD's share) and occupancy cap. */
int cdi_batch_set_launch(cdi_batch *b, int32_t workgroups, int32_t blocks_per_cu);
int cdi_batch_get_launch(const cdi_batch *b, int32_t *workgroups, int32_t *blocks_per_cu);

/* Autotuner for the batched launches' grid size: snapshots all members, times candidate
 * grid sizes over `steps` steps of the given modes, restores every member and
 * keeps the fastest. Synchronises. */
int cdi_batch_autotune(cdi_batch *b, int32_t steps, const int32_t *modes, int32_t *workgroups,
                       double *ms_per_step);

/* ------------------------------------------------------------ electric potential
 * Poisson's equation for the potential, Eq. (4), with the charge density of
 * Eq. (5), and a constant potential on the electrode surface as the Dirichlet
 * condition at the liquid-solid interface (Sec. 2). In thermal voltages
 * psi~ = e psi / k_B T and lattice units, with lambda_D the Debye length of a
 * symmetric electrolyte at c0 (lambda_D^2 = eps_r eps_0 k_B T / (2 e F c0),
 * the length in Eq. (10)), the equation reads
 *   lap psi~ = -(kappa2 / (2 c0)) sum_i z_i C_i,   kappa2 = (dx / lambda_D)^2.
 * Finite volumes on the fluid voxels: a face between two fluid cells carries
 * psi_N - psi_P, an electrode face 2 (psi_electrode - psi_P) (the value holds
 * on the face, half a cell from the centre), an inert face nothing, and each
 * x-end face is Dirichlet (value psi_x), field-free, or periodic (both ends).
 * The symmetric positive definite system is solved on the GPU by mixed-
 * precision iterative refinement: each round forms the FP64 residual of the
 * FP64 iterate and solves for the correction by Jacobi-preconditioned
 * conjugate gradients on FP32 vectors (sums in FP64), until the FP64
 * residual meets tol; a round that gains less than 4x hands over to the same
 * CG on FP64 vectors (fp64 = 1: that CG alone). The result (stored as FP32) becomes the potential of
 * every later ion step. */
enum { CDI_PSIX_DIRICHLET = 0, CDI_PSIX_NEUMANN = 1, CDI_PSIX_PERIODIC = 2 };

typedef struct {
    double psi_electrode;  /* psi~ on every electrode (label 1) face */
    int32_t x_bc[2];       /* CDI_PSIX_* of the faces x = 0 and x = nx */
    double psi_x[2];       /* their Dirichlet values */
    double kappa2;         /* (dx / lambda_D)^2 >= 0; 0 = Laplace (charge neglected) */
    double tol;            /* stop at |b - A psi|_2 <= tol |b|_2 (FP64 residual) */
    int32_t max_iter;      /* iteration cap */
    int32_t check_every;   /* iterations between convergence read-backs (0 = 32) */
    int32_t warm_start;    /* 1: start from the field in use (if any), 0: from zero */
    int32_t fp64;          /* 1: CG on FP64 vectors throughout (no FP32 rounds);
                              0: mixed-precision refinement */
} cdi_potential;

typedef struct {
    int32_t iterations;    /* CG iterations taken (over all refinement rounds) */
    double residual;       /* final |b - A psi|_2 / |b|_2 */
    int32_t fp32_rounds;   /* refinement rounds with an FP32 correction solve */
    int32_t fp64_iterations; /* of the iterations, those on FP64 vectors */
} cdi_potential_result;

/* Device workspace of the solve (5 FP64 and 5 FP32 vectors and a byte per node, plus
 * per-workgroup sums); needed only during the call. The solve reads face
 * neighbours from the solver's neighbour list when the potential's x ends
 * are periodic exactly when the lattice's are, else through the voxel map;
 * the result is the same. Iterates are bitwise repeatable on one device (the
 * number of persistent workgroups, which fixes the summation order, follows
 * the device's compute-unit count). */
int cdi_potential_bytes(const cdi_solver *s, uint64_t *bytes);

/* Solve for the potential of the current concentrations. ws: device, >=
 * cdi_potential_bytes, 256-byte aligned. Synchronises once per check_every
 * iterations. The iterate is the same for any check_every (the stop is
 * decided on the device). Returns OK; NOT_CONVERGED after max_iter (the last
 * iterate is installed); INVALID without any Dirichlet face (the potential is
 * then fixed only up to a constant) or for bad settings; DIVERGED on a
 * non-finite residual or a breakdown (nothing installed). out (host,
 * nullable) receives iterations and residual. */
int cdi_solve_potential(cdi_solver *s, const cdi_potential *pot, void *ws, uint64_t ws_bytes,
                        cdi_potential_result *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture aside, tight serving loops, harnesses that forbid hipMalloc):
 * cdi_solve_potential with the library's own scratch instead of a caller
 * workspace: a 64 MiB device array per GPU, held until the process ends, so
 * lattices whose cdi_potential_bytes exceeds 64 MiB (about a million fluid
 * nodes) are refused with CDI_E_BUFFER. The call allocates nothing. Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (two
 * host threads, or solvers on different streams) race; serialise them.
 * Same results as cdi_solve_potential, statuses as there. */
int cdi_solve_potential_noalloc(cdi_solver *s, const cdi_potential *pot, cdi_potential_result *out);

/* Coupled Poisson-Nernst-Planck: nsteps ion steps (fused_flow as in
 * cdi_np_step), with the potential solved afresh from the concentrations
 * before every `every`-th step (explicit, lagged coupling; the positivity
 * check of cdi_np_step runs after every solve). The coupling adds the
 * dielectric relaxation rate D kappa2 to each species' update, which the
 * positivity check does not bound: keep dt D kappa2 well below 1. */
int cdi_np_step_coupled(cdi_solver *s, int64_t nsteps, int32_t fused_flow, const cdi_potential *pot,
                        int32_t every, void *ws, uint64_t ws_bytes);

/* The potential in use (thermal voltages), N_f floats in fluid-node order:
 * the solved or given field, else the ramp. Synchronous. */
int cdi_copy_potential(cdi_solver *s, float *psi);

/* ------------------------------------------------------------ implicit ion transport
 * The paper discretises Eq. (3) with an implicit finite-volume method (Sec. 2).
 * For the frozen advecting flux and the current potential each species'
 * outflow is affine in its concentrations, out(C) = A C - b (the explicit
 * step's face fluxes, adsorption and ghost terms; coefficients evaluated in
 * FP32 as the explicit step does, applied in FP64). A backward-Euler step of
 * length dt solves (I/dt + A) C' = C/dt + b; the steady state solves A C = b;
 * both by BiCGSTAB with the diagonal as preconditioner, both species
 * together, to the relative residual tol (|rhs - M C'| <= tol |rhs|). The
 * stop is decided on the device; the iterate is bitwise repeatable on one
 * device. The scheme is unconditionally positive and stable (no positivity
 * check is needed or made). */

/* Device workspace of the ion solves (7 FP64 vector pairs and an FP32 pair
 * per node, plus per-workgroup sums); needed only during a call. */
int cdi_np_solve_bytes(const cdi_solver *s, uint64_t *bytes);

/* The steady concentrations on the frozen flow, from the current ones
 * (installed as the current state; the accumulators and step count are not
 * changed). ws: device, >= cdi_np_solve_bytes, 256-byte aligned.
 * Synchronises every 32 iterations. OK, NOT_CONVERGED after max_iter (the
 * last iterate is installed) or DIVERGED (nothing installed). iterations
 * (host, nullable): the larger of the two species' counts. */
int cdi_np_steady(cdi_solver *s, double tol, int32_t max_iter, void *ws, uint64_t ws_bytes, int32_t *iterations);

/* nsteps backward-Euler steps of length dt > 0; after each, the new state's
 * adsorption, inflow and outflow rates times dt enter the accumulators (the
 * balance M + A + Out - In is kept to the solver tolerance). iterations: the
 * total over the steps. Statuses as cdi_np_steady (a failed step ends the call). */
int cdi_np_implicit(cdi_solver *s, double dt, int64_t nsteps, double tol, int32_t max_iter, void *ws,
                    uint64_t ws_bytes, int32_t *iterations);

/* Rates of the current concentrations per species, FP64: out[3 sp + 0]
 * adsorption, + 1 inflow, + 2 outflow (amount per unit time). Synchronises. */
int cdi_np_rates(cdi_solver *s, double out[6]);

/* ------------------------------------------------------------ diagnostics (Sec. 4)
 * The dimensionless numbers and averages the paper reports. */
typedef struct {
    int64_t n_surface;       /* fluid-electrode voxel faces (x wraps only with the body-force drive) */
    int64_t n_inlet;         /* fluid voxels of the x = 0 plane */
    double specific_surface; /* s = n_surface / N_vox (electrode area per volume, lattice units) */
    double l_c;              /* characteristic length pi / s */
    double U;                /* U = sum_i u_i / (N phi): streamwise velocity of the current
                                populations summed over the fluid, over N_f */
    double Pe[2], Da[2];     /* U l_c / D_i and K_a l_c / D_i per species */
} cdi_diag;

/* Surface, velocity and the dimensionless numbers (FP64 sums in a fixed
 * order). Synchronises. */
int cdi_diagnostics(cdi_solver *s, cdi_diag *out);

/* Vertically averaged concentrations along the flow axis (Figs. 6 and 9):
 * out (host, 3 nx doubles): out[x], out[nx + x] = mean C of Na, Cl over the
 * fluid voxels of plane x, out[2 nx + x] = their number. Synchronises. */
int cdi_profile_x(cdi_solver *s, double *out);

/* Salt removal over a window of nsteps ion steps between two cdi_mass_balance
 * read-backs bal0, bal1 (host): P_rm = (C_in - C_out) / C_in per species
 * (out[0], out[1]) with C_in = c0 and C_out the flux-weighted outlet
 * concentration, (Out1 - Out0) / (u_in n_inlet nsteps); out[2] = their mean
 * (salt); out[3] = U A P_rm nsteps / (V_t phi), the amount removed per pore
 * volume in the window (Sec. 4.1), A = ny nz, V_t phi = N_f, U and n_inlet
 * from cdi_diagnostics. Host arithmetic only. */
int cdi_salt_removal(const cdi_solver *s, const double bal0[8], const double bal1[8], int64_t nsteps,
                     int64_t n_inlet, double U, double out[4]);

/* Checkpoint: the complete device state (populations, moments, fields,
 * potential, accumulators, counters, AA parity) to and from host memory. */
int cdi_snapshot_bytes(cdi_solver *s, uint64_t *bytes);
int cdi_snapshot(cdi_solver *s, void *host, uint64_t bytes);
int cdi_restore(cdi_solver *s, const void *host, uint64_t bytes);

/* ------------------------------------------------------------ bandwidth probe
 * Streaming kernels of exactly known traffic with 128-bit accesses, one or
 * two 16-byte words per thread over a grid sized to the data. They give the
 * HBM bandwidth a kernel attains on the device, the yardstick beside the
 * 8 TB/s peak for the step kernels' bytes per update, and a launch of known
 * size to calibrate profiler byte counters. Not part of the model.
 *   CDI_PROBE_COPY  dst[0, bytes) = src[0, bytes): reads and writes bytes
 *   CDI_PROBE_READ  16-byte word k of dst = XOR of the 16-byte words of
 *                   src[8192 k, 8192 (k + 1)) (dst holds 16 ceil(bytes / 8192)
 *                   bytes): reads bytes, writes 1/512 of that
 *   CDI_PROBE_FILL  dst[0, bytes) = the 32-bit value repeated: writes bytes
 * dst and src are device pointers, 16-byte aligned; bytes a multiple of 16;
 * the ranges must not overlap. Asynchronous on stream. INVALID on a bad
 * argument, DEVICE on a launch error. */
enum { CDI_PROBE_COPY = 0, CDI_PROBE_READ = 1, CDI_PROBE_FILL = 2 };
int cdi_bandwidth_probe(int32_t mode, void *dst, const void *src, uint64_t bytes, uint32_t value, void *stream);

const char *cdi_last_error(void);

/* sizeof of the public struct called name ("cdi_geometry", "cdi_params",
 * "cdi_plan_info", "cdi_solver_info", "cdi_tuning", "cdi_potential",
 * "cdi_potential_result", "cdi_diag") as this library was compiled, so that a
 * binding can check its own layout before the first call. Host only (no
 * device call). Returns OK, or INVALID for an unknown name or a null
 * argument. */
int cdi_struct_size(const char *name, uint64_t *bytes);

#ifdef __cplusplus
}
#endif
#endif
