// np_solve_internal.h -- argument block and launchers of the implicit ion
// transport (np_solve.hip): backward-Euler steps and the steady state of the
// Nernst-Planck equations, Eq. (3), on a frozen flow and potential.
#pragma once

#include "cdi_internal.h"

namespace cdi {

constexpr int kNpsMaxWorkgroups = 4096;
constexpr int kNpsWorkgroupsPerCU = 4;  // cap on resident solver workgroups per compute unit

// Solver state (doubles): per species s, active flag (1 while iterating),
// iterations done, |r|^2 of the last test, |rhs|^2, tol^2 |rhs|^2; then a
// global stop code.
enum {
    kNsActive = 0,  // + s
    kNsIters = 2,   // + s
    kNsRr = 4,      // + s
    kNsBb = 6,      // + s
    kNsThr = 8,     // + s
    kNsDone = 10,   // 0 running, 1 converged, 2 diverged / breakdown
    kNsSlots = 12
};

struct NpsArgs {
    Grid g;
    Phys p;
    const float *C;    // concentrations of the state the step starts from (2 planes of P)
    const float *j;    // frozen advecting mass flux (d planes of P)
    double idt;        // 1 / dt of a backward-Euler step, 0 for the steady state
    // FP64 vectors, 2 planes (species) of P each
    double *x, *r, *rh, *pv, *v, *sv, *t;
    float *dg;         // diagonal of (I/dt + A), 2 planes of P
    double *part;      // per-workgroup partial sums (nps_part_doubles)
    double *state;     // kNsSlots doubles
    double *acc;       // the solver's per-tile accumulators (rates pass)
};

uint64_t nps_part_doubles();
hipError_t nps_workgroups(int dim, int ntiles, int *G);
// x = C, r = rhat = C idt + b - A x, diagonal, |rhs|^2, rho_0 and the state.
hipError_t launch_nps_setup(int dim, const NpsArgs &a, int G, double tol, hipStream_t s);
// BiCGSTAB iteration k (direction, A p, s, A s, update); returns at once after the stop.
hipError_t launch_nps_iter(int dim, const NpsArgs &a, int G, int k, hipStream_t s);
// The stop test before iteration k (one workgroup).
hipError_t launch_nps_check(const NpsArgs &a, int G, int k, hipStream_t s);
// C_out = (float) x for the fluid nodes.
hipError_t launch_nps_store(const NpsArgs &a, float *Cout, __half2 *Clo, hipStream_t s);
// Rates of adsorption, inflow and outflow of the concentrations C (FP64 per
// tile), times scale, added to acc (scale = dt of an implicit step) or
// written to part and reduced into out[0..5] (out != nullptr).
hipError_t launch_nps_rates(int dim, const Grid &g, const Phys &p, const float *C, const float *j, double scale,
                            double *acc, double *part, double *out, hipStream_t s);

}  // namespace cdi
