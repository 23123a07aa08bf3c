// pot_internal.h -- argument block and launchers of the potential solve
// (pot.hip): Poisson's equation, Eq. (4), with the charge of Eq. (5), by
// Jacobi-preconditioned conjugate gradients on the compacted lattice.
#pragma once

#include "cdi_internal.h"

namespace cdi {

// x-end faces of the potential problem (same numbering as the public enum)
constexpr int kPsixDirichlet = 0, kPsixNeumann = 1, kPsixPeriodic = 2;

// upper bound of the persistent workgroups of the solve kernels
constexpr int kPotMaxWorkgroups = 4096;
constexpr int kPotWorkgroupsPerCU = 4;  // cap on resident solver workgroups per compute unit
// A refinement round's FP32 correction solve reduces its residual by this
// factor (or to the overall tolerance, if that is nearer); a round that cuts
// the FP64 residual by less than kPotRefineMinGain hands over to FP64 CG.
constexpr double kPotInnerTol = 1e-4;
constexpr double kPotRefineMinGain = 4.0;

// Solver state in device memory (doubles): stop code, iterations done,
// |r|^2 of the last check, |b|^2, tol^2 |b|^2, Dirichlet faces counted.
enum { kStDone = 0, kStIters = 1, kStRr = 2, kStBb = 3, kStTol2Bb = 4, kStNdir = 5, kStSlots = 8 };
constexpr double kDoneConverged = 1, kDoneDiverged = 2, kDoneBreakdown = 3;

struct PotArgs {
    Grid g;
    int xbc[2];          // kPsix* of the x = 0 and x = nx faces
    double psi_e;        // electrode face value
    double psi_x[2];     // Dirichlet x-face values
    double src;          // kappa2 / (2 c0): charge term per unit sum z C
    float z[2];          // valences
    const float *C;      // concentrations, 2 planes of P
    const float *psi0;   // start (the field in use) or nullptr (zero)
    double *x, *r, *q;   // CG vectors, P each
    double *p, *p2;      // search direction, alternating between two buffers
    float *xf, *rf, *qf; // the FP32 vectors of a refinement round's correction solve
    float *pf, *pf2;
    const int *nbr;      // face neighbours (planes 0 .. 2D-1 of the node list) or nullptr
    uint8_t *dg;         // diagonal of A per node (0 .. 12)
    double *part;        // per-workgroup partial sums (pot_part_doubles)
    double *state;       // kStSlots doubles
};

// Persistent workgroups of a solve on the current device (at most
// kPotMaxWorkgroups, at most one per tile).
hipError_t pot_workgroups(int dim, int ntiles, bool nbr, int *G);
// Doubles of the partial-sum area (sized for kPotMaxWorkgroups).
uint64_t pot_part_doubles();
// x = x0, the diagonal, |b|^2 and the Dirichlet face count into the state;
// the residual of x0 and the stop test come with the first refinement round.
hipError_t launch_pot_setup(int dim, const PotArgs &a, int G, double tol, hipStream_t s);
// CG iteration k (stop test, direction and A p; then the x and r updates) on
// the FP64 vectors or (f32) on the FP32 set; returns at once after a stop.
hipError_t launch_pot_iter(int dim, const PotArgs &a, int G, int k, bool f32, hipStream_t s);
// Refinement round: the FP64 residual of x, the outer stop test (tol), and
// the start of the FP32 correction solve with its own stop threshold (its
// residual falls by max(tol_min, tol |b| / |r|)); f64: the start of FP64 CG
// iterations on x itself instead (tol_min = 0 then stops them at tol).
hipError_t launch_pot_refine(int dim, const PotArgs &a, int G, double tol, double tol_min, bool f64, hipStream_t s);
// x += the FP32 correction.
hipError_t launch_pot_correct(const PotArgs &a, hipStream_t s);
// The stop test of iteration k alone (after iterations up to k - 1).
hipError_t launch_pot_check(const PotArgs &a, int G, int k, hipStream_t s);
// psi[n] = (float) x[n] for the fluid nodes.
hipError_t launch_pot_store(const PotArgs &a, float *psi, hipStream_t s);

}  // namespace cdi
