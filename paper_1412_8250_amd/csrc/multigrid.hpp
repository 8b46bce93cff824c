// Geometric multigrid preconditioner for the periodic Poisson solve (the
// real-space preconditioner the paper's conclusion calls for, Section 5.5).
//
// M approximates the inverse of the 12th-order -L_h (+ kappa for the shifted
// systems) with one V(nu, nu) cycle of the second-order 7-point operator
// (+ kappa): damped Jacobi smoothing, full
// weighting restriction (R = P^T / 8), trilinear prolongation, every axis
// halved per level, and an exact DFT solve on the coarsest grid (at most 16
// points per axis).  The cycle is a fixed linear operator, symmetric and
// positive definite on zero-mean vectors (complex symmetric for a complex
// shift), so CG (COCG) preconditioned by it converges at a rate set by the
// spectral equivalence of the two operators, independent of the grid size.
#pragma once

#include <vector>

#include "common.hpp"

namespace ofdft {

struct MgLevel {
    int nx = 0, ny = 0, nz = 0;
    double cx = 0, cy = 0, cz = 0;   // 1 / h_a^2
    int64_t n = 0;
    void *u = nullptr, *t = nullptr, *f = nullptr, *r = nullptr;   // FP64 or complex128
};

struct Multigrid {
    std::vector<MgLevel> lv;
    static constexpr int nu = 2; // Jacobi sweeps before and after the coarse correction
    double omega = 0.8;          // Jacobi damping
    int elem = 8;                // input / output element bytes: 8 (FP64) or 16 (complex128)
    bool fp32 = true;            // level arrays and their arithmetic in FP32 (else FP64)
    int groups = 1;              // systems whose level arrays the hierarchy holds (same grid)
    std::vector<void *> allocs;
};

constexpr int kMgCoarseMax = 16;     // coarsest grid: at most this many points per axis

// Hierarchy for grid g, applied to FP64 (elem_bytes 8) or complex128 (16)
// vectors; the level arrays (and the arithmetic on them) are FP32 / complex64
// when fp32 is set: the cycle then reads r and writes z in FP64 but is a fixed
// linear operator only to FP32 rounding, which the flexible and preconditioned
// Krylov loops here tolerate without extra iterations.  Every axis is halved
// while all are even and one exceeds kMgCoarseMax; INVALID_ARG if the
// coarsest grid would be larger than that.
// `groups` systems of this grid get level arrays of their own (system q's
// part of a level array starts q * n elements in), so that one launch per
// kernel can run the cycles of all of them.
int mg_create(Multigrid &mg, const ofdft_grid &g, int elem_bytes, bool fp32, int groups = 1);
void mg_free(Multigrid &mg);
// z = M r for -Delta + kappa, kappa >= 0 real (device FP64 arrays of the fine
// grid; z must not alias r).
int mg_apply(Multigrid &mg, const double *r, double *z, hipStream_t s, double kappa = 0.0);
// The same cycle, every kernel returning at once while *run != 0 (device
// flag, for cycles inside captured blocks of an iteration that may be over).
int mg_apply_run(Multigrid &mg, const double *r, double *z, hipStream_t s, double kappa, const int *run);
// z = M r for -Delta + kappa (complex128 arrays).  kappa points to device
// memory holding {Re, Im} and is read by every launch, so a captured launch
// sequence follows later changes of the shift; if `run` is given, every
// kernel returns at once unless *run == 0 (a converged system of a batch).
// Not accounted in the profile (the caller accounts cycles).
// System q of the hierarchy's group does the cycle.
int mg_apply_shifted(Multigrid &mg, int q, const double2 *r, double2 *z, const double *kappa, const int *run,
                     hipStream_t s);
// The cycles of systems 0 .. count-1 of the group in one launch per kernel:
// system q reads r[q], writes z[q] (device tables of device pointers), its
// shift at kappa + q kstride and its run flag at run + q rstride (run may be
// null).  Not accounted in the profile.
int mg_apply_shifted_group(Multigrid &mg, int count, const double2 *const *r, double2 *const *z,
                           const double *kappa, int kstride, const int *run, int rstride, hipStream_t s);
// Algorithmic HBM bytes of one cycle.
double mg_cycle_bytes(const Multigrid &mg);

}  // namespace ofdft
