// Geometric multigrid preconditioner for the periodic Poisson solve (the
// real-space preconditioner the paper's conclusion calls for, Section 5.5).
//
// M approximates the inverse of the 12th-order -L_h with one V(nu, nu) cycle
// of the second-order 7-point operator: damped Jacobi smoothing, full
// weighting restriction (R = P^T / 8), trilinear prolongation, every axis
// halved per level, and an exact DFT solve on the coarsest grid (at most 16
// points per axis).  The cycle is a fixed linear operator, symmetric and
// positive definite on zero-mean vectors, so CG preconditioned by it
// converges at a rate set by the spectral equivalence of the two operators,
// independent of the grid size.
#pragma once

#include <vector>

#include "common.hpp"

namespace ofdft {

struct MgLevel {
    int nx = 0, ny = 0, nz = 0;
    double cx = 0, cy = 0, cz = 0;   // 1 / h_a^2
    int64_t n = 0;
    double *u = nullptr, *t = nullptr, *f = nullptr, *r = nullptr;
};

struct Multigrid {
    std::vector<MgLevel> lv;
    int nu = 2;                  // Jacobi sweeps before and after the coarse correction
    double omega = 0.8;          // Jacobi damping
    std::vector<void *> allocs;
};

constexpr int kMgCoarseMax = 16;     // coarsest grid: at most this many points per axis

// Hierarchy for grid g: halve every axis while all are even and one exceeds
// kMgCoarseMax.  INVALID_ARG if the coarsest grid would be larger than that.
int mg_create(Multigrid &mg, const ofdft_grid &g);
void mg_free(Multigrid &mg);
// z = M r (device FP64 arrays of the fine grid; z must not alias r).
int mg_apply(Multigrid &mg, const double *r, double *z, hipStream_t s);

}  // namespace ofdft
