// Shared declarations of the shifted-system (Helmholtz) solvers: the system
// table, complex helpers and the batch context.  Two schedules exist:
//  * stepped (default): every COCG phase is one launch over the tiles of all
//    running systems, iterations are replayed from a captured HIP graph;
//  * persistent: one cooperative launch in which groups of workgroups run
//    whole solves, taking systems from a device queue.
#pragma once

#include <vector>

#include "multigrid.hpp"
#include "stencil_core.hpp"
#include "tuning.hpp"
#include "vec.hpp"

namespace ofdft {

// H_IDLE marks systems that do not take part in a pass.
enum HDone { H_RUNNING = 0, H_CONVERGED = 1, H_BREAKDOWN = 2, H_NONFINITE = 3, H_MAXIT = 4, H_IDLE = 5 };

struct HSys {
    int nx, ny, nz;
    int nunits;
    TileGeom tg;
    int64_t n;
    Coef<double> coef;
    Coef<float> coef32;
    double kre, kim;          // adjacent: the multigrid cycle reads them as {Re, Im}
    void *x, *r, *pA, *pB, *Ap;
    void *z;                  // preconditioned residual M r (nullptr: no preconditioner)
    const void *f;
};

struct HState;
struct GroupCtl;
struct StepState;

template <typename T> struct CX;
template <> struct CX<double2> {
    using S = double;
    __device__ static double2 mk(double a, double b) { return make_double2(a, b); }
};
template <> struct CX<float2> {
    using S = float;
    __device__ static float2 mk(double a, double b) { return make_float2((float)a, (float)b); }
};

template <typename T>
__device__ inline T cfma(T a, T b, T c) {     // a*b + c (complex)
    T o;
    o.x = c.x + a.x * b.x - a.y * b.y;
    o.y = c.y + a.x * b.y + a.y * b.x;
    return o;
}


template <typename T>
__device__ inline const Coef<typename VT<T>::S> &coef_of(const HSys &s);
template <>
__device__ inline const Coef<double> &coef_of<double2>(const HSys &s) { return s.coef; }
template <>
__device__ inline const Coef<float> &coef_of<float2>(const HSys &s) { return s.coef32; }

// Tile shape actually used for complex element type T: complex128 keeps
// the z queue in registers only with one or two rows per thread, so its
// 16-row shapes map to the 64 x 8 tile of 512 threads.
template <typename T>
inline int cocg_shape(int shape) {
    if (sizeof(T) == 16 && (shape == SHAPE_64x4x4 || shape == SHAPE_64x8x2)) return SHAPE_64x8x1;
    return shape;
}

template <typename T, class F>
inline int dispatch_cocg_shape(int shape, F &&f) {
    if constexpr (sizeof(T) == 16) {
        switch (cocg_shape<T>(shape)) {
            case SHAPE_32x8x2: return f(ShapeTag<32, 8, 2>{});
            case SHAPE_64x8x1: return f(ShapeTag<64, 8, 1>{});
            default: return f(ShapeTag<64, 4, 2>{});
        }
    } else {
        return dispatch_shape(shape, f);
    }
}

}  // namespace ofdft

namespace ofdft {
// Default z-chunk target of the stepped schedule (planes per chunk).
constexpr int kStepPlanes = 80;
}  // namespace ofdft

struct ofdft_batch {
    int nsys = 0, radius = 6;
    ofdft_dtype dtype = OFDFT_C128;
    std::vector<ofdft_grid> grids;
    std::vector<void *> allocs;
    // per system workspaces (complex128: r, pA, pB, Ap; complex64 adds r128, f32, x32)
    std::vector<void *> r, pA, pB, Ap, r128, f32, x32;
    ofdft::HSys *d_sys = nullptr;
    ofdft::HState *d_st = nullptr;
    int *d_order = nullptr;
    ofdft::GroupCtl *d_ctl = nullptr;
    double (*d_part)[4] = nullptr;    // 2 * groups_cap rows of 4 partial sums
    unsigned int *d_queue = nullptr;
    int *d_abort = nullptr;
    double *d_totals = nullptr;   // 2 per system
    ofdft::RedBuf rb{};
    int groups_cap = 0;
    // launch configuration: shape (< 0: default), persistent group size
    // (0: stepped schedule) and the stepped schedule's z-chunk target (planes)
    int shape = -1, P = 0, zplanes = ofdft::kStepPlanes;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // stepped schedule
    ofdft::StepState *d_step = nullptr, *h_step = nullptr;   // per system (host copy pinned)
    int *d_ublk = nullptr, *d_vblk = nullptr;                 // block prefix sums (nsys + 1)
    int *d_xpre = nullptr;       // per XCD: prefix sums of its share of every system's tiles (8 x (nsys + 1))
    int step_grid = 0;           // stencil-phase workgroups: 8 x the longest XCD share
    unsigned int *d_ctr = nullptr;                           // per-system arrival counters
    double *d_spart = nullptr;                               // per-system partial slots
    int step_shape = -1, step_units = 0, step_vblocks = 0;
    std::vector<int> h_ublk, h_vblk;
    hipGraphExec_t step_graph = nullptr;
    hipStream_t step_cap = nullptr;
    int step_graph_key[4] = {-1, -1, -1, -1};
    // preconditioner (OFDFT_PRECOND_*): z = M r per system
    int precond = 0;
    double *d_kap = nullptr;      // {Re, Im} for ofdft_batch_apply_preconditioner
    std::vector<void *> z;
    std::vector<ofdft::Multigrid *> mg_of, mg_own;
    // consecutive systems on one grid form a group: one hierarchy holds their
    // level arrays (system j is member mg_q[j]) and one launch per kernel runs
    // their cycles; groups as (first system, count)
    std::vector<int> mg_q;
    std::vector<std::pair<int, int>> mg_groups;
    void **d_rtab = nullptr, **d_ztab = nullptr;   // r[j], z[j] (device tables)
    // the groups' cycles run on kMgLanes side streams (group g on lane
    // g % lanes), forked from and joined back into the solve's stream, so
    // the latency-bound coarse levels of different groups overlap
    std::vector<hipStream_t> mg_lane;
    std::vector<hipEvent_t> mg_join;
    hipEvent_t mg_fork = nullptr;
};

namespace ofdft {

constexpr int kMgLanes = 4;
constexpr int kMgGroupMax = 64;     // systems per grouped cycle

// Stepped schedule: run COCG on the systems in `which` (system table `hs`
// already uploaded; maxit[j] per system) to relative residual tol.  On return
// iters[j] and done[j] hold the per-system iteration counts and outcomes.
int stepped_run(ofdft_batch *b, bool c64, int shape, const std::vector<HSys> &hs,
                const std::vector<int> &which, const std::vector<int> &maxit, double tol,
                std::vector<int> &iters, std::vector<int> &done, hipStream_t s);
void stepped_free(ofdft_batch *b);
// z-chunk length of the stepped stencil phases on grid g for chunks of about
// `planes` planes (depends only on g, the shape and the batch's setting, so a
// system's reduction order does not depend on the rest of the batch).
int stepped_zlen(const ofdft_grid &g, bool c64, int shape, int planes = kStepPlanes);

}  // namespace ofdft
