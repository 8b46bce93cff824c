// Stepped schedule of the batched COCG solver for the shifted systems
// (-L_h + kappa_j) u_j = f_j (Section 3.1; COCG = conjugate gradients with
// the unconjugated bilinear form x^T y, valid because -L_h + kappa is complex
// symmetric).
//
// Each COCG phase is ONE launch over all running systems of the batch:
//  * stencil phase: the stencil runs on r alone (A r = -L r + kappa r); the
//    new direction and its image follow point by point from the previous
//    ones, p = r + beta p_old and Ap = A r + beta Ap_old (A is linear), so
//    only one array is read with a halo; p^T Ap is reduced;  the grid holds
//    the stencil tiles of every system, so eight 320^3 systems give
//    thousands of workgroups per launch.  Each XCD takes one contiguous
//    eighth of every system's tiles (neighbouring tiles share their halos
//    in that XCD's L2, and the systems still running keep every XCD busy
//    when the others have converged);
//  * vector phase: x += alpha p, r -= alpha Ap, r^T r and |r|^2 reduced.
// The scalars of every system (alpha, beta, r^T r, status) live on the
// device: the last workgroup of a system to finish a phase combines that
// system's partial sums (fixed order, so results do not depend on timing or
// on the other systems of the batch) and updates its scalars.  Converged
// systems' workgroups exit at once.  Iterations are captured once in a HIP
// graph and replayed; the host only polls the status array between replays.
// No workgroup ever waits for another inside a launch.
//
// With a preconditioner M (one multigrid cycle per system, complex
// symmetric) the iteration is preconditioned COCG: after the vector phase
// z = M r is formed by the cycle's own launches, a dot phase reduces
// rho = r^T z and sets beta = rho_new / rho, and the stencil phase runs on z:
// p = z + beta p_old, Ap = A z + beta Ap_old.
#include <algorithm>
#include <cmath>

#include "helmholtz.hpp"

namespace ofdft {

struct StepState {
    double rr_re, rr_im;     // r^T r (preconditioned: r^T z) of the current residual
    double al_re, al_im;     // alpha of the current iteration
    double be_re, be_im;     // beta of the next direction
    double rn2, fn2, tol2;   // |r|^2, |f|^2, tol^2 |f|^2
    int iter, done, maxit, parity;   // parity: 0 -> p_old in pA, 1 -> p_old in pB
    int xpend, pad;          // x += alpha p of the last direction still to apply
};

namespace {

constexpr int kStepIters = 4;          // iterations per captured graph
constexpr int kVecThreadsStep = 256;
constexpr int kVecMaxBlocks = 1024;    // per system

// System of logical block b: start[j] <= b < start[j + 1].
__device__ inline int find_sys(const int *start, int nsys, int b) {
    int lo = 0, hi = nsys;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename T>
struct StepLoadX {
    GPtr<T> x;
    __device__ T operator()(int64_t i) const { return x[i]; }
};


template <typename T>
struct StepEpiInit {     // r = f - (-L x + kappa x); acc {r^T r re, im, |r|^2, |f|^2}
    GPtr<T> f, r;
    T kappa;
    double acc[4];
    T fv[4];
    __device__ void pre(int q, int64_t i) { fv[q] = f[i]; }
    __device__ void point(int q, int64_t i, T c, T s) {
        const T ax = cfma(kappa, c, T{-s.x, -s.y});
        const T fi = fv[q];
        const T rv{fi.x - ax.x, fi.y - ax.y};
        r.st(i, rv);
        const double a = rv.x, b = rv.y;
        acc[0] += a * a - b * b;
        acc[1] += 2.0 * a * b;
        acc[2] += a * a + b * b;
        acc[3] += (double)fi.x * fi.x + (double)fi.y * fi.y;
    }
};

// Centre = r (z when preconditioned), s = L r.  p = r + beta p_old and
// Ap = (-L r + kappa r) + beta Ap_old, Ap updated in place (each point is read
// and written by the same thread); the previous iteration's x += alpha p_old
// is applied here too, where p_old is read anyway (the vector phase then
// moves r and Ap only; the last direction's update is left to step_finish).
// The first iteration (beta = 0, no previous direction) reads neither p_old,
// Ap_old nor x.  acc {p^T Ap re, im}.  The first iteration is
// a kernel of its own: with a run-time flag the loads and their use sit in
// branches, and the compiler then waits for the halo fetches of the previous
// plane before it reuses the registers of these loads.
template <typename T, bool First>
struct StepEpiPAp {
    GPtr<T> p_old, p_out, Ap, x;
    T kappa, beta, alpha;
    double acc[2];
    T po[4], ao[4], xo[4];
    __device__ void pre(int q, int64_t i) {
        if constexpr (!First) {
            po[q] = p_old[i];
            ao[q] = Ap[i];
            xo[q] = x[i];
        }
    }
    __device__ void point(int q, int64_t i, T c, T s) {
        T a = cfma(kappa, c, T{-s.x, -s.y});
        T p = c;
        if constexpr (!First) {
            x.st(i, cfma(alpha, po[q], xo[q]));
            p = cfma(beta, po[q], c);
            a = cfma(beta, ao[q], a);
        }
        p_out.st(i, p);
        Ap.st(i, a);
        acc[0] += (double)p.x * a.x - (double)p.y * a.y;
        acc[1] += (double)p.x * a.y + (double)p.y * a.x;
    }
};

enum StepPhase { PH_INIT = 0, PH_PAP = 1, PH_PAP_FIRST = 2 };

// Stencil phases.  part: 4 slots per unit, system j's region starts at
// 4 * ublk[j] and is laid out [k][unit].
template <typename T, int TX, int TYT, int RY, int Phase>
__global__ void __launch_bounds__(TX * TYT)
step_stencil(const HSys *sys, StepState *st, const int *ublk, const int *xpre, int nsys,
             unsigned int *ctr, double *part, double tol) {
    using CT = CX<T>;
    __shared__ T lds[StencilLds<T, TX, TYT, RY>::kElems];
    __shared__ double scratch[4 * (TX * TYT / 64)];
    // workgroup b runs on XCD b % 8; that XCD's list holds, system after
    // system, the tiles [n x / 8, n (x + 1) / 8) of each system of n tiles
    constexpr int kXcd = 8;
    const int x = blockIdx.x % kXcd, l = blockIdx.x / kXcd;
    const int *xp = xpre + x * (nsys + 1);
    if (l >= xp[nsys]) return;
    const int j = find_sys(xp, nsys, l);
    StepState *sj = st + j;
    const int done = sj->done;
    if (done != H_RUNNING) return;
    const HSys &h = sys[j];
    const int nunits = ublk[j + 1] - ublk[j];
    const int unit = (int)(((int64_t)nunits * x) / kXcd) + (l - xp[j]);
    double *pj = part + 4 * (size_t)ublk[j];
    const T kappa = CT::mk(h.kre, h.kim);
    if constexpr (Phase == PH_INIT) {
        StepLoadX<T> ld{GPtr<T>(h.x)};
        StepEpiInit<T> ep{GPtr<T>(h.f), GPtr<T>(h.r), kappa, {0, 0, 0, 0}, {}};
        stencil_tile<T, TX, TYT, RY>(h.tg, coef_of<T>(h), ld, ep, unit, lds);
        double acc[4] = {ep.acc[0], ep.acc[1], ep.acc[2], ep.acc[3]};
        block_sum<4>(acc, scratch);
        double t[4];
        if (reduce_grid<4>(acc, pj, nunits, unit, ctr + j, scratch, t)) {
            sj->rr_re = t[0];
            sj->rr_im = t[1];
            sj->rn2 = t[2];
            sj->fn2 = t[3];
            sj->tol2 = tol * tol * t[3];
            sj->iter = 0;
            sj->parity = 0;
            int d = !isfinite(t[2]) ? H_NONFINITE : (t[2] <= sj->tol2 ? H_CONVERGED : H_RUNNING);
            if (d == H_RUNNING && sj->maxit <= 0) d = H_MAXIT;
            sj->done = d;
        }
    } else {
        // PH_PAP_FIRST runs iteration 0 of every running system, PH_PAP the
        // later ones (the host launches the first right after the init phase)
        const void *p_old = sj->parity ? h.pB : h.pA;
        const void *p_new = sj->parity ? h.pA : h.pB;
        const void *base = h.z ? h.z : h.r;
        StepLoadX<T> ld{GPtr<T>(base)};
        // alpha of the previous iteration: the last workgroup below sets this
        // iteration's only after every workgroup has arrived
        StepEpiPAp<T, Phase == PH_PAP_FIRST> ep{GPtr<T>(p_old), GPtr<T>(p_new), GPtr<T>(h.Ap), GPtr<T>(h.x),
                                                kappa, CT::mk(sj->be_re, sj->be_im),
                                                CT::mk(sj->al_re, sj->al_im), {0, 0}, {}, {}, {}};
        stencil_tile<T, TX, TYT, RY>(h.tg, coef_of<T>(h), ld, ep, unit, lds);
        double acc[2] = {ep.acc[0], ep.acc[1]};
        block_sum<2>(acc, scratch);
        double t[2];
        if (reduce_grid<2>(acc, pj, nunits, unit, ctr + j, scratch, t)) {
            const double den = t[0] * t[0] + t[1] * t[1];
            // the previous direction's x update is applied by now
            sj->xpend = 0;
            if (!isfinite(den)) {
                sj->done = H_NONFINITE;
            } else if (den == 0.0) {
                sj->done = H_BREAKDOWN;
            } else {
                sj->al_re = (sj->rr_re * t[0] + sj->rr_im * t[1]) / den;
                sj->al_im = (sj->rr_im * t[0] - sj->rr_re * t[1]) / den;
                sj->xpend = 1;
            }
        }
    }
}

// Vector phase: r -= alpha Ap (x follows in the next stencil phase or in
// step_finish); then beta (unpreconditioned) and status.  part region of system j starts at 4 * vblk[j] (the caller
// offsets part past the stencil slots).
template <typename T>
__global__ void __launch_bounds__(kVecThreadsStep)
step_update(const HSys *sys, StepState *st, const int *vblk, int nsys, unsigned int *ctr,
            double *part) {
    using CT = CX<T>;
    __shared__ double scratch[3 * (kVecThreadsStep / 64)];
    const int b = blockIdx.x;
    const int j = find_sys(vblk, nsys, b);
    StepState *sj = st + j;
    if (sj->done != H_RUNNING) return;
    const HSys &h = sys[j];
    const int lb = b - vblk[j], nb = vblk[j + 1] - vblk[j];
    const GPtr<T> r(h.r), Ap(h.Ap);
    const T nal = CT::mk(-sj->al_re, -sj->al_im);
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)nb * kVecThreadsStep;
    for (int64_t i = (int64_t)lb * kVecThreadsStep + threadIdx.x; i < h.n; i += stride) {
        const T rv = cfma(nal, Ap[i], r[i]);
        r.st(i, rv);
        const double a = rv.x, c = rv.y;
        acc[0] += a * a - c * c;
        acc[1] += 2.0 * a * c;
        acc[2] += a * a + c * c;
    }
    block_sum<3>(acc, scratch);
    double t[3];
    if (reduce_grid<3>(acc, part + 4 * (size_t)vblk[j], nb, lb, ctr + j, scratch, t)) {
        const bool pre = h.z != nullptr;        // rho and beta come from the dot phase
        if (!pre) {
            const double rr_re = sj->rr_re, rr_im = sj->rr_im;
            const double d2 = rr_re * rr_re + rr_im * rr_im;
            sj->be_re = (t[0] * rr_re + t[1] * rr_im) / d2;
            sj->be_im = (t[1] * rr_re - t[0] * rr_im) / d2;
            sj->rr_re = t[0];
            sj->rr_im = t[1];
        }
        sj->rn2 = t[2];
        const int iter = sj->iter + 1;
        sj->iter = iter;
        sj->parity ^= 1;
        int d = H_RUNNING;
        if (!isfinite(t[2])) d = H_NONFINITE;
        else if (t[2] <= sj->tol2) d = H_CONVERGED;
        else if (!pre && t[0] * t[0] + t[1] * t[1] <= 1e-60 * t[2] * t[2]) d = H_BREAKDOWN;
        else if (iter >= sj->maxit) d = H_MAXIT;
        sj->done = d;
    }
}

// x += alpha p of the last direction of every system whose update is still
// pending (the stencil phase applies each direction's update one iteration
// late, so a converged, capped or stopped system owes its last one).
template <typename T>
__global__ void __launch_bounds__(kVecThreadsStep)
step_finish(const HSys *sys, const StepState *st, const int *vblk, int nsys) {
    using CT = CX<T>;
    const int b = blockIdx.x;
    const int j = find_sys(vblk, nsys, b);
    const StepState *sj = st + j;
    if (!sj->xpend) return;
    const HSys &h = sys[j];
    const int lb = b - vblk[j], nb = vblk[j + 1] - vblk[j];
    // the direction written by the last stencil phase (parity has flipped since)
    const GPtr<T> x(h.x), p(sj->parity ? h.pB : h.pA);
    const T al = CT::mk(sj->al_re, sj->al_im);
    const int64_t stride = (int64_t)nb * kVecThreadsStep;
    for (int64_t i = (int64_t)lb * kVecThreadsStep + threadIdx.x; i < h.n; i += stride)
        x.st(i, cfma(al, p[i], x[i]));
}

// Dot phase of the preconditioned iteration: rho = r^T z, |z|^2; first call
// of a solve (iter 0) sets rho, later ones beta = rho_new / rho and rho.
template <typename T>
__global__ void __launch_bounds__(kVecThreadsStep)
step_dot(const HSys *sys, StepState *st, const int *vblk, int nsys, unsigned int *ctr, double *part) {
    __shared__ double scratch[3 * (kVecThreadsStep / 64)];
    const int b = blockIdx.x;
    const int j = find_sys(vblk, nsys, b);
    StepState *sj = st + j;
    const HSys &h = sys[j];
    if (sj->done != H_RUNNING || !h.z) return;
    const int lb = b - vblk[j], nb = vblk[j + 1] - vblk[j];
    const GPtr<T> r(h.r), z(h.z);
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)nb * kVecThreadsStep;
    for (int64_t i = (int64_t)lb * kVecThreadsStep + threadIdx.x; i < h.n; i += stride) {
        const T a = r[i], c = z[i];
        acc[0] += (double)a.x * c.x - (double)a.y * c.y;
        acc[1] += (double)a.x * c.y + (double)a.y * c.x;
        acc[2] += (double)c.x * c.x + (double)c.y * c.y;
    }
    block_sum<3>(acc, scratch);
    double t[3];
    if (reduce_grid<3>(acc, part + 4 * (size_t)vblk[j], nb, lb, ctr + j, scratch, t)) {
        if (!isfinite(t[0]) || !isfinite(t[1]) || !isfinite(t[2])) {
            sj->done = H_NONFINITE;
        } else if (t[0] * t[0] + t[1] * t[1] <= 1e-60 * sj->rn2 * t[2]) {
            sj->done = H_BREAKDOWN;
        } else {
            if (sj->iter > 0) {
                const double rr_re = sj->rr_re, rr_im = sj->rr_im;
                const double d2 = rr_re * rr_re + rr_im * rr_im;
                sj->be_re = (t[0] * rr_re + t[1] * rr_im) / d2;
                sj->be_im = (t[1] * rr_re - t[0] * rr_im) / d2;
            }
            sj->rr_re = t[0];
            sj->rr_im = t[1];
        }
    }
}

template <typename T, int TX, int TYT, int RY>
int launch_phase(ofdft_batch *b, int phase, double tol, hipStream_t s) {
    const int grid = b->step_grid;
    auto kern = phase == PH_INIT ? step_stencil<T, TX, TYT, RY, PH_INIT>
                : phase == PH_PAP_FIRST ? step_stencil<T, TX, TYT, RY, PH_PAP_FIRST>
                : step_stencil<T, TX, TYT, RY, PH_PAP>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(TX, TYT), 0, s, b->d_sys, b->d_step, b->d_ublk, b->d_xpre,
                       b->nsys, b->d_ctr, b->d_spart, tol);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

template <typename T>
int launch_stencil_phase(ofdft_batch *b, int shape, int phase, double tol, hipStream_t s) {
    return dispatch_cocg_shape<T>(shape, [&](auto sh) {
        using S = decltype(sh);
        return launch_phase<T, S::TX, S::TYT, S::RY>(b, phase, tol, s);
    });
}

template <typename T>
int launch_update(ofdft_batch *b, hipStream_t s) {
    hipLaunchKernelGGL(step_update<T>, dim3(b->step_vblocks), dim3(kVecThreadsStep), 0, s, b->d_sys,
                       b->d_step, b->d_vblk, b->nsys, b->d_ctr, b->d_spart + 4 * (size_t)b->step_units);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

// z = M r of every preconditioned system, then rho = r^T z (and beta).
// Systems that are not running skip both inside the kernels.  The cycles run
// on the batch's side streams (forked from s and joined back; inside a graph
// capture this makes parallel branches).  Timed: the host reads the
// statuses first and launches (and times) only the cycles of running
// systems, one after another on s, so each cycle's duration is its own;
// otherwise the caller accounts them.
int precondition(ofdft_batch *b, hipStream_t s, bool timed) {
    if (timed) {
        OFDFT_CHECK_HIP(hipMemcpyAsync(b->h_step, b->d_step, sizeof(StepState) * b->nsys, hipMemcpyDeviceToHost, s));
        OFDFT_CHECK_HIP(hipStreamSynchronize(s));
    }
    static_assert(sizeof(HSys) % sizeof(double) == 0 && sizeof(StepState) % sizeof(int) == 0,
                  "per-system shift and status strides");
    const int lanes = timed ? 0 : (int)b->mg_lane.size();
    if (lanes) OFDFT_CHECK_HIP(hipEventRecord(b->mg_fork, s));
    for (int k = 0; k < lanes; ++k) OFDFT_CHECK_HIP(hipStreamWaitEvent(b->mg_lane[k], b->mg_fork, 0));
    if (timed) {
        // one cycle per running system, one after another on s, each timed
        for (int j = 0; j < b->nsys; ++j) {
            if (b->h_step[j].done != H_RUNNING) continue;
            // bytes are added after the pass from the iteration counts
            ProfScope ps(K_MULTIGRID_C, 0.0, s);
            OFDFT_TRY(mg_apply_shifted(*b->mg_of[j], b->mg_q[j], (const double2 *)b->r[j], (double2 *)b->z[j],
                                       &b->d_sys[j].kre, &b->d_step[j].done, s));
        }
    } else {
        // one grouped cycle per group: shift {kre, kim} and status of system j
        // at d_sys[j] and d_step[j]; converged systems' workgroups return at once
        for (size_t g = 0; g < b->mg_groups.size(); ++g) {
            const int j0 = b->mg_groups[g].first, cnt = b->mg_groups[g].second;
            hipStream_t q = lanes ? b->mg_lane[g % lanes] : s;
            OFDFT_TRY(mg_apply_shifted_group(*b->mg_of[j0], cnt, (const double2 *const *)(b->d_rtab + j0),
                                             (double2 *const *)(b->d_ztab + j0), &b->d_sys[j0].kre,
                                             (int)(sizeof(HSys) / sizeof(double)), &b->d_step[j0].done,
                                             (int)(sizeof(StepState) / sizeof(int)), q));
        }
    }
    for (int k = 0; k < lanes; ++k) {
        OFDFT_CHECK_HIP(hipEventRecord(b->mg_join[k], b->mg_lane[k]));
        OFDFT_CHECK_HIP(hipStreamWaitEvent(s, b->mg_join[k], 0));
    }
    ProfScope ps(K_COCG_UPDATE, 0.0, s, timed);
    hipLaunchKernelGGL(step_dot<double2>, dim3(b->step_vblocks), dim3(kVecThreadsStep), 0, s, b->d_sys,
                       b->d_step, b->d_vblk, b->nsys, b->d_ctr, b->d_spart + 4 * (size_t)b->step_units);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

// `iters` iterations of all phases.  Timed: each launch is accounted and
// timed on its own; otherwise (graph capture) the caller accounts replays.
template <typename T>
int step_iterations(ofdft_batch *b, int shape, int iters, hipStream_t s, bool timed) {
    for (int k = 0; k < iters; ++k) {
        {
            ProfScope ps(K_COCG, 0.0, s, timed);
            OFDFT_TRY(launch_stencil_phase<T>(b, shape, PH_PAP, 0.0, s));
        }
        {
            ProfScope ps(K_COCG_UPDATE, 0.0, s, timed);
            OFDFT_TRY(launch_update<T>(b, s));
        }
        if (b->precond) OFDFT_TRY(precondition(b, s, timed));
    }
    return OFDFT_OK;
}

// Iteration 0 of every running system (eager: the captured block holds
// later iterations only).  Accounted like the init phase.
template <typename T>
int first_iteration(ofdft_batch *b, int shape, hipStream_t s, bool timed) {
    {
        ProfScope ps(K_COCG, 0.0, s);
        OFDFT_TRY(launch_stencil_phase<T>(b, shape, PH_PAP_FIRST, 0.0, s));
    }
    {
        ProfScope ps(K_COCG_UPDATE, 0.0, s);
        OFDFT_TRY(launch_update<T>(b, s));
    }
    if (b->precond) {
        OFDFT_TRY(precondition(b, s, timed));
        if (!timed) {
            prof_add(K_COCG_UPDATE, 0.0, 1);
            prof_add(K_MULTIGRID_C, 0.0, b->nsys);
        }
    }
    return OFDFT_OK;
}

template <typename T>
int graph_get(ofdft_batch *b, int shape) {
    const int key[4] = {shape, (int)sizeof(T), b->step_units, b->precond};
    if (b->step_graph && std::equal(key, key + 4, b->step_graph_key)) return OFDFT_OK;
    if (b->step_graph) {
        (void)hipGraphExecDestroy(b->step_graph);
        b->step_graph = nullptr;
    }
    if (!b->step_cap) OFDFT_CHECK_HIP(hipStreamCreateWithFlags(&b->step_cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    OFDFT_CHECK_HIP(hipStreamBeginCapture(b->step_cap, hipStreamCaptureModeThreadLocal));
    const int rc = step_iterations<T>(b, shape, kStepIters, b->step_cap, false);
    const hipError_t e = hipStreamEndCapture(b->step_cap, &graph);
    if (rc != OFDFT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    OFDFT_CHECK_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&b->step_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    OFDFT_CHECK_HIP(ei);
    for (int i = 0; i < 4; ++i) b->step_graph_key[i] = key[i];
    return OFDFT_OK;
}

// Block tables of the current system table (units from the uploaded tile
// geometries, vector blocks from the sizes) and the partial-slot buffer.
int prepare_layout(ofdft_batch *b, const std::vector<HSys> &hs, hipStream_t s) {
    const int nsys = b->nsys;
    std::vector<int> ublk(nsys + 1, 0), vblk(nsys + 1, 0);
    for (int j = 0; j < nsys; ++j) {
        ublk[j + 1] = ublk[j] + hs[j].tg.nblocks;
        const int64_t want = (hs[j].n + 8 * kVecThreadsStep - 1) / (8 * kVecThreadsStep);
        vblk[j + 1] = vblk[j] + (int)std::max<int64_t>(1, std::min<int64_t>(want, kVecMaxBlocks));
    }
    if (ublk == b->h_ublk && vblk == b->h_vblk) return OFDFT_OK;
    if (b->step_graph) {                    // captured with the old tables
        OFDFT_CHECK_HIP(hipStreamSynchronize(s));
        (void)hipGraphExecDestroy(b->step_graph);
        b->step_graph = nullptr;
    }
    // per-XCD shares of every system's tiles (see step_stencil)
    std::vector<int> xpre(8 * (size_t)(nsys + 1), 0);
    int longest = 0;
    for (int x = 0; x < 8; ++x) {
        int *xp = xpre.data() + x * (nsys + 1);
        for (int j = 0; j < nsys; ++j) {
            const int64_t nu = ublk[j + 1] - ublk[j];
            xp[j + 1] = xp[j] + (int)(nu * (x + 1) / 8 - nu * x / 8);
        }
        longest = std::max(longest, xp[nsys]);
    }
    if (!b->d_ublk) {
        OFDFT_CHECK_HIP(hipMalloc(&b->d_xpre, sizeof(int) * 8 * (nsys + 1)));
        OFDFT_CHECK_HIP(hipMalloc(&b->d_ublk, sizeof(int) * (nsys + 1)));
        OFDFT_CHECK_HIP(hipMalloc(&b->d_vblk, sizeof(int) * (nsys + 1)));
        OFDFT_CHECK_HIP(hipMalloc(&b->d_ctr, sizeof(unsigned int) * nsys));
        OFDFT_CHECK_HIP(hipMalloc(&b->d_step, sizeof(StepState) * nsys));
        OFDFT_CHECK_HIP(hipHostMalloc(&b->h_step, sizeof(StepState) * nsys, hipHostMallocDefault));
        OFDFT_CHECK_HIP(hipMemsetAsync(b->d_ctr, 0, sizeof(unsigned int) * nsys, s));
    }
    const size_t slots = 4 * ((size_t)ublk[nsys] + (size_t)vblk[nsys]);
    const size_t have = 4 * ((size_t)(b->h_ublk.empty() ? 0 : b->h_ublk[nsys]) +
                             (size_t)(b->h_vblk.empty() ? 0 : b->h_vblk[nsys]));
    if (!b->d_spart || slots > have) {
        if (b->d_spart) OFDFT_CHECK_HIP(hipFree(b->d_spart));
        b->d_spart = nullptr;
        OFDFT_CHECK_HIP(hipMalloc(&b->d_spart, sizeof(double) * slots));
    }
    OFDFT_CHECK_HIP(hipMemcpyAsync(b->d_ublk, ublk.data(), sizeof(int) * (nsys + 1), hipMemcpyHostToDevice, s));
    OFDFT_CHECK_HIP(hipMemcpyAsync(b->d_xpre, xpre.data(), sizeof(int) * xpre.size(), hipMemcpyHostToDevice, s));
    OFDFT_CHECK_HIP(hipMemcpyAsync(b->d_vblk, vblk.data(), sizeof(int) * (nsys + 1), hipMemcpyHostToDevice, s));
    OFDFT_CHECK_HIP(hipStreamSynchronize(s));
    b->h_ublk = ublk;
    b->h_vblk = vblk;
    b->step_units = ublk[nsys];
    b->step_grid = 8 * std::max(longest, 1);
    b->step_vblocks = vblk[nsys];
    return OFDFT_OK;
}

template <typename T>
int run_t(ofdft_batch *b, int shape, const std::vector<HSys> &hs, const std::vector<int> &which, const std::vector<int> &maxit,
          double tol, std::vector<int> &iters, std::vector<int> &done, hipStream_t s) {
    const int nsys = b->nsys;
    for (int j = 0; j < nsys; ++j) {
        b->h_step[j] = StepState{};
        b->h_step[j].done = H_IDLE;
        b->h_step[j].maxit = maxit[j];
    }
    for (int j : which) b->h_step[j].done = H_RUNNING;
    OFDFT_CHECK_HIP(hipMemcpyAsync(b->d_step, b->h_step, sizeof(StepState) * nsys, hipMemcpyHostToDevice, s));
    const bool timed = prof_timed(K_COCG) || prof_timed(K_COCG_UPDATE) ||
                       (b->precond && prof_timed(K_MULTIGRID_C));
    {
        ProfScope ps(K_COCG, 0.0, s);
        OFDFT_TRY(launch_stencil_phase<T>(b, shape, PH_INIT, tol, s));
    }
    if (b->precond) {
        OFDFT_TRY(precondition(b, s, timed));
        if (!timed) {
            prof_add(K_COCG_UPDATE, 0.0, 1);
            prof_add(K_MULTIGRID_C, 0.0, nsys);
        }
    }
    int reps = 1;
    std::vector<double> rn2_0(nsys, 0.0);     // residual after the init phase
    bool first = true;
    for (;;) {
        OFDFT_CHECK_HIP(hipMemcpyAsync(b->h_step, b->d_step, sizeof(StepState) * nsys, hipMemcpyDeviceToHost, s));
        OFDFT_CHECK_HIP(hipStreamSynchronize(s));
        bool running = false;
        for (int j : which) running = running || b->h_step[j].done == H_RUNNING;
        if (!running) break;
        if (first) {
            for (int j : which) rn2_0[j] = b->h_step[j].rn2;
            first = false;
            OFDFT_TRY(first_iteration<T>(b, shape, s, timed));
        } else {
            // replays until the slowest running system is predicted to converge,
            // from its mean residual reduction per iteration so far
            double need = 0.0;
            bool known = true;
            for (int j : which) {
                const StepState &q = b->h_step[j];
                if (q.done != H_RUNNING) continue;
                const double rate = q.iter > 0 && rn2_0[j] > 0 ? std::log(q.rn2 / rn2_0[j]) / q.iter : 0.0;
                if (!(rate < -1e-3) || !std::isfinite(rate)) {
                    known = false;
                    break;
                }
                need = std::max(need, std::log(q.tol2 / q.rn2) / rate);
            }
            reps = known ? (int)std::ceil(std::max(need, 1.0) / kStepIters) : reps * 2;
            reps = std::max(1, std::min(reps, 32));
        }
        if (timed) {
            OFDFT_TRY(step_iterations<T>(b, shape, reps * kStepIters, s, true));
        } else {
            OFDFT_TRY(graph_get<T>(b, shape));
            for (int k = 0; k < reps; ++k) OFDFT_CHECK_HIP(hipGraphLaunch(b->step_graph, s));
            prof_add(K_COCG, 0.0, reps * kStepIters);
            prof_add(K_COCG_UPDATE, 0.0, reps * kStepIters * (b->precond ? 2 : 1));
            if (b->precond) prof_add(K_MULTIGRID_C, 0.0, (int64_t)reps * kStepIters * nsys);
        }
    }
    // the last directions' x updates (read x, p; write x)
    double fin = 0.0;
    for (int j : which)
        if (b->h_step[j].xpend) fin += 3.0 * sizeof(T) * (double)hs[j].n;
    if (fin > 0.0) {
        ProfScope ps(K_COCG_UPDATE, fin, s);
        hipLaunchKernelGGL(step_finish<T>, dim3(b->step_vblocks), dim3(kVecThreadsStep), 0, s, b->d_sys, b->d_step,
                           b->d_vblk, b->nsys);
        OFDFT_CHECK_HIP(hipGetLastError());
    }
    for (int j = 0; j < nsys; ++j) {
        iters[j] = b->h_step[j].iter;
        done[j] = b->h_step[j].done;
    }
    return OFDFT_OK;
}

}  // namespace

// Chunks of about `planes` planes (default 80): long enough for little
// queue warm-up, short enough that one or two systems still running (the
// tail of a batch) spread over more workgroups than the chip's CUs
// (measured: 80 beat 160 and 40 at 320^3; the autotuner times others); they
// shrink down to 8 planes while a system would have fewer than 32 tiles.
int stepped_zlen(const ofdft_grid &g, bool, int shape, int planes) {
    int tx, ty;
    shape_extent(shape, tx, ty);
    const int64_t tiles = (int64_t)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
    planes = std::max(planes, 8);
    int chunks = std::max(1, (g.nz + planes - 1) / planes);
    while (tiles * chunks < 32 && g.nz / (chunks + 1) >= 8) ++chunks;
    return (g.nz + chunks - 1) / chunks;
}

int stepped_run(ofdft_batch *b, bool c64, int shape, const std::vector<HSys> &hs,
                const std::vector<int> &which, const std::vector<int> &maxit, double tol,
                std::vector<int> &iters, std::vector<int> &done, hipStream_t s) {
    if (b->precond && c64) return OFDFT_INVALID_ARG;
    OFDFT_TRY(prepare_layout(b, hs, s));
    if (c64) return run_t<float2>(b, shape, hs, which, maxit, tol, iters, done, s);
    return run_t<double2>(b, shape, hs, which, maxit, tol, iters, done, s);
}

void stepped_free(ofdft_batch *b) {
    if (b->step_graph) (void)hipGraphExecDestroy(b->step_graph);
    if (b->step_cap) (void)hipStreamDestroy(b->step_cap);
    if (b->d_xpre) (void)hipFree(b->d_xpre);
    if (b->d_ublk) (void)hipFree(b->d_ublk);
    if (b->d_vblk) (void)hipFree(b->d_vblk);
    if (b->d_ctr) (void)hipFree(b->d_ctr);
    if (b->d_step) (void)hipFree(b->d_step);
    if (b->h_step) (void)hipHostFree(b->h_step);
    if (b->d_spart) (void)hipFree(b->d_spart);
    b->step_graph = nullptr;
    b->step_cap = nullptr;
    b->d_ublk = b->d_vblk = b->d_xpre = nullptr;
    b->d_ctr = nullptr;
    b->d_step = b->h_step = nullptr;
    b->d_spart = nullptr;
}

}  // namespace ofdft
