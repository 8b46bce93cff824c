// cg_poisson_solve: periodic Poisson problem -L_h phi = P g, sum(phi) = 0
// (Section 3.3 Poisson equation, well-posed for a neutral cell; Section 4:
// zero-integral convention, warm starts).
//
// Forms:
//  * plain FP64 CG;
//  * FP32 stencil + FP32 CG inside FP64 residual refinement: the outer loop
//    forms the true residual with the FP64 stencil, removes its mean in FP64,
//    scales it to unit norm, solves A d = r_hat in FP32 to a loose tolerance
//    (dot products accumulated in FP64) and adds ||r|| d to the FP64 iterate;
//  * learned: see poisson_learned.hip.
#include <algorithm>
#include <cmath>

#include "poisson.hpp"

namespace ofdft {

template <typename T>
int cg_k1(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, const T *r, const T *p_old,
          T *p_new, T *Ap, CgState *st, const RedBuf &rb, hipStream_t s) {
    ProfScope ps(K_CG_STENCIL, (double)npoints(g) * sizeof(T) * 4, s);
    return launch_stencil<T>(g, c, LoadCgP<T>{r, p_old, st, 0},
                             EpiCgAp<T>{p_new, Ap, st, rb.partials, rb.counter, 0.0}, s);
}

template <typename T>
int residual_pass(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, const T *x,
                  const double *gp, T *r, double *totals, const RedBuf &rb, hipStream_t s) {
    ProfScope ps(K_RESIDUAL, (double)npoints(g) * (2 * sizeof(T) + 8), s);
    return launch_stencil<T>(g, c, LoadPlain<T>{x},
                             EpiResidual<T>{gp, r, totals, rb.partials, rb.counter, 0.0, 0.0}, s);
}

template int cg_k1<double>(const ofdft_grid &, const Coef<double> &, const double *, const double *,
                           double *, double *, CgState *, const RedBuf &, hipStream_t);
template int cg_k1<float>(const ofdft_grid &, const Coef<float> &, const float *, const float *,
                          float *, float *, CgState *, const RedBuf &, hipStream_t);
template int residual_pass<double>(const ofdft_grid &, const Coef<double> &, const double *,
                                   const double *, double *, double *, const RedBuf &, hipStream_t);

// ---- small vector kernels --------------------------------------------------
struct SumOp {           // totals {sum a, sum a^2}
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 8;
    const double *a;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const double v = a[i];
        acc[0] += v;
        acc[1] = ::fma(v, v, acc[1]);
    }
};

struct ShiftOp {         // out = a - mean (mean = totals[0] / n), totals' {., sum out^2}
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 16;
    const double *a;
    double *out;
    const double *totals;
    double inv_n, mean;
    __device__ bool skip() const { return false; }
    __device__ void prepare() { mean = totals[0] * inv_n; }
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const double v = a[i] - mean;
        out[i] = v;
        acc[0] += v;
        acc[1] = ::fma(v, v, acc[1]);
    }
};

struct CastScaleOp {     // r32 = (r - mean) * inv_norm, d32 = 0, totals {., sum r32^2}
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 16;
    const double *r;
    float *r32;
    float *d32;
    const double *totals;      // {sum r, sum r^2}
    double inv_n, mean, scale;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {
        mean = totals[0] * inv_n;
        const double nrm2 = fmax(totals[1] - totals[0] * mean, 0.0);
        scale = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    }
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const float v = (float)((r[i] - mean) * scale);
        r32[i] = v;
        d32[i] = 0.0f;
        acc[0] += (double)v;
        acc[1] = ::fma((double)v, (double)v, acc[1]);
    }
};

struct AddScaledOp {     // x += ||r|| d32   (||r|| from the residual totals)
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 20;
    double *x;
    const float *d32;
    const double *totals;
    double inv_n, nrm;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {
        const double mean = totals[0] * inv_n;
        nrm = sqrt(fmax(totals[1] - totals[0] * mean, 0.0));
    }
    __device__ void operator()(int64_t i, double (&)[1]) const { x[i] = ::fma(nrm, (double)d32[i], x[i]); }
};

// Poisson right-hand side from a density and the nuclear charge (Section 3.3,
// Poisson equation: -(1/4 pi) Lap phi = rho + b): g = 4 pi (rho + b); totals {sum g}.
struct RhsSumOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24;
    const double *rho, *b;
    double *g;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        const double v = 4.0 * 3.14159265358979323846 * (rho[i] + b[i]);
        g[i] = v;
        acc[0] += v;
    }
};

struct InitCgFin {       // set rr, tol2 from totals and arm the solver
    CgState *st;
    double tol_rel2;
    int maxit;
    __device__ void operator()(const double (&t)[2]) const {
        st->rr = t[1];
        st->tol2 = tol_rel2 * t[1];
        st->iter = 0;
        st->first = 1;
        st->beta = 0.0;
        st->maxit = maxit;
        st->done = isfinite(t[1]) ? (t[1] > 0.0 ? CG_RUNNING : CG_CONVERGED) : CG_NONFINITE;
    }
};

// Enqueue `count` (even) CG iterations; the p buffers return to their roles.
template <typename T>
static int cg_block(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, T *x, T *r, T *pA, T *pB,
                    T *Ap, CgState *st, const RedBuf &rb, hipStream_t s, int count) {
    const int64_t n = npoints(g);
    T *p_old = pA, *p_new = pB;
    for (int k = 0; k < count; ++k) {
        OFDFT_TRY(cg_k1<T>(g, c, r, p_old, p_new, Ap, st, rb, s));
        CgUpdate<T> up{x, r, p_new, Ap, st, 0};
        OFDFT_TRY((launch_reduce<1>(n, up, CgUpdateFin{st}, rb, s)));
        std::swap(p_old, p_new);
    }
    return OFDFT_OK;
}

// A captured block of kGraphIters iterations for one set of buffers.
constexpr int kGraphIters = 16;
struct CgGraph {
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    const void *key[6] = {};
};

static void graph_release(CgGraph &gr) {
    if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
    if (gr.cap) (void)hipStreamDestroy(gr.cap);
    gr = CgGraph{};
}

template <typename T>
static int graph_get(CgGraph &gr, const ofdft_grid &g, const Coef<typename VT<T>::S> &c, T *x, T *r,
                     T *pA, T *pB, T *Ap, CgState *st, const RedBuf &rb) {
    const void *key[6] = {x, r, pA, pB, Ap, st};
    bool same = gr.exec != nullptr;
    for (int i = 0; i < 6 && same; ++i) same = gr.key[i] == key[i];
    if (same) return OFDFT_OK;
    if (gr.exec) {
        (void)hipGraphExecDestroy(gr.exec);
        gr.exec = nullptr;
    }
    if (!gr.cap) OFDFT_CHECK_HIP(hipStreamCreateWithFlags(&gr.cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    OFDFT_CHECK_HIP(hipStreamBeginCapture(gr.cap, hipStreamCaptureModeThreadLocal));
    const int rc = cg_block<T>(g, c, x, r, pA, pB, Ap, st, rb, gr.cap, kGraphIters);
    const hipError_t e = hipStreamEndCapture(gr.cap, &graph);
    if (rc != OFDFT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    OFDFT_CHECK_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&gr.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    OFDFT_CHECK_HIP(ei);
    for (int i = 0; i < 6; ++i) gr.key[i] = key[i];
    return OFDFT_OK;
}

// Per-iteration algorithmic bytes, to account replayed blocks.
template <typename T>
static void account_block(const ofdft_grid &g, int iters) {
    const double n = (double)npoints(g);
    prof_add(K_CG_STENCIL, n * sizeof(T) * 4 * iters, iters);
    prof_add(K_CG_UPDATE, n * sizeof(T) * 6 * iters, iters);
}

template <typename T>
int cg_iterate(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, T *x, T *r, T *pA, T *pB,
               T *Ap, CgState *st, CgState *st_host, const RedBuf &rb, hipStream_t s, int &iters,
               int &done, CgGraph *graph) {
    // Captured blocks replace per-kernel launches unless launches are being
    // timed individually.
    const bool use_graph = graph && !prof_timed(K_CG_STENCIL) && !prof_timed(K_CG_UPDATE);
    int chunk = 8;
    for (;;) {
        if (use_graph) {
            OFDFT_TRY(graph_get<T>(*graph, g, c, x, r, pA, pB, Ap, st, rb));
            const int reps = std::max(1, chunk / kGraphIters);
            for (int k = 0; k < reps; ++k) OFDFT_CHECK_HIP(hipGraphLaunch(graph->exec, s));
            account_block<T>(g, reps * kGraphIters);
        } else {
            OFDFT_TRY(cg_block<T>(g, c, x, r, pA, pB, Ap, st, rb, s, chunk));
        }
        OFDFT_CHECK_HIP(hipMemcpyAsync(st_host, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        OFDFT_CHECK_HIP(hipStreamSynchronize(s));
        if (st_host->done != CG_RUNNING) break;
        chunk = std::min(chunk * 2, 128);
    }
    iters = st_host->iter;
    done = st_host->done;
    return OFDFT_OK;
}

template int cg_iterate<double>(const ofdft_grid &, const Coef<double> &, double *, double *,
                                double *, double *, double *, CgState *, CgState *,
                                const RedBuf &, hipStream_t, int &, int &, CgGraph *);
template int cg_iterate<float>(const ofdft_grid &, const Coef<float> &, float *, float *, float *,
                               float *, float *, CgState *, CgState *, const RedBuf &,
                               hipStream_t, int &, int &, CgGraph *);

int status_from_done(int done) {
    switch (done) {
        case CG_CONVERGED: return OFDFT_OK;
        case CG_BREAKDOWN: return OFDFT_BREAKDOWN;
        case CG_NONFINITE: return OFDFT_NONFINITE;
        default: return OFDFT_NOT_CONVERGED;
    }
}

// ---- solver context ----------------------------------------------------------
int poisson_alloc(ofdft_poisson *s) {
    const int64_t n = npoints(s->g);
    const size_t b8 = sizeof(double) * n, b4 = sizeof(float) * n;
    OFDFT_CHECK_HIP(hipMalloc(&s->gp, b8));
    OFDFT_CHECK_HIP(hipMalloc(&s->r, b8));
    OFDFT_CHECK_HIP(hipMalloc(&s->pA, b8));
    OFDFT_CHECK_HIP(hipMalloc(&s->pB, b8));
    OFDFT_CHECK_HIP(hipMalloc(&s->Ap, b8));
    if (s->mode == OFDFT_REFINED_F32 || s->mode == OFDFT_LEARNED_REFINED) {
        OFDFT_CHECK_HIP(hipMalloc(&s->r32, b4));
        OFDFT_CHECK_HIP(hipMalloc(&s->d32, b4));
        OFDFT_CHECK_HIP(hipMalloc(&s->qA, b4));
        OFDFT_CHECK_HIP(hipMalloc(&s->qB, b4));
        OFDFT_CHECK_HIP(hipMalloc(&s->Aq, b4));
    }
    OFDFT_CHECK_HIP(hipMalloc(&s->st, sizeof(CgState)));
    OFDFT_CHECK_HIP(hipMemset(s->st, 0, sizeof(CgState)));
    OFDFT_CHECK_HIP(hipHostMalloc(&s->st_host, sizeof(CgState), hipHostMallocDefault));
    OFDFT_CHECK_HIP(hipMalloc(&s->totals, sizeof(double) * 16));
    OFDFT_CHECK_HIP(hipHostMalloc(&s->totals_host, sizeof(double) * 16, hipHostMallocDefault));
    OFDFT_TRY(redbuf_alloc(s->rb));
    OFDFT_CHECK_HIP(hipEventCreate(&s->ev0));
    OFDFT_CHECK_HIP(hipEventCreate(&s->ev1));
    s->graph64 = new CgGraph();
    s->graph32 = new CgGraph();
    return OFDFT_OK;
}

void poisson_free(ofdft_poisson *s) {
    if (s->mggraph) (void)hipGraphExecDestroy(s->mggraph);
    if (s->mgcap) (void)hipStreamDestroy(s->mgcap);
    if (s->pdev) (void)hipFree(s->pdev);
    if (s->pdev_h) (void)hipHostFree(s->pdev_h);
    s->mggraph = nullptr;
    s->mgcap = nullptr;
    s->pdev = s->pdev_h = nullptr;
    if (s->graph64) {
        graph_release(*s->graph64);
        delete s->graph64;
    }
    if (s->graph32) {
        graph_release(*s->graph32);
        delete s->graph32;
    }
    if (s->mg) {
        mg_free(*s->mg);
        delete s->mg;
    }
    void *dev[] = {s->gp, s->r, s->pA, s->pB, s->Ap, s->r32, s->d32, s->qA, s->qB, s->Aq, s->st,
                   s->totals, s->z, s->xbest};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    if (s->st_host) (void)hipHostFree(s->st_host);
    if (s->totals_host) (void)hipHostFree(s->totals_host);
    redbuf_free(s->rb);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
}

// Project the right-hand side: gp = g - mean(g); totals[2..3] = {sum gp, ||gp||^2}.
int project_rhs(ofdft_poisson *s, const double *rhs, hipStream_t st) {
    const int64_t n = npoints(s->g);
    OFDFT_TRY((launch_reduce<2>(n, SumOp{rhs}, StoreTotals<2>{s->totals}, s->rb, st)));
    ShiftOp sh{rhs, s->gp, s->totals, 1.0 / (double)n, 0.0};
    OFDFT_TRY((launch_reduce<2>(n, sh, StoreTotals<2>{s->totals + 2}, s->rb, st)));
    return OFDFT_OK;
}

// x <- x - mean(x), then the true FP64 residual of the projected system;
// totals[4..5] = residual {sum r, sum r^2}.
int finalize_solution(ofdft_poisson *s, double *x, hipStream_t st) {
    const int64_t n = npoints(s->g);
    OFDFT_TRY((launch_reduce<2>(n, SumOp{x}, StoreTotals<2>{s->totals + 6}, s->rb, st)));
    ShiftOp sh{x, x, s->totals + 6, 1.0 / (double)n, 0.0};
    OFDFT_TRY((launch_reduce<2>(n, sh, NoFin{}, s->rb, st)));
    OFDFT_TRY(residual_pass<double>(s->g, s->coef, x, s->gp, s->r, s->totals + 4, s->rb, st));
    return OFDFT_OK;
}

int solve_plain(ofdft_poisson *s, double *x, double rel_tol, int max_iter,
                ofdft_solve_stats &stats, hipStream_t st) {
    const int64_t n = npoints(s->g);
    OFDFT_TRY(residual_pass<double>(s->g, s->coef, x, s->gp, s->r, s->totals + 4, s->rb, st));
    // arm: rr = ||r||^2, tol2 = rel_tol^2 ||P g||^2
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->totals_host, s->totals, sizeof(double) * 8,
                                   hipMemcpyDeviceToHost, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    const double g2 = s->totals_host[3], r2 = s->totals_host[5];
    CgState &init = *s->st_host;
    init = CgState{};
    init.rr = r2;
    init.tol2 = rel_tol * rel_tol * g2;
    init.maxit = max_iter;
    init.first = 1;
    init.done = std::isfinite(r2) ? (r2 <= init.tol2 ? CG_CONVERGED : CG_RUNNING) : CG_NONFINITE;
    if (max_iter <= 0 && init.done == CG_RUNNING) init.done = CG_MAXIT;
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->st, s->st_host, sizeof(CgState), hipMemcpyHostToDevice, st));
    int iters = 0, done = init.done;
    if (done == CG_RUNNING)
        OFDFT_TRY(cg_iterate<double>(s->g, s->coef, x, s->r, s->pA, s->pB, s->Ap, s->st, s->st_host,
                                     s->rb, st, iters, done, s->use_graphs ? s->graph64 : nullptr));
    stats.iters = iters;
    (void)n;
    return status_from_done(done);
}

int solve_refined(ofdft_poisson *s, double *x, double rel_tol, int max_iter,
                         ofdft_solve_stats &stats, hipStream_t st) {
    const int64_t n = npoints(s->g);
    // Each FP32 inner solve targets the reduction still needed (with margin),
    // bounded below by what FP32 CG reliably reaches and above so that every
    // outer step makes real progress.
    const double inner_min = s->inner_min, inner_max = s->inner_max;
    const int max_outer = 12;
    int total = 0, outer = 0, status = OFDFT_NOT_CONVERGED;
    for (; outer <= max_outer; ++outer) {
        OFDFT_TRY(residual_pass<double>(s->g, s->coef, x, s->gp, s->r, s->totals + 4, s->rb, st));
        OFDFT_CHECK_HIP(hipMemcpyAsync(s->totals_host, s->totals, sizeof(double) * 8,
                                       hipMemcpyDeviceToHost, st));
        OFDFT_CHECK_HIP(hipStreamSynchronize(st));
        const double g2 = s->totals_host[3];
        const double rs = s->totals_host[4], r2 = s->totals_host[5];
        const double rn2 = std::max(r2 - rs * rs / (double)n, 0.0);
        if (!std::isfinite(r2)) {
            status = OFDFT_NONFINITE;
            break;
        }
        if (rn2 <= rel_tol * rel_tol * g2) {
            status = OFDFT_OK;
            break;
        }
        if (outer == max_outer || total >= max_iter) break;
        const double rel = g2 > 0 ? std::sqrt(rn2 / g2) : 0.0;
        const double inner_tol = std::min(inner_max, std::max(inner_min, 0.3 * rel_tol / rel));
        // r_hat = (r - mean) / ||r - mean|| in FP32, d = 0
        CastScaleOp cs{s->r, s->r32, s->d32, s->totals + 4, 1.0 / (double)n, 0, 0};
        OFDFT_TRY((launch_reduce<2>(n, cs, InitCgFin{s->st, inner_tol * inner_tol, max_iter - total},
                                    s->rb, st)));
        int iters = 0, done = 0;
        OFDFT_TRY(cg_iterate<float>(s->g, s->coef32, s->d32, s->r32, s->qA, s->qB, s->Aq, s->st,
                                    s->st_host, s->rb, st, iters, done, s->use_graphs ? s->graph32 : nullptr));
        total += iters;
        if (done == CG_NONFINITE) {
            status = OFDFT_NONFINITE;
            break;
        }
        AddScaledOp ad{x, s->d32, s->totals + 4, 1.0 / (double)n, 0};
        OFDFT_TRY((launch_reduce<1>(n, ad, NoFin{}, s->rb, st)));
        if (done == CG_BREAKDOWN && iters == 0) {
            status = OFDFT_BREAKDOWN;
            break;
        }
    }
    stats.iters = total;
    stats.outer_iters = outer;
    return status;
}

int poisson_solve(ofdft_poisson *s, const double *rhs, double *x, double rel_tol, int max_iter,
                  ofdft_solve_stats &stats, hipStream_t st) {
    const int64_t n = npoints(s->g);
    OFDFT_TRY(project_rhs(s, rhs, st));
    int status;
    if (s->mode == OFDFT_REFINED_F32) status = solve_refined(s, x, rel_tol, max_iter, stats, st);
    else if (s->mode == OFDFT_LEARNED || s->mode == OFDFT_LEARNED_REFINED)
        status = poisson_solve_learned(s, x, rel_tol, max_iter, stats, st);
    else if (s->mode == OFDFT_MULTIGRID || s->mode == OFDFT_MULTIGRID_F64)
        status = poisson_solve_mg(s, x, rel_tol, max_iter, stats, st);
    else status = solve_plain(s, x, rel_tol, max_iter, stats, st);
    if (status < 0 && status != OFDFT_BREAKDOWN && status != OFDFT_NONFINITE) return status;
    OFDFT_TRY(finalize_solution(s, x, st));
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->totals_host, s->totals, sizeof(double) * 8,
                                   hipMemcpyDeviceToHost, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    const double g2 = s->totals_host[3];
    stats.removed_mean = s->totals_host[0] / (double)n;
    const double r2 = s->totals_host[5];
    stats.rel_res = g2 > 0 ? std::sqrt(r2 / g2) : 0.0;
    if (!std::isfinite(stats.rel_res)) status = OFDFT_NONFINITE;
    else if (status == OFDFT_OK && stats.rel_res > rel_tol) status = OFDFT_NOT_CONVERGED;
    else if (status == OFDFT_NOT_CONVERGED && stats.rel_res <= rel_tol) status = OFDFT_OK;
    return status;
}

}  // namespace ofdft

using namespace ofdft;

extern "C" int ofdft_poisson_create(const ofdft_grid *grid, int radius, int mode,
                                    ofdft_poisson **out) {
    OFDFT_TRY(check_grid(grid, radius));
    if (!out) {
        set_error("ofdft_poisson_create: out is NULL");
        return OFDFT_INVALID_ARG;
    }
    if (mode != OFDFT_PLAIN_F64 && mode != OFDFT_REFINED_F32 && mode != OFDFT_LEARNED &&
        mode != OFDFT_MULTIGRID && mode != OFDFT_MULTIGRID_F64 && mode != OFDFT_LEARNED_REFINED) {
        set_error("ofdft_poisson_create: unknown mode %d", mode);
        return OFDFT_INVALID_ARG;
    }
    ofdft_poisson *s = new (std::nothrow) ofdft_poisson();
    if (!s) return OFDFT_NO_MEMORY;
    s->g = *grid;
    s->radius = radius;
    s->mode = mode;
    s->coef = make_coef(*grid, radius);
    s->coef32 = to_float(s->coef);
    int st = poisson_alloc(s);
    if (st == OFDFT_OK && (mode == OFDFT_MULTIGRID || mode == OFDFT_MULTIGRID_F64)) {
        s->mg = new (std::nothrow) Multigrid();
        if (!s->mg) st = OFDFT_NO_MEMORY;
        else st = mg_create(*s->mg, *grid, 8, mode == OFDFT_MULTIGRID);
        if (st == OFDFT_OK && hipMalloc(&s->z, sizeof(double) * npoints(*grid)) != hipSuccess) {
            set_error("ofdft_poisson_create: out of device memory");
            st = OFDFT_NO_MEMORY;
        }
    }
    if (st != OFDFT_OK) {
        poisson_free(s);
        delete s;
        return st;
    }
    *out = s;
    return OFDFT_OK;
}

extern "C" int ofdft_poisson_destroy(ofdft_poisson *s) {
    if (!s) return OFDFT_OK;
    poisson_free(s);
    delete s;
    return OFDFT_OK;
}

// Bounds of the FP32 inner tolerance of the refined form (defaults 1e-5, 1e-1).
extern "C" int ofdft_poisson_set_refinement(ofdft_poisson *s, double inner_min, double inner_max) {
    if (!s || !(inner_min > 0) || !(inner_max >= inner_min) || !(inner_max < 1)) {
        set_error("ofdft_poisson_set_refinement: need 0 < inner_min <= inner_max < 1");
        return OFDFT_INVALID_ARG;
    }
    s->inner_min = inner_min;
    s->inner_max = inner_max;
    return OFDFT_OK;
}

// g = 4 pi (rho + b) with its mean removed (net-charge projection, FP64
// sums); the removed mean is returned.  Synchronises the stream.
extern "C" int ofdft_poisson_rhs(ofdft_poisson *s, const double *rho, const double *b, double *g,
                                 double *removed_mean, void *stream) {
    if (!s || !rho || !b || !g) {
        set_error("ofdft_poisson_rhs: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = npoints(s->g);
    OFDFT_TRY((launch_reduce<1>(n, RhsSumOp{rho, b, g}, StoreTotals<1>{s->totals + 8}, s->rb, st)));
    ShiftOp sh{g, g, s->totals + 8, 1.0 / (double)n, 0.0};
    OFDFT_TRY((launch_reduce<2>(n, sh, NoFin{}, s->rb, st)));
    double t = 0.0;
    OFDFT_CHECK_HIP(hipMemcpyAsync(&t, s->totals + 8, sizeof(double), hipMemcpyDeviceToHost, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    if (removed_mean) *removed_mean = t / (double)n;
    return std::isfinite(t) ? OFDFT_OK : OFDFT_NONFINITE;
}

// Enable (1, default) or disable (0) captured iteration blocks for a solver.
extern "C" int ofdft_poisson_set_graphs(ofdft_poisson *s, int enable) {
    if (!s) return OFDFT_INVALID_ARG;
    s->use_graphs = enable != 0;
    return OFDFT_OK;
}

extern "C" int cg_poisson_solve(ofdft_poisson *s, const double *rhs, double *x, double rel_tol,
                                int max_iter, ofdft_solve_stats *stats, void *stream) {
    if (!s || !rhs || !x) {
        set_error("cg_poisson_solve: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    if (!(rel_tol > 0) || max_iter < 0) {
        set_error("cg_poisson_solve: rel_tol must be > 0 and max_iter >= 0");
        return OFDFT_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    ofdft_solve_stats local{};
    OFDFT_CHECK_HIP(hipEventRecord(s->ev0, st));
    int status = poisson_solve(s, rhs, x, rel_tol, max_iter, local, st);
    OFDFT_CHECK_HIP(hipEventRecord(s->ev1, st));
    OFDFT_CHECK_HIP(hipEventSynchronize(s->ev1));
    float ms = 0;
    OFDFT_CHECK_HIP(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    local.seconds = ms * 1e-3;
    local.status = status;
    if (stats) *stats = local;
    if (status < 0 && status != OFDFT_HIP_ERROR) set_error("cg_poisson_solve: status %d", status);
    return status;
}
