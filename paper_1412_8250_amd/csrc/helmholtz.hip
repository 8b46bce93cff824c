// cg_helmholtz_solve_batched: (-L_h + kappa_j) u_j = f_j for many systems on
// uneven grids (Section 3.1, Helmholtz equations multiplied by (2 kF)^2).
//
// The matrix -L_h + kappa is complex symmetric (L_h is real symmetric), so the
// solver is COCG: conjugate gradients with the unconjugated bilinear form
// x^T y.  The default schedule is the stepped one (helmholtz_stepped.hip:
// one launch per COCG phase over all systems, replayed from a HIP graph).
// The persistent schedule, selected with a group size, runs all systems in
// ONE cooperative launch:
//  * the grid is split into groups of P workgroups; a group takes systems from
//    a device work queue ordered longest-first (LPT: estimated iterations
//    times points) and runs a whole COCG solve on it;
//  * within a group the P workgroups share the system's stencil tiles and
//    vector slices and meet at a global-memory barrier twice per iteration
//    (after p.Ap and after r.r); every workgroup combines the P partial sums
//    in the same fixed order, so all take identical decisions and the result is
//    bitwise repeatable;
//  * barrier waits are bounded (spin limit): on expiry the kernel raises an
//    abort flag and every workgroup leaves.
// Complex64 runs COCG in complex64 inside complex128 residual refinement: the
// host loop forms r = f - A x in complex128, scales it to unit norm, solves in
// complex64 to 1e-4 and adds ||r|| d to x.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "helmholtz.hpp"

namespace ofdft {

constexpr int kMaxGroupP = 1024;
constexpr long kSpinLimit = 1L << 22;



struct HState {
    double rr_re, rr_im, al_re, al_im, be_re, be_im, tol2, rnorm2, fnorm2;
    int iter, done, maxit, first;
};

struct GroupCtl {
    unsigned int count, gen;
    int sys, pad;
};

// Bounded global-memory barrier for the P workgroups of one group.  Returns
// false (in every thread) if the wait expired or the abort flag is raised.
__device__ inline bool group_barrier(GroupCtl *c, int P, int *abort_flag, int *s_flag) {
    __syncthreads();
    const bool leader = threadIdx.x == 0 && threadIdx.y == 0;
    if (leader) {
        int ok = 1;
        if (P > 1) {
            __threadfence();
            const unsigned int gen = __hip_atomic_load(&c->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned int arrived = atomicAdd(&c->count, 1u);
            if (arrived == (unsigned int)P - 1) {
                __hip_atomic_store(&c->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&c->gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                long spins = 0;
                while (__hip_atomic_load(&c->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > kSpinLimit ||
                        __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        atomicExch(abort_flag, 1);
                        ok = 0;
                        break;
                    }
                }
            }
            __threadfence();
        }
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        *s_flag = ok;
    }
    __syncthreads();
    return *s_flag != 0;
}

// ---- loaders / epilogues of the stencil phases -------------------------------
template <typename T>
struct LoadX {
    GPtr<T> x;
    __device__ void prepare() {}
    __device__ T operator()(int64_t i) const { return x[i]; }
};

template <typename T>
struct LoadCocgP {       // r + beta p_old (complex beta); first iteration: p_old = r, beta = 0
    GPtr<T> r, p_old;
    T beta;
    __device__ void prepare() {}
    __device__ T operator()(int64_t i) const { return cfma(beta, p_old[i], r[i]); }
};

template <typename T>
struct EpiInitRes {      // r = f - (-L x + kappa x); acc {r.r re, r.r im, |r|^2, |f|^2}
    GPtr<T> f, r;
    T kappa;
    double acc[4];
    T fv[4];
    __device__ void pre(int q, int64_t i) { fv[q] = f[i]; }
    __device__ void point(int q, int64_t i, T c, T s) {
        T ax = cfma(kappa, c, T{-s.x, -s.y});
        const T fi = fv[q];
        T rv{fi.x - ax.x, fi.y - ax.y};
        r.st(i, rv);
        const double a = rv.x, b = rv.y;
        acc[0] += a * a - b * b;
        acc[1] += 2.0 * a * b;
        acc[2] += a * a + b * b;
        acc[3] += (double)fi.x * fi.x + (double)fi.y * fi.y;
    }
};

template <typename T>
struct EpiCocgAp {       // p_new = centre, Ap = -L p + kappa p; acc {p.Ap re, im}
    GPtr<T> p_out, Ap;
    T kappa;
    double acc[4];
    __device__ void pre(int, int64_t) {}
    __device__ void point(int, int64_t i, T c, T s) {
        T a = cfma(kappa, c, T{-s.x, -s.y});
        p_out.st(i, c);
        Ap.st(i, a);
        acc[0] += (double)c.x * a.x - (double)c.y * a.y;
        acc[1] += (double)c.x * a.y + (double)c.y * a.x;
    }
};

// Sum the P partial rows of a group into out[0..3], by the first wave: lane q
// accumulates rows q, q+64, ... then a fixed shuffle tree combines the lanes,
// so the result does not depend on timing.
__device__ inline void combine(const double (*part)[4], int P, double *out) {
    const int lane = threadIdx.x + threadIdx.y * blockDim.x;
    if (lane >= 64) return;
    double a[4] = {0, 0, 0, 0};
    for (int q = lane; q < P; q += 64)
        for (int k = 0; k < 4; ++k)
            a[k] += __hip_atomic_load(&part[q][k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int k = 0; k < 4; ++k) {
        const double t = wave_sum(a[k]);
        if (lane == 0) out[k] = t;
    }
}

template <typename T, int TX, int TYT, int RY>
struct CocgShape {
    using TS = TileShape<TX, TYT, RY>;
};

template <typename T, int TX, int TYT, int RY, class Load, class Epi>
__device__ inline void stencil_units(const HSys &s, const Coef<typename VT<T>::S> &w, const Load &ld,
                                     Epi &ep, int rank, int P, T *lds) {
    // two ring buffers: this kernel also holds the COCG scalars in registers
    for (int u = rank; u < s.nunits; u += P)
        stencil_tile<T, TX, TYT, RY, Load, Epi, StencilLds<T, TX, TYT, RY>::kLead, 2>(s.tg, w, ld, ep, u, lds);
}


// Block-reduce acc[4] and publish it in part[rank]; leader only writes.
__device__ inline void publish4(double (&acc)[4], double (*part)[4], int rank, double *scratch) {
    block_sum<4>(acc, scratch);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        for (int k = 0; k < 4; ++k)
            __hip_atomic_store(&part[rank][k], acc[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int TX, int TYT, int RY>
__device__ void cocg_solve_one(const HSys &s, HState *st, GroupCtl *c, double (*partA)[4],
                               double (*partB)[4], int P, int rank, T *lds, double *scratch,
                               double *bcast, int *abort_flag, int *s_flag, double tol) {
    using CT = CX<T>;
    const bool leader = threadIdx.x == 0 && threadIdx.y == 0;
    const int tid = threadIdx.y * TX + threadIdx.x;
    constexpr int NT = TX * TYT;
    const Coef<typename VT<T>::S> &w = coef_of<T>(s);
    const T kappa = CT::mk(s.kre, s.kim);
    const GPtr<T> x(s.x), r(s.r), Ap(s.Ap), f(s.f);
    const int maxit = st->maxit;

    // initial residual r = f - A x
    {
        LoadX<T> ld{x};
        EpiInitRes<T> ep{f, r, kappa, {0, 0, 0, 0}};
        stencil_units<T, TX, TYT, RY>(s, w, ld, ep, rank, P, lds);
        publish4(ep.acc, partB, rank, scratch);
    }
    if (!group_barrier(c, P, abort_flag, s_flag)) return;
    combine(partB, P, bcast);
    __syncthreads();
    double rr_re = bcast[0], rr_im = bcast[1], rn2 = bcast[2];
    const double fn2 = bcast[3];
    const double tol2 = tol * tol * fn2;
    int done = !isfinite(rn2) ? H_NONFINITE : (rn2 <= tol2 ? H_CONVERGED : H_RUNNING);
    if (done == H_RUNNING && maxit <= 0) done = H_MAXIT;
    int iter = 0;
    double be_re = 0.0, be_im = 0.0;
    GPtr<T> p_old(s.pA), p_new(s.pB);
    __syncthreads();

    while (done == H_RUNNING) {
        // Phase A: p = r + beta p_old; Ap = (-L + kappa) p; p.Ap
        {
            LoadCocgP<T> ld{r, iter == 0 ? r : p_old, CT::mk(iter == 0 ? 0.0 : be_re, iter == 0 ? 0.0 : be_im)};
            EpiCocgAp<T> ep{p_new, Ap, kappa, {0, 0, 0, 0}};
            stencil_units<T, TX, TYT, RY>(s, w, ld, ep, rank, P, lds);
            publish4(ep.acc, partA, rank, scratch);
        }
        if (!group_barrier(c, P, abort_flag, s_flag)) return;
        combine(partA, P, bcast);
        __syncthreads();
        const double pa_re = bcast[0], pa_im = bcast[1];
        const double den = pa_re * pa_re + pa_im * pa_im;
        __syncthreads();
        if (!isfinite(den)) { done = H_NONFINITE; break; }
        if (den == 0.0) { done = H_BREAKDOWN; break; }
        const double al_re = (rr_re * pa_re + rr_im * pa_im) / den;
        const double al_im = (rr_im * pa_re - rr_re * pa_im) / den;

        // Phase B: x += alpha p; r -= alpha Ap; r.r and |r|^2
        {
            const T al = CT::mk(al_re, al_im), nal = CT::mk(-al_re, -al_im);
            double acc[4] = {0, 0, 0, 0};
            const int64_t stride = (int64_t)P * NT;
            for (int64_t i = (int64_t)rank * NT + tid; i < s.n; i += stride) {
                x.st(i, cfma(al, p_new[i], x[i]));
                const T rv = cfma(nal, Ap[i], r[i]);
                r.st(i, rv);
                const double a = rv.x, b = rv.y;
                acc[0] += a * a - b * b;
                acc[1] += 2.0 * a * b;
                acc[2] += a * a + b * b;
            }
            publish4(acc, partB, rank, scratch);
        }
        if (!group_barrier(c, P, abort_flag, s_flag)) return;
        combine(partB, P, bcast);
        __syncthreads();
        const double nr_re = bcast[0], nr_im = bcast[1];
        rn2 = bcast[2];
        __syncthreads();
        const double d2 = rr_re * rr_re + rr_im * rr_im;
        be_re = (nr_re * rr_re + nr_im * rr_im) / d2;
        be_im = (nr_im * rr_re - nr_re * rr_im) / d2;
        rr_re = nr_re;
        rr_im = nr_im;
        ++iter;
        GPtr<T> tmp = p_old;
        p_old = p_new;
        p_new = tmp;
        if (!isfinite(rn2)) done = H_NONFINITE;
        else if (rn2 <= tol2) done = H_CONVERGED;
        else if (rr_re * rr_re + rr_im * rr_im <= 1e-60 * rn2 * rn2) done = H_BREAKDOWN;
        else if (iter >= maxit) done = H_MAXIT;
    }
    if (leader && rank == 0) {
        st->iter = iter;
        st->done = done;
        st->rnorm2 = rn2;
        st->fnorm2 = fn2;
        st->tol2 = tol2;
    }
}

template <typename T, int TX, int TYT, int RY>
__global__ void __launch_bounds__(TX * TYT)
cocg_persistent(const HSys *sys, HState *st, const int *order, int nsys, GroupCtl *ctl,
                double (*part)[4], int P, unsigned int *queue, int *abort_flag, double tol) {
    using TS = TileShape<TX, TYT, RY>;
    __shared__ T lds[StencilLds<T, TX, TYT, RY>::kElems];
    __shared__ double scratch[4 * (TX * TYT / 64)];
    __shared__ double bcast[4];
    __shared__ int s_flag, s_sys;
    const int group = blockIdx.x / P, rank = blockIdx.x % P;
    GroupCtl *c = ctl + group;
    // partial-sum rows of this group: [A: gridDim rows][B: gridDim rows]
    double(*partA)[4] = part + (size_t)group * P;
    double(*partB)[4] = part + gridDim.x + (size_t)group * P;
    const bool leader = threadIdx.x == 0 && threadIdx.y == 0;
    for (;;) {
        if (rank == 0 && leader) {
            const unsigned int q = atomicAdd(queue, 1u);
            __hip_atomic_store(&c->sys, q < (unsigned int)nsys ? order[q] : -1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!group_barrier(c, P, abort_flag, &s_flag)) return;
        if (leader) s_sys = __hip_atomic_load(&c->sys, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int sidx = s_sys;
        __syncthreads();
        if (sidx < 0) return;
        cocg_solve_one<T, TX, TYT, RY>(sys[sidx], st + sidx, c, partA, partB, P, rank, lds, scratch,
                                       bcast, abort_flag, &s_flag, tol);
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    }
}

// ---- per-system helper kernels (refinement and final residual) ---------------
template <typename T>
struct EpiHRes {         // r = f - A x in complex128; totals {|r|^2, |f|^2}
    const double2 *__restrict__ f;
    double2 *__restrict__ r;
    double2 kappa;
    double *totals;
    double *partials;
    unsigned int *counter;
    double acc0, acc1;
    double2 fv[4];
    __device__ bool skip() const { return false; }
    __device__ void pre(int q, int64_t i) { fv[q] = f[i]; }
    __device__ void point(int q, int64_t i, double2 c, double2 s) {
        double2 ax = cfma(kappa, c, double2{-s.x, -s.y});
        const double2 fi = fv[q];
        double2 rv{fi.x - ax.x, fi.y - ax.y};
        if (r) r[i] = rv;
        acc0 += rv.x * rv.x + rv.y * rv.y;
        acc1 += fi.x * fi.x + fi.y * fi.y;
    }
    __device__ void finish(int block, int nblocks, double *scratch) {
        double v[2] = {acc0, acc1};
        block_sum<2>(v, scratch);
        double t[2];
        if (reduce_grid<2>(v, partials, nblocks, block, counter, scratch, t)) {
            totals[0] = t[0];
            totals[1] = t[1];
        }
    }
};

struct CastC64 {         // f32 = r / ||r||, x32 = 0
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 32;
    const double2 *r;
    float2 *f32;
    float2 *x32;
    const double *totals;
    double scale;
    __device__ bool skip() const { return false; }
    __device__ void prepare() { scale = totals[0] > 0 ? 1.0 / sqrt(totals[0]) : 0.0; }
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double2 v = r[i];
        f32[i] = make_float2((float)(v.x * scale), (float)(v.y * scale));
        x32[i] = make_float2(0.f, 0.f);
    }
};

struct AddC64 {          // x += ||r|| x32
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 40;
    double2 *x;
    const float2 *x32;
    const double *totals;
    double nrm;
    __device__ bool skip() const { return false; }
    __device__ void prepare() { nrm = sqrt(totals[0]); }
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const float2 d = x32[i];
        x[i] = make_double2(::fma(nrm, (double)d.x, x[i].x), ::fma(nrm, (double)d.y, x[i].y));
    }
};

}  // namespace ofdft

using namespace ofdft;


namespace {

int zlen_for_units(const ofdft_grid &g, int shape) { return zlen_for_blocks(g, shape, 8); }

double est_cost(const ofdft_grid &g, double kre, double kim) {
    double lmax = 0.0;
    const double h[3] = {g.hx, g.hy, g.hz};
    for (double hh : h) lmax += 4.0 * 7.1 / (hh * hh) / 4.0;   // |symbol| at pi, 12th order
    const double mag = std::hypot(kre, kim);
    const double dist = kre >= 0 ? mag : std::fabs(kim) + 1e-3;
    return (double)npoints(g) * std::sqrt((lmax + mag) / dist);
}

template <typename T, int TX, int TYT, int RY>
int launch_persistent(ofdft_batch *b, int P, int nsys_run, double tol, hipStream_t s) {
    auto kern = cocg_persistent<T, TX, TYT, RY>;
    int dev = 0;
    OFDFT_CHECK_HIP(hipGetDevice(&dev));
    int cus = 0, coop = 0;
    OFDFT_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    OFDFT_CHECK_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    int per_cu = 0;
    OFDFT_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, TX * TYT, 0));
    if (per_cu < 1 || !coop) {
        set_error("persistent COCG kernel cannot be made resident (occupancy %d, coop %d)", per_cu, coop);
        return OFDFT_HIP_ERROR;
    }
    const int resident = std::min(per_cu * cus, b->groups_cap);
    if (P <= 0) {
        // few systems: spread the whole GPU over them; many: one or two workgroups each
        P = std::max(1, resident / std::max(1, nsys_run));
        if (nsys_run >= resident / 2) P = std::max(1, resident / nsys_run);
    }
    P = std::min(P, resident);
    int groups = resident / P;
    groups = std::min(groups, std::max(1, nsys_run));
    const int blocks = groups * P;
    OFDFT_CHECK_HIP(hipMemsetAsync(b->d_ctl, 0, sizeof(GroupCtl) * groups, s));
    OFDFT_CHECK_HIP(hipMemsetAsync(b->d_queue, 0, sizeof(unsigned int), s));
    OFDFT_CHECK_HIP(hipMemsetAsync(b->d_abort, 0, sizeof(int), s));
    const HSys *sys = b->d_sys;
    HState *st = b->d_st;
    const int *order = b->d_order;
    GroupCtl *ctl = b->d_ctl;
    double(*part)[4] = b->d_part;
    unsigned int *queue = b->d_queue;
    int *abort_flag = b->d_abort;
    void *args[] = {(void *)&sys, (void *)&st, (void *)&order, (void *)&nsys_run, (void *)&ctl,
                    (void *)&part, (void *)&P, (void *)&queue, (void *)&abort_flag, (void *)&tol};
    ProfScope ps(K_COCG, 0.0, s);     // bytes are added after the run from the iteration counts
    OFDFT_CHECK_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3(blocks), dim3(TX, TYT), args,
                                               0, s));
    return OFDFT_OK;
}

template <typename T>
int run_persistent(ofdft_batch *b, int shape, int P, int nsys_run, double tol, hipStream_t s) {
    return dispatch_cocg_shape<T>(shape, [&](auto sh) {
        using S = decltype(sh);
        return launch_persistent<T, S::TX, S::TYT, S::RY>(b, P, nsys_run, tol, s);
    });
}

int residual_c128(ofdft_batch *b, int j, const double2 *f, const double2 *x, double2 *r,
                  double kre, double kim, double *totals, hipStream_t s) {
    const ofdft_grid &g = b->grids[j];
    const Coef<double> c = make_coef(g, b->radius);
    TileGeom tg = make_tile_geom<64, 4, 2>(g, zlen_for_blocks(g, SHAPE_64x4x2, 512));
    LoadPlain<double2> ld{x};
    EpiHRes<double2> ep{f, r, make_double2(kre, kim), totals, b->rb.partials, b->rb.counter, 0.0, 0.0};
    ProfScope ps(K_RESIDUAL, (double)npoints(g) * (r ? 48 : 32), s);
    hipLaunchKernelGGL((stencil_kernel<double2, 64, 4, 2, LoadPlain<double2>, EpiHRes<double2>>),
                       dim3(tg.nblocks), dim3(64, 4), 0, s, tg, c, ld, ep);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

// Frees the preconditioner's buffers; the captured iteration graph holds
// their addresses, so it goes too (the caller has synchronised).
void precond_free(ofdft_batch *b) {
    if (b->step_graph) {
        (void)hipGraphExecDestroy(b->step_graph);
        b->step_graph = nullptr;
    }
    for (Multigrid *mg : b->mg_own) {
        mg_free(*mg);
        delete mg;
    }
    for (void *p : b->z)
        if (p) (void)hipFree(p);
    if (b->d_kap) (void)hipFree(b->d_kap);
    b->d_kap = nullptr;
    if (b->d_rtab) (void)hipFree(b->d_rtab);
    if (b->d_ztab) (void)hipFree(b->d_ztab);
    b->d_rtab = b->d_ztab = nullptr;
    b->mg_q.clear();
    b->mg_groups.clear();
    for (hipStream_t q : b->mg_lane) (void)hipStreamDestroy(q);
    for (hipEvent_t e : b->mg_join) (void)hipEventDestroy(e);
    if (b->mg_fork) (void)hipEventDestroy(b->mg_fork);
    b->mg_lane.clear();
    b->mg_join.clear();
    b->mg_fork = nullptr;
    b->mg_own.clear();
    b->mg_of.clear();
    b->z.clear();
    b->precond = OFDFT_PRECOND_NONE;
}

void batch_free(ofdft_batch *b) {
    stepped_free(b);
    precond_free(b);
    for (void *p : b->allocs)
        if (p) (void)hipFree(p);
    b->allocs.clear();
    redbuf_free(b->rb);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
}

template <typename P_>
int dalloc(ofdft_batch *b, P_ **p, size_t bytes) {
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
        set_error("ofdft_batch: out of device memory (%zu bytes)", bytes);
        return OFDFT_NO_MEMORY;
    }
    b->allocs.push_back(q);
    *p = (P_ *)q;
    return OFDFT_OK;
}

// Fill the device system table for one pass.  elem = complex element type of
// the inner solve; x/f pointers per system.
int upload_systems(ofdft_batch *b, const double *kappa, const std::vector<const void *> &f,
                   const std::vector<void *> &x, bool c64, int shape, bool stepped,
                   std::vector<HSys> &hs, hipStream_t s) {
    hs.assign(b->nsys, HSys{});
    for (int j = 0; j < b->nsys; ++j) {
        const ofdft_grid &g = b->grids[j];
        HSys &h = hs[j];
        h.nx = g.nx;
        h.ny = g.ny;
        h.nz = g.nz;
        const int eff = c64 ? cocg_shape<float2>(shape) : cocg_shape<double2>(shape);
        const int zl = stepped ? stepped_zlen(g, c64, eff, b->zplanes) : zlen_for_units(g, eff);
        dispatch_shape(eff, [&](auto sh) {
            using S = decltype(sh);
            h.tg = make_tile_geom<S::TX, S::TYT, S::RY>(g, zl);
            return 0;
        });
        h.nunits = h.tg.nblocks;
        h.n = npoints(g);
        h.coef = make_coef(g, b->radius);
        h.coef32 = to_float(h.coef);
        h.kre = kappa[2 * j];
        h.kim = kappa[2 * j + 1];
        h.x = x[j];
        h.f = f[j];
        h.z = b->precond ? b->z[j] : nullptr;
        if (c64) {
            h.r = b->r[j];
            h.pA = b->pA[j];
            h.pB = b->pB[j];
            h.Ap = b->Ap[j];
        } else {
            h.r = b->r[j];
            h.pA = b->pA[j];
            h.pB = b->pB[j];
            h.Ap = b->Ap[j];
        }
    }
    OFDFT_CHECK_HIP(hipMemcpyAsync(b->d_sys, hs.data(), sizeof(HSys) * b->nsys, hipMemcpyHostToDevice, s));
    OFDFT_CHECK_HIP(hipStreamSynchronize(s));
    return OFDFT_OK;
}

int default_shape(const ofdft_batch *b) {
    if (b->dtype == OFDFT_C64) return SHAPE_64x4x2;
    int small = 0;
    for (auto &g : b->grids) small += g.nx <= 40;
    return small * 2 > b->nsys ? SHAPE_32x8x2 : SHAPE_64x8x1;
}

}  // namespace

extern "C" int ofdft_batch_create(int nsys, const ofdft_grid *grids, int radius, ofdft_dtype dtype,
                                  ofdft_batch **out) {
    if (!out || nsys < 1 || !grids || (dtype != OFDFT_C128 && dtype != OFDFT_C64)) {
        set_error("ofdft_batch_create: need nsys >= 1, grids, dtype C128 or C64");
        return OFDFT_INVALID_ARG;
    }
    for (int j = 0; j < nsys; ++j) OFDFT_TRY(check_grid(&grids[j], radius));
    ofdft_batch *b = new (std::nothrow) ofdft_batch();
    if (!b) return OFDFT_NO_MEMORY;
    b->nsys = nsys;
    b->radius = radius;
    b->dtype = dtype;
    b->grids.assign(grids, grids + nsys);
    auto fail = [&](int st) {
        batch_free(b);
        delete b;
        return st;
    };
    const bool c64 = dtype == OFDFT_C64;
    const size_t e = c64 ? sizeof(float2) : sizeof(double2);
    b->r.resize(nsys);
    b->pA.resize(nsys);
    b->pB.resize(nsys);
    b->Ap.resize(nsys);
    b->r128.resize(nsys);
    b->f32.resize(nsys);
    b->x32.resize(nsys);
    for (int j = 0; j < nsys; ++j) {
        const size_t n = (size_t)npoints(grids[j]);
        int st = OFDFT_OK;
        if ((st = dalloc(b, &b->r[j], n * e)) || (st = dalloc(b, &b->pA[j], n * e)) ||
            (st = dalloc(b, &b->pB[j], n * e)) || (st = dalloc(b, &b->Ap[j], n * e)))
            return fail(st);
        if (c64) {
            if ((st = dalloc(b, &b->r128[j], n * sizeof(double2))) ||
                (st = dalloc(b, &b->f32[j], n * e)) || (st = dalloc(b, &b->x32[j], n * e)))
                return fail(st);
        }
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(OFDFT_HIP_ERROR);
    b->groups_cap = std::max(1, cus * 8);
    int st = OFDFT_OK;
    if ((st = dalloc(b, &b->d_sys, sizeof(HSys) * nsys)) ||
        (st = dalloc(b, &b->d_st, sizeof(HState) * nsys)) ||
        (st = dalloc(b, &b->d_order, sizeof(int) * nsys)) ||
        (st = dalloc(b, &b->d_ctl, sizeof(GroupCtl) * b->groups_cap)) ||
        (st = dalloc(b, &b->d_part, sizeof(double) * 4 * 2 * b->groups_cap)) ||
        (st = dalloc(b, &b->d_queue, 256)) || (st = dalloc(b, &b->d_abort, 256)) ||
        (st = dalloc(b, &b->d_totals, sizeof(double) * 2 * nsys)))
        return fail(st);
    if ((st = redbuf_alloc(b->rb))) return fail(st);
    if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess)
        return fail(OFDFT_HIP_ERROR);
    *out = b;
    return OFDFT_OK;
}

extern "C" int ofdft_batch_destroy(ofdft_batch *b) {
    if (!b) return OFDFT_OK;
    batch_free(b);
    delete b;
    return OFDFT_OK;
}

// Choose the launch configuration used by later solves (shape < 0: default).
extern "C" int ofdft_batch_set_config(ofdft_batch *b, int shape, int P) {
    if (!b || shape >= SHAPE_COUNT || P < 0 || P > kMaxGroupP) {
        set_error("ofdft_batch_set_config: bad shape %d or group size %d", shape, P);
        return OFDFT_INVALID_ARG;
    }
    b->shape = shape;
    b->P = P;
    return OFDFT_OK;
}

// Autotuner of a batch's schedule: times `iters` COCG iterations of the
// given systems (from copies of x; tolerance out of reach, so every
// candidate runs the same iterations) for each stepped tile shape and z-chunk
// target and, without a preconditioner, the persistent schedule with two
// group sizes, then keeps the fastest (the untuned configuration unless
// beaten by more than 2%).
extern "C" int ofdft_batch_tune(ofdft_batch *b, const double *kappa, const void *const *rhs,
                                const void *const *x, int iters, ofdft_tune_result *out, void *stream) {
    if (!b || !kappa || !rhs || !x || iters < 1 || iters > 10000) {
        set_error("ofdft_batch_tune: bad arguments (1 <= iters <= 10000)");
        return OFDFT_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int nsys = b->nsys;
    std::vector<void *> tmp(nsys, nullptr);
    auto release = [&]() {
        for (void *p : tmp)
            if (p) (void)hipFree(p);
    };
    for (int j = 0; j < nsys; ++j) {
        if (!x[j] || !rhs[j]) {
            release();
            set_error("ofdft_batch_tune: NULL array for system %d", j);
            return OFDFT_INVALID_ARG;
        }
        if (hipMalloc(&tmp[j], sizeof(double2) * npoints(b->grids[j])) != hipSuccess) {
            (void)hipGetLastError();
            release();
            set_error("ofdft_batch_tune: out of device memory");
            return OFDFT_NO_MEMORY;
        }
    }
    struct Cand {
        int shape, P, planes;
    };
    const bool c64 = b->dtype == OFDFT_C64;
    const Cand def{default_shape(b), 0, kStepPlanes};
    std::vector<Cand> cand;
    const std::vector<int> shapes = c64 ? std::vector<int>{SHAPE_64x4x2, SHAPE_64x4x4, SHAPE_32x8x2, SHAPE_64x8x2,
                                                           SHAPE_64x8x1}
                                        : std::vector<int>{SHAPE_64x8x1, SHAPE_64x4x2, SHAPE_32x8x2};
    for (int sh : shapes)
        for (int planes : {40, kStepPlanes, 160}) cand.push_back({sh, 0, planes});
    if (!b->precond)
        for (int P : {16, 64}) cand.push_back({def.shape, P, kStepPlanes});
    const int keep_shape = b->shape, keep_P = b->P, keep_planes = b->zplanes;
    std::vector<ofdft_solve_stats> st(nsys);
    double best = -1.0, def_ms = -1.0;
    Cand pick = def;
    int rc = OFDFT_OK;
    for (const Cand &k : cand) {
        b->shape = k.shape;
        b->P = k.P;
        b->zplanes = k.planes;
        double t = 0.0;
        for (int rep = 0; rep < 2 && rc >= 0; ++rep) {     // the first run captures graphs / lays out
            for (int j = 0; j < nsys && rc >= 0; ++j)
                if (hipMemcpyAsync(tmp[j], x[j], sizeof(double2) * npoints(b->grids[j]), hipMemcpyDeviceToDevice,
                                   s) != hipSuccess)
                    rc = OFDFT_HIP_ERROR;
            if (rc < 0) break;
            rc = cg_helmholtz_solve_batched(b, kappa, rhs, tmp.data(), 1e-300, iters, st.data(), stream);
            t = st[0].seconds * 1e3;
        }
        if (rc < 0) break;
        rc = OFDFT_OK;
        if (k.shape == def.shape && k.P == def.P && k.planes == def.planes) def_ms = t;
        if (best < 0.0 || t < best) {
            best = t;
            pick = k;
        }
    }
    release();
    if (rc < 0) {
        b->shape = keep_shape;
        b->P = keep_P;
        b->zplanes = keep_planes;
        return rc;
    }
    if (def_ms > 0.0 && best > 0.98 * def_ms) {
        pick = def;
        best = def_ms;
    }
    b->shape = pick.shape;
    b->P = pick.P;
    b->zplanes = pick.planes;
    if (out) {
        *out = ofdft_tune_result{};
        out->shape = pick.shape;
        out->zlen = pick.planes;
        out->group = pick.P;
        out->candidates = (int)cand.size();
        out->best_ms = best;
        out->default_ms = def_ms;
    }
    return OFDFT_OK;
}

extern "C" int ofdft_batch_set_preconditioner(ofdft_batch *b, int kind) {
    if (!b || (kind != OFDFT_PRECOND_NONE && kind != OFDFT_PRECOND_MULTIGRID &&
               kind != OFDFT_PRECOND_MULTIGRID_F64)) {
        set_error("ofdft_batch_set_preconditioner: unknown kind %d", kind);
        return OFDFT_INVALID_ARG;
    }
    if (kind == b->precond) return OFDFT_OK;
    if (b->precond != OFDFT_PRECOND_NONE && kind != OFDFT_PRECOND_NONE) {     // switch precision
        const int st = ofdft_batch_set_preconditioner(b, OFDFT_PRECOND_NONE);
        if (st != OFDFT_OK) return st;
    }
    if (kind == OFDFT_PRECOND_NONE) {
        OFDFT_CHECK_HIP(hipDeviceSynchronize());
        precond_free(b);
        return OFDFT_OK;
    }
    if (b->dtype != OFDFT_C128) {
        set_error("ofdft_batch_set_preconditioner: multigrid needs dtype C128");
        return OFDFT_INVALID_ARG;
    }
    // build everything first, so a failure leaves the batch unchanged
    std::vector<Multigrid *> own, of(b->nsys, nullptr);
    std::vector<void *> z(b->nsys, nullptr);
    std::vector<int> qidx(b->nsys, 0);
    std::vector<std::pair<int, int>> groups;
    double *kap = nullptr;
    void **rtab = nullptr, **ztab = nullptr;
    const int lanes = std::min(b->nsys, kMgLanes);
    std::vector<hipStream_t> lane;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    auto undo = [&](int st) {
        for (Multigrid *mg : own) {
            mg_free(*mg);
            delete mg;
        }
        for (void *p : z)
            if (p) (void)hipFree(p);
        if (kap) (void)hipFree(kap);
        if (rtab) (void)hipFree(rtab);
        if (ztab) (void)hipFree(ztab);
        for (hipStream_t q : lane) (void)hipStreamDestroy(q);
        for (hipEvent_t e : join) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        return st;
    };
    for (int k = 0; k < lanes; ++k) {
        hipStream_t q = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) return undo(OFDFT_HIP_ERROR);
        lane.push_back(q);
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return undo(OFDFT_HIP_ERROR);
        join.push_back(e);
    }
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return undo(OFDFT_HIP_ERROR);
    if (hipMalloc(&kap, 2 * sizeof(double)) != hipSuccess) {
        kap = nullptr;
        set_error("ofdft_batch_set_preconditioner: out of device memory");
        return undo(OFDFT_NO_MEMORY);
    }
    auto same = [](const ofdft_grid &p, const ofdft_grid &q) {
        return q.nx == p.nx && q.ny == p.ny && q.nz == p.nz && q.hx == p.hx && q.hy == p.hy && q.hz == p.hz;
    };
    for (int j = 0; j < b->nsys;) {
        int k = j + 1;
        while (k < b->nsys && k - j < kMgGroupMax && same(b->grids[k], b->grids[j])) ++k;
        Multigrid *mg = new (std::nothrow) Multigrid();
        if (!mg) return undo(OFDFT_NO_MEMORY);
        own.push_back(mg);
        const int st = mg_create(*mg, b->grids[j], 16, kind == OFDFT_PRECOND_MULTIGRID, k - j);
        if (st != OFDFT_OK) return undo(st);
        for (int i = j; i < k; ++i) {
            of[i] = mg;
            qidx[i] = i - j;
        }
        groups.push_back({j, k - j});
        j = k;
    }
    for (int j = 0; j < b->nsys; ++j) {
        const ofdft_grid &g = b->grids[j];
        if (hipMalloc(&z[j], sizeof(double2) * (size_t)npoints(g)) != hipSuccess) {
            z[j] = nullptr;
            set_error("ofdft_batch_set_preconditioner: out of device memory");
            return undo(OFDFT_NO_MEMORY);
        }
    }
    {
        std::vector<void *> rt(b->r.begin(), b->r.begin() + b->nsys);
        if (hipMalloc(&rtab, sizeof(void *) * b->nsys) != hipSuccess) {
            rtab = nullptr;
            set_error("ofdft_batch_set_preconditioner: out of device memory");
            return undo(OFDFT_NO_MEMORY);
        }
        if (hipMalloc(&ztab, sizeof(void *) * b->nsys) != hipSuccess) {
            ztab = nullptr;
            set_error("ofdft_batch_set_preconditioner: out of device memory");
            return undo(OFDFT_NO_MEMORY);
        }
        if (hipMemcpy(rtab, rt.data(), sizeof(void *) * b->nsys, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ztab, z.data(), sizeof(void *) * b->nsys, hipMemcpyHostToDevice) != hipSuccess)
            return undo(OFDFT_HIP_ERROR);
    }
    OFDFT_CHECK_HIP(hipDeviceSynchronize());
    precond_free(b);
    b->mg_own = own;
    b->mg_of = of;
    b->mg_q = qidx;
    b->mg_groups = groups;
    b->d_rtab = rtab;
    b->d_ztab = ztab;
    b->z = z;
    b->d_kap = kap;
    b->mg_lane = lane;
    b->mg_join = join;
    b->mg_fork = fork;
    b->precond = kind;
    return OFDFT_OK;
}

extern "C" int ofdft_batch_apply_preconditioner(ofdft_batch *b, int j, const double *kappa, const void *r,
                                                void *z, void *stream) {
    if (!b || !b->precond || j < 0 || j >= b->nsys || !kappa || !r || !z || r == z) {
        set_error("ofdft_batch_apply_preconditioner: bad arguments (preconditioner set, 0 <= j < nsys, z != r)");
        return OFDFT_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    OFDFT_CHECK_HIP(hipMemcpyAsync(b->d_kap, kappa, 2 * sizeof(double), hipMemcpyHostToDevice, s));
    {
        ProfScope ps(K_MULTIGRID_C, mg_cycle_bytes(*b->mg_of[j]), s);
        OFDFT_TRY(mg_apply_shifted(*b->mg_of[j], b->mg_q[j], (const double2 *)r, (double2 *)z, b->d_kap, nullptr, s));
    }
    OFDFT_CHECK_HIP(hipStreamSynchronize(s));
    return OFDFT_OK;
}

static int batch_solve(ofdft_batch *b, const double *kappa, const void *const *rhs, void *const *x,
                       double rel_tol, int max_iter, ofdft_solve_stats *stats, hipStream_t s) {
    const int nsys = b->nsys;
    const bool c64 = b->dtype == OFDFT_C64;
    const int shape = b->shape >= 0 ? b->shape : default_shape(b);
    const int P = b->P;      // 0: stepped schedule; > 0: persistent groups of P workgroups
    if (b->precond && P > 0) {
        set_error("cg_helmholtz_solve_batched: the preconditioner needs the stepped schedule (group 0)");
        return OFDFT_INVALID_ARG;
    }
    // LPT order: longest estimated solve first
    std::vector<double> cost(nsys);
    for (int j = 0; j < nsys; ++j) cost[j] = est_cost(b->grids[j], kappa[2 * j], kappa[2 * j + 1]);
    std::vector<int> order(nsys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });

    std::vector<HState> hst(nsys);
    std::vector<double> tot(2 * nsys);
    std::vector<int> iters(nsys, 0), outer(nsys, 0), done(nsys, H_RUNNING);
    std::vector<HSys> hs;
    std::vector<int> caps(nsys), it_pass(nsys), done_pass(nsys);
    auto run_pass = [&](const std::vector<int> &which, double tol, int cap,
                        const std::vector<const void *> &fs, const std::vector<void *> &xs) -> int {
        const bool stepped = P == 0;
        OFDFT_TRY(upload_systems(b, kappa, fs, xs, c64, shape, stepped, hs, s));
        const double e = c64 ? 8.0 : 16.0;
        if (stepped) {
            for (int j = 0; j < nsys; ++j) caps[j] = std::max(0, cap - iters[j]);
            OFDFT_TRY(stepped_run(b, c64, shape, hs, which, caps, tol, it_pass, done_pass, s));
            double bs = 0.0, bu = 0.0;
            for (int j : which) {
                iters[j] += it_pass[j];
                done[j] = done_pass[j];
                // init: read x, f, write r; stencil phase: read r (z), p_old,
                // Ap_old, x, write p, Ap, x (the first one reads r only and
                // writes p, Ap); vector phase: read r, Ap, write r (the last
                // direction's x update is accounted by the run itself)
                const double n = (double)npoints(b->grids[j]);
                bs += n * e * (3.0 + (it_pass[j] > 0 ? 7.0 * it_pass[j] - 4.0 : 0.0));
                bu += n * e * 3.0 * it_pass[j];
                if (b->precond) {
                    // one cycle and one dot phase (read r, z) after the init
                    // phase and after each iteration but the last
                    const int cycles = it_pass[j];
                    bu += n * e * 2.0 * cycles;
                    prof_add(K_MULTIGRID_C, mg_cycle_bytes(*b->mg_of[j]) * cycles, 0);
                }
            }
            prof_add(K_COCG, bs, 0);
            prof_add(K_COCG_UPDATE, bu, 0);
            return OFDFT_OK;
        }
        for (int j = 0; j < nsys; ++j) {
            hst[j] = HState{};
            hst[j].maxit = std::max(0, cap - iters[j]);
        }
        OFDFT_CHECK_HIP(hipMemcpyAsync(b->d_st, hst.data(), sizeof(HState) * nsys, hipMemcpyHostToDevice, s));
        OFDFT_CHECK_HIP(hipMemcpyAsync(b->d_order, which.data(), sizeof(int) * which.size(),
                                       hipMemcpyHostToDevice, s));
        if (c64) OFDFT_TRY(run_persistent<float2>(b, shape, P, (int)which.size(), tol, s));
        else OFDFT_TRY(run_persistent<double2>(b, shape, P, (int)which.size(), tol, s));
        OFDFT_CHECK_HIP(hipMemcpyAsync(hst.data(), b->d_st, sizeof(HState) * nsys, hipMemcpyDeviceToHost, s));
        int ab = 0;
        OFDFT_CHECK_HIP(hipMemcpyAsync(&ab, b->d_abort, sizeof(int), hipMemcpyDeviceToHost, s));
        OFDFT_CHECK_HIP(hipStreamSynchronize(s));
        if (ab) {
            set_error("cg_helmholtz_solve_batched: persistent kernel aborted (barrier wait expired)");
            return OFDFT_HIP_ERROR;
        }
        double bytes = 0.0;
        for (int j : which) {
            iters[j] += hst[j].iter;
            done[j] = hst[j].done;
            // init: read x, f, write r; per iteration: read r, p_old, write p, Ap;
            // read x, p, r, Ap, write x, r
            bytes += (double)npoints(b->grids[j]) * e * (3.0 + 10.0 * hst[j].iter);
        }
        prof_add(K_COCG, bytes, 0);
        return OFDFT_OK;
    };

    std::vector<const void *> fs(nsys);
    std::vector<void *> xs(nsys);
    if (!c64) {
        for (int j = 0; j < nsys; ++j) {
            fs[j] = rhs[j];
            xs[j] = x[j];
        }
        OFDFT_TRY(run_pass(order, rel_tol, max_iter, fs, xs));
    } else {
        std::vector<int> active = order;
        for (int step = 0; step < 10 && !active.empty(); ++step) {
            for (int j : active)
                OFDFT_TRY(residual_c128(b, j, (const double2 *)rhs[j], (const double2 *)x[j],
                                        (double2 *)b->r128[j], kappa[2 * j], kappa[2 * j + 1],
                                        b->d_totals + 2 * j, s));
            OFDFT_CHECK_HIP(hipMemcpyAsync(tot.data(), b->d_totals, sizeof(double) * 2 * nsys,
                                           hipMemcpyDeviceToHost, s));
            OFDFT_CHECK_HIP(hipStreamSynchronize(s));
            std::vector<int> next;
            for (int j : active) {
                if (!std::isfinite(tot[2 * j])) done[j] = H_NONFINITE;
                else if (tot[2 * j] <= rel_tol * rel_tol * tot[2 * j + 1]) done[j] = H_CONVERGED;
                else if (iters[j] >= max_iter) done[j] = H_MAXIT;
                else next.push_back(j);
            }
            if (next.empty()) break;
            for (int j : next) {
                CastC64 cc{(const double2 *)b->r128[j], (float2 *)b->f32[j], (float2 *)b->x32[j],
                           b->d_totals + 2 * j, 0.0};
                OFDFT_TRY((launch_reduce<1>(npoints(b->grids[j]), cc, NoFin{}, b->rb, s)));
                ++outer[j];
            }
            for (int j = 0; j < nsys; ++j) {
                fs[j] = b->f32[j];
                xs[j] = b->x32[j];
            }
            OFDFT_TRY(run_pass(next, 1e-4, max_iter, fs, xs));
            for (int j : next) {
                if (done[j] == H_NONFINITE) continue;
                AddC64 ad{(double2 *)x[j], (const float2 *)b->x32[j], b->d_totals + 2 * j, 0.0};
                OFDFT_TRY((launch_reduce<1>(npoints(b->grids[j]), ad, NoFin{}, b->rb, s)));
            }
            active.clear();
            for (int j : next)
                if (done[j] != H_NONFINITE && done[j] != H_BREAKDOWN) active.push_back(j);
        }
    }
    // final true residual of every system in complex128
    for (int j = 0; j < nsys; ++j)
        OFDFT_TRY(residual_c128(b, j, (const double2 *)rhs[j], (const double2 *)x[j], nullptr,
                                kappa[2 * j], kappa[2 * j + 1], b->d_totals + 2 * j, s));
    OFDFT_CHECK_HIP(hipMemcpyAsync(tot.data(), b->d_totals, sizeof(double) * 2 * nsys,
                                   hipMemcpyDeviceToHost, s));
    OFDFT_CHECK_HIP(hipStreamSynchronize(s));
    int status = OFDFT_OK;
    for (int j = 0; j < nsys; ++j) {
        const double rel = tot[2 * j + 1] > 0 ? std::sqrt(tot[2 * j] / tot[2 * j + 1]) : 0.0;
        int sj;
        if (!std::isfinite(rel) || done[j] == H_NONFINITE) sj = OFDFT_NONFINITE;
        else if (rel <= rel_tol) sj = OFDFT_OK;
        else if (done[j] == H_BREAKDOWN) sj = OFDFT_BREAKDOWN;
        else sj = OFDFT_NOT_CONVERGED;
        if (stats) {
            stats[j] = ofdft_solve_stats{};
            stats[j].iters = iters[j];
            stats[j].outer_iters = outer[j];
            stats[j].status = sj;
            stats[j].rel_res = rel;
        }
        if (sj < 0 && (status >= 0 || sj < status)) status = sj;
        else if (sj == OFDFT_NOT_CONVERGED && status == OFDFT_OK) status = sj;
    }
    return status;
}

extern "C" int cg_helmholtz_solve_batched(ofdft_batch *b, const double *kappa, const void *const *rhs,
                                          void *const *x, double rel_tol, int max_iter,
                                          ofdft_solve_stats *stats, void *stream) {
    if (!b || !kappa || !rhs || !x || !(rel_tol > 0) || max_iter < 0) {
        set_error("cg_helmholtz_solve_batched: bad arguments");
        return OFDFT_INVALID_ARG;
    }
    for (int j = 0; j < b->nsys; ++j) {
        if (!rhs[j] || !x[j]) {
            set_error("cg_helmholtz_solve_batched: NULL array for system %d", j);
            return OFDFT_INVALID_ARG;
        }
        if (kappa[2 * j] == 0.0 && kappa[2 * j + 1] == 0.0) {
            set_error("cg_helmholtz_solve_batched: kappa of system %d is zero", j);
            return OFDFT_INVALID_ARG;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    OFDFT_CHECK_HIP(hipEventRecord(b->ev0, s));
    int status = batch_solve(b, kappa, rhs, x, rel_tol, max_iter, stats, s);
    OFDFT_CHECK_HIP(hipEventRecord(b->ev1, s));
    OFDFT_CHECK_HIP(hipEventSynchronize(b->ev1));
    float ms = 0;
    OFDFT_CHECK_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    if (stats)
        for (int j = 0; j < b->nsys; ++j) stats[j].seconds = ms * 1e-3;
    return status;
}
