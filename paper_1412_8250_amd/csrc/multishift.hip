// Multi-shift COCG: the shifted systems (-L_h + kappa_r) u_r = f of ONE
// right-hand side (the kernel convolutions of Section 3.1 and the order-2
// terms of Section 2 apply several shifts to the same f) solved with one
// Krylov sequence.  The Krylov space of -L_h + kappa does not depend on kappa,
// so COCG on a seed system A = -L_h + kappa_s yields every shift's iterate
// through scalar recurrences (shifted COCG, Takayama et al., Phys. Rev. B 73,
// 165108 (2006)); with sigma = kappa_r - kappa_s:
//   r_k^(r) = r_k / pi_k^(r),
//   pi_{k+1} = (1 + alpha_k sigma) pi_k + (alpha_k beta_{k-1} / alpha_{k-1}) (pi_k - pi_{k-1}),
//   alpha_k^(r) = alpha_k pi_k / pi_{k+1},  beta_{k-1}^(r) = (pi_{k-1} / pi_k)^2 beta_{k-1}.
// One stencil application per iteration serves all shifts; iterates start at
// zero.  A shift whose residual |r_k| / |pi_k| reaches the tolerance is
// frozen; the seed sequence runs until every shift is frozen.  The recurred
// residual and the true one drift apart in floating point, so each shift's
// true residual is recomputed at the end, and a shift still above the
// tolerance gets correction solves (iterative refinement): e from
// (-L_h + kappa_r) e = f - (-L_h + kappa_r) x_r by a one-shift sequence from
// zero, x_r += e, until the true residual meets the tolerance.
//
// Two launches per iteration:
//  * stencil phase: the stencil runs on r alone; the seed direction and its
//    image follow point by point, p = r + beta p_old and q = A r + beta q_old
//    (A linear; q updated in place), p^T q is reduced; the last workgroup
//    sets alpha_k and every running shift's pi_{k+1} and alpha_k^(r);
//  * vector phase: every running shift forms p^(r) = r / pi^(r) + beta^(r)
//    p^(r) (the seed's was written by the stencil phase) and x^(r) +=
//    alpha^(r) p^(r); r -= alpha q; r^T r and |r|^2 are reduced and the last
//    workgroup sets beta_k, the next beta^(r), advances pi and freezes the
//    converged shifts.
// Per point and iteration this moves 5 complex128 vectors in the stencil
// phase and 3 + 3 (seed) + 4 per other running shift in the vector phase,
// against 11 per system for separate COCG solves.  The scalars live on the
// device; the host reads the status every few iterations, and launches made
// after the end exit at once.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "helmholtz.hpp"

namespace ofdft {
namespace {

constexpr int kMsMax = 16;          // shifts per solve
constexpr int kMsThreads = 256;     // vector-phase workgroup
constexpr int kMsMaxVBlocks = 4096;
constexpr int kMsPoll = 8;          // iterations between status reads

struct MsShift {
    double2 *x, *p;              // iterate (caller's array); direction (unused for the seed)
    double sre, sim;             // sigma = kappa_r - kappa_seed
    double pi_re, pi_im;         // pi_k
    double pp_re, pp_im;         // pi_{k-1}
    double pn_re, pn_im;         // pi_{k+1} (set by the stencil phase)
    double ir_re, ir_im;         // 1 / pi_k
    double al_re, al_im;         // alpha_k^(r)
    double be_re, be_im;         // beta_{k-1}^(r)
    int run, stat, iters, pad;   // run: updated this iteration; stat: HDone code
};

struct MsState {
    double rho_re, rho_im;       // r_k^T r_k
    double al_re, al_im;         // alpha_k
    double alp_re, alp_im;       // alpha_{k-1}
    double be_re, be_im;         // beta_{k-1}
    double rn2, fn2, tol2;       // |r_k|^2, |f|^2, tol^2 |f|^2
    int iter, done, maxit, nshift, seed, parity;   // parity 0: seed p_old in pA
};

__device__ inline double2 c2(double a, double b) { return make_double2(a, b); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// r = f, every iterate zero; {f^T f re, im, |f|^2}.
__global__ void __launch_bounds__(kMsThreads)
ms_init(MsState *st, const MsShift *sh, const double2 *f, double2 *r, int64_t n, double tol,
        double *part, unsigned int *ctr) {
    __shared__ double scratch[3 * (kMsThreads / 64)];
    __shared__ double2 *s_x[kMsMax];
    const int S = st->nshift;
    if ((int)threadIdx.x < S) s_x[threadIdx.x] = sh[threadIdx.x].x;
    __syncthreads();
    const GPtr<double2> F(f), R(r);
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kMsThreads;
    for (int64_t i = (int64_t)blockIdx.x * kMsThreads + threadIdx.x; i < n; i += stride) {
        const double2 fv = F[i];
        R.st(i, fv);
        for (int j = 0; j < S; ++j) GPtr<double2>(s_x[j]).st(i, c2(0.0, 0.0));
        acc[0] += fv.x * fv.x - fv.y * fv.y;
        acc[1] += 2.0 * fv.x * fv.y;
        acc[2] += fv.x * fv.x + fv.y * fv.y;
    }
    block_sum<3>(acc, scratch);
    double t[3];
    if (reduce_grid<3>(acc, part, gridDim.x, blockIdx.x, ctr, scratch, t)) {
        st->rho_re = t[0];
        st->rho_im = t[1];
        st->rn2 = t[2];
        st->fn2 = t[2];
        st->tol2 = tol * tol * t[2];
        int d = H_RUNNING;
        if (!isfinite(t[2])) d = H_NONFINITE;
        else if (t[2] == 0.0) d = H_CONVERGED;
        else if (st->maxit <= 0) d = H_MAXIT;
        st->done = d;
    }
}

struct MsLoadR {
    GPtr<double2> r;
    __device__ double2 operator()(int64_t i) const { return r[i]; }
};

// Centre c = r, s = L r: p = r + beta p_old and q = (-L r + kappa_s r) +
// beta q_old written (q in place: each point is read and written by the same
// thread); the first iteration (beta = 0, its own kernel) reads neither.
// acc {p^T q re, im}.
template <bool First>
struct MsEpiQ {
    GPtr<double2> p_old, p_out, q;
    double2 kappa, beta;
    double acc[2];
    double2 po[2], qo[2];
    __device__ void pre(int r, int64_t i) {
        if constexpr (!First) {
            po[r] = p_old[i];
            qo[r] = q[i];
        }
    }
    __device__ void point(int r, int64_t i, double2 c, double2 s) {
        double2 a = cfma(kappa, c, c2(-s.x, -s.y));
        double2 p = c;
        if constexpr (!First) {
            p = cfma(beta, po[r], c);
            a = cfma(beta, qo[r], a);
        }
        p_out.st(i, p);
        q.st(i, a);
        acc[0] += p.x * a.x - p.y * a.y;
        acc[1] += p.x * a.y + p.y * a.x;
    }
};

// First: iteration 0 (launched as the first stencil phase after ms_init).
template <int TX, int TYT, int RY, bool First>
__global__ void __launch_bounds__(TX * TYT)
ms_stencil(TileGeom tg, Coef<double> coef, double kre, double kim, MsState *st, MsShift *sh,
           const double2 *r, double2 *pA, double2 *pB, double2 *q, double *part, unsigned int *ctr) {
    using SLd = StencilLds<double2, TX, TYT, RY>;
    __shared__ double2 lds[SLd::kElems];
    __shared__ double scratch[2 * (TX * TYT / 64)];
    if (st->done != H_RUNNING) return;
    const int total = tg.nblocks;
    const int lb = xcd_remap(blockIdx.x, total);
    constexpr bool first = First;
    const double2 *p_old = st->parity ? pB : pA;
    double2 *p_new = st->parity ? pA : pB;
    MsLoadR ld{GPtr<double2>(r)};
    MsEpiQ<First> ep{GPtr<double2>(p_old), GPtr<double2>(p_new), GPtr<double2>(q), c2(kre, kim),
                     c2(st->be_re, st->be_im), {0.0, 0.0}, {}, {}};
    stencil_tile<double2, TX, TYT, RY>(tg, coef, ld, ep, lb, lds);
    double acc[2] = {ep.acc[0], ep.acc[1]};
    block_sum<2>(acc, scratch);
    double t[2];
    if (!reduce_grid<2>(acc, part, total, lb, ctr, scratch, t)) return;
    const double2 pq = c2(t[0], t[1]);
    if (!cfinite(pq)) {
        st->done = H_NONFINITE;
        return;
    }
    if (cabs2(pq) == 0.0) {
        st->done = H_BREAKDOWN;
        return;
    }
    const double2 al = cdiv(c2(st->rho_re, st->rho_im), pq);
    st->al_re = al.x;
    st->al_im = al.y;
    // alpha_k beta_{k-1} / alpha_{k-1} (zero in the first iteration: beta_{-1} = 0)
    const double2 c = first ? c2(0.0, 0.0) : cdiv(cmul(al, c2(st->be_re, st->be_im)), c2(st->alp_re, st->alp_im));
    for (int j = 0; j < st->nshift; ++j) {
        MsShift &s = sh[j];
        if (!s.run) continue;
        const double2 pi = c2(s.pi_re, s.pi_im), pp = c2(s.pp_re, s.pp_im);
        const double2 ga = c2(1.0 + al.x * s.sre - al.y * s.sim, al.x * s.sim + al.y * s.sre);
        const double2 pn = cfma(c, csub(pi, pp), cmul(ga, pi));
        s.pn_re = pn.x;
        s.pn_im = pn.y;
        if (!cfinite(pn) || cabs2(pn) == 0.0) {
            s.run = 0;
            s.stat = cfinite(pn) ? H_BREAKDOWN : H_NONFINITE;
            s.iters = st->iter;
            continue;
        }
        const double2 aj = cdiv(cmul(al, pi), pn);
        s.al_re = aj.x;
        s.al_im = aj.y;
    }
}

__global__ void __launch_bounds__(kMsThreads)
ms_update(MsState *st, MsShift *sh, double2 *r, const double2 *q, const double2 *pA, const double2 *pB,
          int64_t n, double *part, unsigned int *ctr) {
    __shared__ double scratch[3 * (kMsThreads / 64)];
    __shared__ double2 *s_x[kMsMax];
    __shared__ double2 *s_p[kMsMax];
    __shared__ double2 s_ir[kMsMax], s_be[kMsMax], s_al[kMsMax];
    __shared__ int s_run[kMsMax];
    if (st->done != H_RUNNING) return;
    const int S = st->nshift, seed = st->seed;
    const bool first = st->iter == 0;
    if ((int)threadIdx.x < S) {
        const MsShift &s = sh[threadIdx.x];
        s_x[threadIdx.x] = s.x;
        s_p[threadIdx.x] = (int)threadIdx.x == seed ? nullptr : s.p;
        s_ir[threadIdx.x] = c2(s.ir_re, s.ir_im);
        s_be[threadIdx.x] = c2(s.be_re, s.be_im);
        s_al[threadIdx.x] = c2(s.al_re, s.al_im);
        s_run[threadIdx.x] = s.run;
    }
    __syncthreads();
    const GPtr<double2> R(r), Q(q), PS(st->parity ? pA : pB);   // the seed direction just written
    const double2 nal = c2(-st->al_re, -st->al_im);
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kMsThreads;
    for (int64_t i = (int64_t)blockIdx.x * kMsThreads + threadIdx.x; i < n; i += stride) {
        const double2 rv = R[i];
        const double2 qv = Q[i];
        for (int j = 0; j < S; ++j) {
            if (!s_run[j]) continue;
            double2 pj;
            if (j == seed) {
                pj = PS[i];
            } else {
                const GPtr<double2> P(s_p[j]);
                pj = cmul(rv, s_ir[j]);
                if (!first) pj = cfma(s_be[j], P[i], pj);
                P.st(i, pj);
            }
            const GPtr<double2> X(s_x[j]);
            X.st(i, cfma(s_al[j], pj, X[i]));
        }
        const double2 rn = cfma(nal, qv, rv);
        R.st(i, rn);
        acc[0] += rn.x * rn.x - rn.y * rn.y;
        acc[1] += 2.0 * rn.x * rn.y;
        acc[2] += rn.x * rn.x + rn.y * rn.y;
    }
    block_sum<3>(acc, scratch);
    double t[3];
    if (!reduce_grid<3>(acc, part, gridDim.x, blockIdx.x, ctr, scratch, t)) return;
    const double2 rho = c2(st->rho_re, st->rho_im), rho_new = c2(t[0], t[1]);
    const double2 be = cdiv(rho_new, rho);
    const int iter = st->iter + 1;
    int nrun = 0;
    for (int j = 0; j < S; ++j) {
        MsShift &s = sh[j];
        if (!s.run) continue;
        const double2 pi = c2(s.pi_re, s.pi_im), pn = c2(s.pn_re, s.pn_im);
        const double2 ratio = cdiv(pi, pn);
        const double2 bj = cmul(cmul(ratio, ratio), be);
        const double2 ir = cdiv(c2(1.0, 0.0), pn);
        s.be_re = bj.x;
        s.be_im = bj.y;
        s.pp_re = pi.x;
        s.pp_im = pi.y;
        s.pi_re = pn.x;
        s.pi_im = pn.y;
        s.ir_re = ir.x;
        s.ir_im = ir.y;
        if (t[2] <= st->tol2 * cabs2(pn)) {
            s.run = 0;
            s.stat = H_CONVERGED;
            s.iters = iter;
        } else {
            ++nrun;
        }
    }
    st->alp_re = st->al_re;
    st->alp_im = st->al_im;
    st->be_re = be.x;
    st->be_im = be.y;
    st->rho_re = t[0];
    st->rho_im = t[1];
    st->rn2 = t[2];
    st->iter = iter;
    st->parity ^= 1;
    int d = H_RUNNING;
    if (nrun == 0) d = H_CONVERGED;
    else if (!isfinite(t[2]) || !cfinite(be)) d = H_NONFINITE;
    else if (cabs2(rho_new) <= 1e-60 * t[2] * t[2]) d = H_BREAKDOWN;
    else if (iter >= st->maxit) d = H_MAXIT;
    if (d != H_RUNNING && d != H_CONVERGED) {
        for (int j = 0; j < S; ++j) {
            if (!sh[j].run) continue;
            sh[j].run = 0;
            sh[j].stat = d;
            sh[j].iters = iter;
        }
    }
    st->done = d;
}

struct MsLoadX {
    GPtr<double2> x;
    __device__ double2 operator()(int64_t i) const { return x[i]; }
};

struct MsEpiRes {        // acc |f - (-L x + kappa x)|^2
    GPtr<double2> f;
    double2 kappa;
    double acc[1];
    double2 fo[2];
    __device__ void pre(int r, int64_t i) { fo[r] = f[i]; }
    __device__ void point(int r, int64_t, double2 c, double2 s) {
        const double2 a = cfma(kappa, c, c2(-s.x, -s.y));
        const double2 d = csub(fo[r], a);
        acc[0] += d.x * d.x + d.y * d.y;
    }
};

template <int TX, int TYT, int RY>
__global__ void __launch_bounds__(TX * TYT)
ms_residual(TileGeom tg, Coef<double> coef, double kre, double kim, const double2 *x, const double2 *f,
            double *part, unsigned int *ctr, double *out) {
    using SLd = StencilLds<double2, TX, TYT, RY>;
    __shared__ double2 lds[SLd::kElems];
    __shared__ double scratch[TX * TYT / 64];
    const int total = tg.nblocks;
    const int lb = xcd_remap(blockIdx.x, total);
    MsLoadX ld{GPtr<double2>(x)};
    MsEpiRes ep{GPtr<double2>(f), c2(kre, kim), {0.0}, {}};
    stencil_tile<double2, TX, TYT, RY>(tg, coef, ld, ep, lb, lds);
    double acc[1] = {ep.acc[0]};
    block_sum<1>(acc, scratch);
    double t[1];
    if (reduce_grid<1>(acc, part, total, lb, ctr, scratch, t)) *out = t[0];
}

struct MsEpiResVec {     // d = f - (-L x + kappa x) written; acc |d|^2
    GPtr<double2> f, d;
    double2 kappa;
    double acc[1];
    double2 fo[2];
    __device__ void pre(int r, int64_t i) { fo[r] = f[i]; }
    __device__ void point(int r, int64_t i, double2 c, double2 s) {
        const double2 a = cfma(kappa, c, c2(-s.x, -s.y));
        const double2 dv = csub(fo[r], a);
        d.st(i, dv);
        acc[0] += dv.x * dv.x + dv.y * dv.y;
    }
};

template <int TX, int TYT, int RY>
__global__ void __launch_bounds__(TX * TYT)
ms_resvec(TileGeom tg, Coef<double> coef, double kre, double kim, const double2 *x, const double2 *f,
          double2 *d, double *part, unsigned int *ctr, double *out) {
    using SLd = StencilLds<double2, TX, TYT, RY>;
    __shared__ double2 lds[SLd::kElems];
    __shared__ double scratch[TX * TYT / 64];
    const int total = tg.nblocks;
    const int lb = xcd_remap(blockIdx.x, total);
    MsLoadX ld{GPtr<double2>(x)};
    MsEpiResVec ep{GPtr<double2>(f), GPtr<double2>(d), c2(kre, kim), {0.0}, {}};
    stencil_tile<double2, TX, TYT, RY>(tg, coef, ld, ep, lb, lds);
    double acc[1] = {ep.acc[0]};
    block_sum<1>(acc, scratch);
    double t[1];
    if (reduce_grid<1>(acc, part, total, lb, ctr, scratch, t)) *out = t[0];
}

// x += e
__global__ void __launch_bounds__(kMsThreads) ms_axpy(double2 *x, const double2 *e, int64_t n) {
    const GPtr<double2> X(x), E(e);
    const int64_t stride = (int64_t)gridDim.x * kMsThreads;
    for (int64_t i = (int64_t)blockIdx.x * kMsThreads + threadIdx.x; i < n; i += stride) {
        const double2 a = X[i], b = E[i];
        X.st(i, c2(a.x + b.x, a.y + b.y));
    }
}

// Seed rank (smaller converges slower): a shift with Re kappa < 0 puts a
// near-resonance -kappa inside the spectrum of -L_h (a subset of [0, inf)),
// worst for the smallest |Im kappa|; otherwise the smallest |kappa| is the
// closest to the spectrum's lower end.
bool slower_shift(double ar, double ai, double br, double bi) {
    const bool a_in = ar < 0.0, b_in = br < 0.0;
    if (a_in != b_in) return a_in;
    return a_in ? std::fabs(ai) < std::fabs(bi) : std::hypot(ar, ai) < std::hypot(br, bi);
}

}  // namespace
}  // namespace ofdft

using namespace ofdft;

struct ofdft_multishift {
    ofdft_grid grid{};
    int radius = 0;
    int max_shifts = 0;
    int shape = 0;               // effective complex128 tile shape
    TileGeom tg{};
    Coef<double> coef{};
    int64_t n = 0;
    int vblocks = 0;
    double2 *r = nullptr, *q = nullptr, *pA = nullptr, *pB = nullptr;
    std::vector<double2 *> p;    // directions of non-seed shifts (max_shifts - 1, at least
                                 // one: p[0] holds the correction of the finishing solves)
    MsState *d_state = nullptr;
    MsShift *d_shift = nullptr;
    double *d_part = nullptr;
    unsigned int *d_ctr = nullptr;
    double *d_res = nullptr;     // kMsMax residual norms
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

void ms_free(ofdft_multishift *m) {
    for (void *p : {(void *)m->r, (void *)m->q, (void *)m->pA, (void *)m->pB, (void *)m->d_state,
                    (void *)m->d_shift, (void *)m->d_part, (void *)m->d_ctr, (void *)m->d_res})
        if (p) (void)hipFree(p);
    for (double2 *p : m->p)
        if (p) (void)hipFree(p);
    m->p.clear();
    if (m->ev0) (void)hipEventDestroy(m->ev0);
    if (m->ev1) (void)hipEventDestroy(m->ev1);
}

template <typename P_>
int ms_alloc(P_ **p, size_t bytes) {
    if (hipMalloc((void **)p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("multi-shift COCG: device allocation of %zu bytes failed", bytes);
        return OFDFT_NO_MEMORY;
    }
    return OFDFT_OK;
}

// The two complex128 tiles the solver uses (32 x 8 for small grids).
template <class F>
int ms_dispatch(int shape, F &&f) {
    if (shape == SHAPE_32x8x2) return f(ShapeTag<32, 8, 2>{});
    return f(ShapeTag<64, 8, 1>{});
}

}  // namespace

extern "C" int ofdft_multishift_create(const ofdft_grid *grid, int radius, int max_shifts,
                                       ofdft_multishift **out) {
    if (!out || !grid || max_shifts < 1 || max_shifts > kMsMax) {
        set_error("ofdft_multishift_create: need a grid and 1 <= max_shifts <= %d", kMsMax);
        return OFDFT_INVALID_ARG;
    }
    OFDFT_TRY(check_grid(grid, radius));
    ofdft_multishift *m = new (std::nothrow) ofdft_multishift();
    if (!m) return OFDFT_NO_MEMORY;
    auto fail = [&](int st) {
        ms_free(m);
        delete m;
        return st;
    };
    m->grid = *grid;
    m->radius = radius;
    m->max_shifts = max_shifts;
    m->n = npoints(*grid);
    m->coef = make_coef(*grid, radius);
    m->shape = cocg_shape<double2>(grid->nx <= 40 ? SHAPE_32x8x2 : SHAPE_64x8x1);
    const int zl = stepped_zlen(*grid, false, m->shape);
    ms_dispatch(m->shape, [&](auto sh) {
        using S = decltype(sh);
        m->tg = make_tile_geom<S::TX, S::TYT, S::RY>(*grid, zl);
        return 0;
    });
    m->vblocks = (int)std::min<int64_t>(kMsMaxVBlocks, (m->n + kMsThreads - 1) / kMsThreads);
    const size_t vb = sizeof(double2) * (size_t)m->n;
    const size_t nslots = (size_t)std::max(m->tg.nblocks, m->vblocks);
    m->p.assign(std::max(max_shifts - 1, 1), nullptr);
    int st = OFDFT_OK;
    if ((st = ms_alloc(&m->r, vb)) || (st = ms_alloc(&m->q, vb)) || (st = ms_alloc(&m->pA, vb)) ||
        (st = ms_alloc(&m->pB, vb)) || (st = ms_alloc(&m->d_state, sizeof(MsState))) ||
        (st = ms_alloc(&m->d_shift, sizeof(MsShift) * kMsMax)) ||
        (st = ms_alloc(&m->d_part, sizeof(double) * 3 * nslots)) ||
        (st = ms_alloc(&m->d_ctr, 256)) || (st = ms_alloc(&m->d_res, sizeof(double) * kMsMax)))
        return fail(st);
    for (auto &p : m->p)
        if ((st = ms_alloc(&p, vb))) return fail(st);
    if (hipMemset(m->d_ctr, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        set_error("ofdft_multishift_create: clearing the reduction counter failed");
        return fail(OFDFT_HIP_ERROR);
    }
    if (hipEventCreate(&m->ev0) != hipSuccess || hipEventCreate(&m->ev1) != hipSuccess)
        return fail(OFDFT_HIP_ERROR);
    *out = m;
    return OFDFT_OK;
}

extern "C" int ofdft_multishift_destroy(ofdft_multishift *m) {
    if (!m) return OFDFT_OK;
    ms_free(m);
    delete m;
    return OFDFT_OK;
}

namespace {

// The shifted COCG sequence of a seed system from zero: fills the final
// device state and per-shift records (hst, hsh) and accounts the bytes.
int ms_iterate(ofdft_multishift *m, int S, const double *kappa, int seed, const double2 *f,
               double2 *const *x, double tol, int maxit, MsState &hst, std::vector<MsShift> &hsh,
               hipStream_t s) {
    // host-side initial scalars: pi = pi_prev = 1, beta = 0, alpha_prev = 1
    hst = MsState{};
    hst.alp_re = 1.0;
    hst.maxit = maxit;
    hst.nshift = S;
    hst.seed = seed;
    hst.done = H_RUNNING;
    hsh.assign(kMsMax, MsShift{});
    int pi = 0;
    for (int j = 0; j < S; ++j) {
        MsShift &h = hsh[j];
        h.x = x[j];
        h.p = j == seed ? nullptr : m->p[pi++];
        h.sre = kappa[2 * j] - kappa[2 * seed];
        h.sim = kappa[2 * j + 1] - kappa[2 * seed + 1];
        h.pi_re = h.pp_re = h.ir_re = 1.0;
        h.run = 1;
        h.stat = H_RUNNING;
    }
    OFDFT_CHECK_HIP(hipMemcpyAsync(m->d_state, &hst, sizeof(MsState), hipMemcpyHostToDevice, s));
    OFDFT_CHECK_HIP(hipMemcpyAsync(m->d_shift, hsh.data(), sizeof(MsShift) * kMsMax, hipMemcpyHostToDevice, s));
    const double e = sizeof(double2), n = (double)m->n;
    {
        ProfScope ps(K_POINTWISE, n * e * (2.0 + S), s);
        hipLaunchKernelGGL(ms_init, dim3(m->vblocks), dim3(kMsThreads), 0, s, m->d_state, m->d_shift, f,
                           m->r, m->n, tol, m->d_part, m->d_ctr);
        OFDFT_CHECK_HIP(hipGetLastError());
    }
    const double kre = kappa[2 * seed], kim = kappa[2 * seed + 1];
    const int rounds = maxit / kMsPoll + 2;
    for (int round = 0; round < rounds; ++round) {
        OFDFT_CHECK_HIP(hipMemcpyAsync(&hst, m->d_state, sizeof(MsState), hipMemcpyDeviceToHost, s));
        OFDFT_CHECK_HIP(hipStreamSynchronize(s));
        if (hst.done != H_RUNNING) break;
        for (int c = 0; c < kMsPoll; ++c) {
            int st = ms_dispatch(m->shape, [&](auto sh) {
                using Sh = decltype(sh);
                ProfScope ps(K_MS_STENCIL, 0.0, s);
                // the first launch after ms_init is iteration 0
                auto kern = round == 0 && c == 0 ? ms_stencil<Sh::TX, Sh::TYT, Sh::RY, true>
                                                 : ms_stencil<Sh::TX, Sh::TYT, Sh::RY, false>;
                hipLaunchKernelGGL(kern, dim3(m->tg.nblocks), dim3(Sh::TX, Sh::TYT), 0, s, m->tg, m->coef, kre,
                                   kim, m->d_state, m->d_shift, m->r, m->pA, m->pB, m->q, m->d_part, m->d_ctr);
                OFDFT_CHECK_HIP(hipGetLastError());
                return OFDFT_OK;
            });
            OFDFT_TRY(st);
            ProfScope ps(K_MS_UPDATE, 0.0, s);
            hipLaunchKernelGGL(ms_update, dim3(m->vblocks), dim3(kMsThreads), 0, s, m->d_state, m->d_shift,
                               m->r, m->q, m->pA, m->pB, m->n, m->d_part, m->d_ctr);
            OFDFT_CHECK_HIP(hipGetLastError());
        }
    }
    OFDFT_CHECK_HIP(hipMemcpyAsync(&hst, m->d_state, sizeof(MsState), hipMemcpyDeviceToHost, s));
    OFDFT_CHECK_HIP(hipMemcpyAsync(hsh.data(), m->d_shift, sizeof(MsShift) * kMsMax, hipMemcpyDeviceToHost, s));
    OFDFT_CHECK_HIP(hipStreamSynchronize(s));
    if (hst.done == H_RUNNING) {
        set_error("cocg_multishift_solve: iteration did not finish");
        return OFDFT_HIP_ERROR;
    }
    // Algorithmic bytes of the iterations taken: the stencil phase reads r,
    // p_old and q_old (r only in the first iteration) and writes p and q; the vector
    // phase reads r, q and writes r, plus 3 vectors for the seed (p, x read,
    // x written) and 4 for every other shift (p, x read and written; 3 in the
    // first iteration) while the shift runs.
    const int steps = hst.iter;
    if (steps > 0) {
        prof_add(K_MS_STENCIL, n * e * (5.0 * steps - 2.0), 0);
        double upd = 3.0 * steps;
        for (int j = 0; j < S; ++j) {
            const int it = hsh[j].stat == H_RUNNING ? steps : hsh[j].iters;
            upd += j == seed ? 3.0 * it : (it > 0 ? 4.0 * it - 1.0 : 0.0);
        }
        prof_add(K_MS_UPDATE, n * e * upd, 0);
    }
    return OFDFT_OK;
}

// |f - (-L_h + kappa) x|^2 into *d_out (and the vector into d when d != NULL).
int ms_true_residual(ofdft_multishift *m, const double *kap, const double2 *x, const double2 *f, double2 *d,
                     double *d_out, hipStream_t s) {
    const double e = sizeof(double2), n = (double)m->n;
    return ms_dispatch(m->shape, [&](auto sh) {
        using Sh = decltype(sh);
        if (d) {
            ProfScope ps(K_RESIDUAL, n * e * 3.0, s);
            hipLaunchKernelGGL((ms_resvec<Sh::TX, Sh::TYT, Sh::RY>), dim3(m->tg.nblocks), dim3(Sh::TX, Sh::TYT),
                               0, s, m->tg, m->coef, kap[0], kap[1], x, f, d, m->d_part, m->d_ctr, d_out);
        } else {
            ProfScope ps(K_RESIDUAL, n * e * 2.0, s);
            hipLaunchKernelGGL((ms_residual<Sh::TX, Sh::TYT, Sh::RY>), dim3(m->tg.nblocks), dim3(Sh::TX, Sh::TYT),
                               0, s, m->tg, m->coef, kap[0], kap[1], x, f, m->d_part, m->d_ctr, d_out);
        }
        OFDFT_CHECK_HIP(hipGetLastError());
        return OFDFT_OK;
    });
}

constexpr int kMsFixRounds = 4;     // correction solves per shift at most

int ms_solve(ofdft_multishift *m, int S, const double *kappa, int seed, const double2 *f,
             double2 *const *x, double tol, int maxit, ofdft_solve_stats *stats, hipStream_t s) {
    MsState hst{};
    std::vector<MsShift> hsh;
    OFDFT_TRY(ms_iterate(m, S, kappa, seed, f, x, tol, maxit, hst, hsh, s));
    const int steps = hst.iter;
    const double fn2 = hst.fn2;
    const int done = hst.done;
    // true residuals
    for (int j = 0; j < S; ++j) OFDFT_TRY(ms_true_residual(m, kappa + 2 * j, x[j], f, nullptr, m->d_res + j, s));
    double res2[kMsMax];
    OFDFT_CHECK_HIP(hipMemcpyAsync(res2, m->d_res, sizeof(double) * S, hipMemcpyDeviceToHost, s));
    OFDFT_CHECK_HIP(hipStreamSynchronize(s));
    int extra_it[kMsMax] = {};
    int worst = OFDFT_OK;
    for (int j = 0; j < S; ++j) {
        const MsShift &h = hsh[j];
        double rel = fn2 > 0.0 ? std::sqrt(res2[j] / fn2) : 0.0;
        int code;
        switch (fn2 == 0.0 ? H_CONVERGED : h.stat) {
            case H_CONVERGED: code = rel <= tol ? OFDFT_OK : OFDFT_NOT_CONVERGED; break;
            case H_BREAKDOWN: code = OFDFT_BREAKDOWN; break;
            case H_NONFINITE: code = OFDFT_NONFINITE; break;
            default: code = OFDFT_NOT_CONVERGED; break;
        }
        // A converged shift whose true residual drifted above the tolerance:
        // correction solves d = f - A x (into r), A e = d from zero (e in p[0],
        // one-shift sequence, target tol |f| / |d| with a margin), x += e.
        if (h.stat == H_CONVERGED && code == OFDFT_NOT_CONVERGED && std::isfinite(rel)) {
            int budget = std::max(maxit - steps, 0);
            for (int round = 0; round < kMsFixRounds && rel > tol && budget > 0; ++round) {
                OFDFT_TRY(ms_true_residual(m, kappa + 2 * j, x[j], f, m->r, m->d_res + j, s));
                double d2 = 0.0;
                OFDFT_CHECK_HIP(hipMemcpyAsync(&d2, m->d_res + j, sizeof(double), hipMemcpyDeviceToHost, s));
                OFDFT_CHECK_HIP(hipStreamSynchronize(s));
                if (!(d2 > 0.0) || !std::isfinite(d2)) break;
                const double tc = std::min(0.5, 0.5 * tol * std::sqrt(fn2 / d2));
                MsState cst{};
                std::vector<MsShift> csh;
                double2 *ex[1] = {m->p[0]};
                OFDFT_TRY(ms_iterate(m, 1, kappa + 2 * j, 0, m->r, ex, tc, budget, cst, csh, s));
                extra_it[j] += cst.iter;
                budget -= cst.iter;
                if (cst.done == H_NONFINITE || cst.done == H_BREAKDOWN) break;
                hipLaunchKernelGGL(ms_axpy, dim3(m->vblocks), dim3(kMsThreads), 0, s, x[j], m->p[0], m->n);
                OFDFT_CHECK_HIP(hipGetLastError());
                prof_add(K_POINTWISE, (double)m->n * sizeof(double2) * 3.0, 1);
                OFDFT_TRY(ms_true_residual(m, kappa + 2 * j, x[j], f, nullptr, m->d_res + j, s));
                OFDFT_CHECK_HIP(hipMemcpyAsync(&d2, m->d_res + j, sizeof(double), hipMemcpyDeviceToHost, s));
                OFDFT_CHECK_HIP(hipStreamSynchronize(s));
                rel = std::sqrt(d2 / fn2);
            }
            code = rel <= tol ? OFDFT_OK : OFDFT_NOT_CONVERGED;
        }
        if (done == H_NONFINITE && code == OFDFT_NOT_CONVERGED) code = OFDFT_NONFINITE;
        if (done == H_BREAKDOWN && code == OFDFT_NOT_CONVERGED) code = OFDFT_BREAKDOWN;
        if (!std::isfinite(rel)) code = OFDFT_NONFINITE;
        if (stats) {
            stats[j] = ofdft_solve_stats{};
            stats[j].iters = (h.stat == H_RUNNING ? steps : h.iters) + extra_it[j];
            stats[j].outer_iters = steps;
            stats[j].status = code;
            stats[j].rel_res = rel;
        }
        if (code < 0 && (worst >= 0 || code < worst)) worst = code;
        else if (code > 0 && worst == OFDFT_OK) worst = code;
    }
    return worst;
}

}  // namespace

extern "C" int cocg_multishift_solve(ofdft_multishift *m, int nshift, const double *kappa, int seed,
                                     const void *rhs, void *const *x, double rel_tol, int max_iter,
                                     ofdft_solve_stats *stats, int *seed_used, void *stream) {
    if (!m || !kappa || !rhs || !x || nshift < 1 || nshift > m->max_shifts || seed < -1 || seed >= nshift ||
        !(rel_tol > 0) || max_iter < 0) {
        set_error("cocg_multishift_solve: bad arguments (1 <= nshift <= %d, -1 <= seed < nshift, "
                  "rel_tol > 0, max_iter >= 0)", m ? m->max_shifts : 0);
        return OFDFT_INVALID_ARG;
    }
    for (int j = 0; j < nshift; ++j) {
        if (!x[j] || x[j] == rhs) {
            set_error("cocg_multishift_solve: solution array %d is NULL or the right-hand side", j);
            return OFDFT_INVALID_ARG;
        }
        for (int i = 0; i < j; ++i)
            if (x[i] == x[j]) {
                set_error("cocg_multishift_solve: solution arrays %d and %d are the same", i, j);
                return OFDFT_INVALID_ARG;
            }
        if (!std::isfinite(kappa[2 * j]) || !std::isfinite(kappa[2 * j + 1]) ||
            (kappa[2 * j] == 0.0 && kappa[2 * j + 1] == 0.0)) {
            set_error("cocg_multishift_solve: kappa of shift %d is zero or not finite", j);
            return OFDFT_INVALID_ARG;
        }
    }
    if (seed < 0) {
        seed = 0;
        for (int j = 1; j < nshift; ++j)
            if (slower_shift(kappa[2 * j], kappa[2 * j + 1], kappa[2 * seed], kappa[2 * seed + 1])) seed = j;
    }
    hipStream_t s = (hipStream_t)stream;
    OFDFT_CHECK_HIP(hipEventRecord(m->ev0, s));
    std::vector<double2 *> xs(nshift);
    for (int j = 0; j < nshift; ++j) xs[j] = (double2 *)x[j];
    const int status = ms_solve(m, nshift, kappa, seed, (const double2 *)rhs, xs.data(), rel_tol, max_iter,
                                stats, s);
    OFDFT_CHECK_HIP(hipEventRecord(m->ev1, s));
    OFDFT_CHECK_HIP(hipEventSynchronize(m->ev1));
    float ms = 0;
    OFDFT_CHECK_HIP(hipEventElapsedTime(&ms, m->ev0, m->ev1));
    if (stats)
        for (int j = 0; j < nshift; ++j) stats[j].seconds = ms * 1e-3;
    if (seed_used) *seed_used = seed;
    return status;
}
