// Conjugate-gradient building blocks for -L_h x = g on the zero-mean subspace
// (Section 3.3 Poisson equation; Section 4 solver notes).
//
// One iteration = two kernels:
//   K1 (stencil pass): p_new = r + beta p_old (fused into the operand loads),
//      Ap = -L_h p_new, partial p_new . Ap; the last block forms alpha.
//   K2 (vector pass):  x += alpha p, r -= alpha Ap, partial r . r; the last
//      block forms beta and the convergence / breakdown flags.
// Scalars stay on the device; kernels exit immediately once `done` is set so
// that the host can enqueue iterations in blocks and check rarely.
#pragma once

#include "stencil_launch.hpp"
#include "vec.hpp"

namespace ofdft {

enum CgDone { CG_RUNNING = 0, CG_CONVERGED = 1, CG_BREAKDOWN = 2, CG_NONFINITE = 3, CG_MAXIT = 4 };

struct CgState {
    double rr;        // r . r of the current residual
    double pAp;
    double alpha, beta;
    double tol2;      // stop when rr <= tol2
    double aux[4];    // scratch totals (means, norms)
    int iter, done, maxit, first;
};

template <typename T>
struct LoadCgP {      // operand of K1: r + beta p_old (first iteration: p_old := r, beta := 0)
    const T *__restrict__ r;
    const T *__restrict__ p_old;
    const CgState *st;
    typename VT<T>::S beta;
    __device__ void prepare() {
        if (st->first) {
            p_old = r;
            beta = 0;
        } else {
            beta = (typename VT<T>::S)st->beta;
        }
    }
    __device__ T operator()(int64_t i) const { return VT<T>::fma(beta, p_old[i], r[i]); }
};

template <typename T>
struct EpiCgAp {
    T *__restrict__ p_out;
    T *__restrict__ Ap;
    CgState *st;
    double *partials;
    unsigned int *counter;
    double acc;
    __device__ bool skip() const { return st->done != CG_RUNNING; }
    __device__ void pre(int, int64_t) {}
    __device__ void point(int, int64_t i, T c, T s) {
        const T a = VT<T>::mul(typename VT<T>::S(-1), s);
        p_out[i] = c;
        Ap[i] = a;
        acc = ::fma((double)c, (double)a, acc);
    }
    __device__ void finish(int block, int nblocks, double *scratch) {
        double x[1] = {acc};
        block_sum<1>(x, scratch);
        double t[1];
        if (reduce_grid<1>(x, partials, nblocks, block, counter, scratch, t)) {
            const double pAp = t[0];
            st->pAp = pAp;
            if (!isfinite(pAp)) st->done = CG_NONFINITE;
            else if (!(pAp > 0.0)) st->done = CG_BREAKDOWN;
            else st->alpha = st->rr / pAp;
        }
    }
};

template <typename T>
struct CgUpdate {     // K2 body
    static constexpr int kClass = K_CG_UPDATE;
    static constexpr int kBytes = 6 * sizeof(T);
    T *__restrict__ x;
    T *__restrict__ r;
    const T *__restrict__ p;
    const T *__restrict__ Ap;
    const CgState *st;
    typename VT<T>::S alpha;
    __device__ bool skip() const { return st->done != CG_RUNNING; }
    __device__ void prepare() { alpha = (typename VT<T>::S)st->alpha; }
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        x[i] = VT<T>::fma(alpha, p[i], x[i]);
        const T rn = VT<T>::fma(-alpha, Ap[i], r[i]);
        r[i] = rn;
        acc[0] = ::fma((double)rn, (double)rn, acc[0]);
    }
};

struct CgUpdateFin {
    CgState *st;
    __device__ void operator()(const double (&t)[1]) const {
        const double rr = t[0];
        st->beta = rr / st->rr;
        st->rr = rr;
        st->first = 0;
        st->iter += 1;
        if (!isfinite(rr)) st->done = CG_NONFINITE;
        else if (rr <= st->tol2) st->done = CG_CONVERGED;
        else if (st->iter >= st->maxit) st->done = CG_MAXIT;
    }
};

// Residual pass: r = g + L_h x (= g - A x with A = -L_h), totals sum r, sum r^2.
template <typename T>
struct EpiResidual {
    const double *__restrict__ g;
    T *__restrict__ r;
    double *totals;        // receives {sum r, sum r^2}
    double *partials;
    unsigned int *counter;
    double acc0, acc1;
    double gv[4];
    __device__ bool skip() const { return false; }
    __device__ void pre(int q, int64_t i) { gv[q] = g[i]; }
    __device__ void point(int q, int64_t i, T, T s) {
        const double v = gv[q] + (double)s;
        r[i] = (T)v;
        acc0 += v;
        acc1 = ::fma(v, v, acc1);
    }
    __device__ void finish(int block, int nblocks, double *scratch) {
        double x[2] = {acc0, acc1};
        block_sum<2>(x, scratch);
        double t[2];
        if (reduce_grid<2>(x, partials, nblocks, block, counter, scratch, t)) {
            totals[0] = t[0];
            totals[1] = t[1];
        }
    }
};

}  // namespace ofdft
