// Vector and stencil passes of flexible CG (truncation 1) on the projected
// Poisson system, shared by the learned and the multigrid-preconditioned
// forms:
//   alpha = <r,z> / <p,Ap>;  x += alpha p;  r_new = r - alpha Ap
//   z_new = M(r_new);  beta = <z_new, r_new - r> / <z, r>;  p = z_new + beta p
// (for a fixed symmetric positive definite M this is preconditioned CG).
#pragma once

#include "poisson.hpp"

namespace ofdft {

struct EpiAp {           // Ap = -L p, acc <p, Ap>
    double *__restrict__ Ap;
    double *totals;
    double *partials;
    unsigned int *counter;
    double acc;
    __device__ bool skip() const { return false; }
    __device__ void pre(int, int64_t) {}
    __device__ void point(int, int64_t i, double c, double s) {
        Ap[i] = -s;
        acc = ::fma(c, -s, acc);
    }
    __device__ void finish(int block, int nblocks, double *scratch) {
        double x[1] = {acc};
        block_sum<1>(x, scratch);
        double t[1];
        if (reduce_grid<1>(x, partials, nblocks, block, counter, scratch, t)) {
            totals[0] = t[0];
        }
    }
};

struct FcgStepOp {       // x += a p; r_old = r; r -= a Ap; totals {<r,r>}
    static constexpr int kClass = K_CG_UPDATE;
    static constexpr int kBytes = 56;
    double *x, *r, *r_old;
    const double *p, *Ap;
    double a;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        x[i] = ::fma(a, p[i], x[i]);
        const double ro = r[i];
        r_old[i] = ro;
        const double rn = ::fma(-a, Ap[i], ro);
        r[i] = rn;
        acc[0] = ::fma(rn, rn, acc[0]);
    }
};

struct FcgDotsOp {       // totals {<z, r - r_old>, <r, z>}
    static constexpr int kClass = K_CG_UPDATE;
    static constexpr int kBytes = 24;
    const double *z, *r, *r_old;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const double zi = z[i], ri = r[i];
        acc[0] = ::fma(zi, ri - r_old[i], acc[0]);
        acc[1] = ::fma(ri, zi, acc[1]);
    }
};

struct DirOp {           // p = z + b p
    static constexpr int kClass = K_CG_UPDATE;
    static constexpr int kBytes = 24;
    double *p;
    const double *z;
    double b;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { p[i] = ::fma(b, p[i], z[i]); }
};

struct AxpyOp {          // y += a x
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24;
    double *y;
    const double *x;
    double a;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { y[i] = ::fma(a, x[i], y[i]); }
};

struct CopyOp2 {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 16;
    double *dst;
    const double *src;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { dst[i] = src[i]; }
};

template <class Load, class Epi>
int pass64(const ofdft_grid &g, const Coef<double> &c, const Load &ld, const Epi &ep, hipStream_t s,
           double bytes_per_point, int cls) {
    ProfScope ps(cls, (double)npoints(g) * bytes_per_point, s);
    return launch_stencil<double>(g, c, ld, ep, s);
}

}  // namespace ofdft
