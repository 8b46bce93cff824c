// The density update U(v) (Appendix C, Algorithm 1; Section 3.3 fixed-point map):
// minimise  h^3 sum [C_F rho^{5/3} + eps_xc(rho) rho + v rho] - (lambda/2) h^3 sum u L_h u
// over u with h^3 sum u^2 = N_e, by Polak-Ribiere non-linear CG with restarts,
// a line search and renormalisation.  Gradient: 2 H u with
//   H u = -(lambda/2) L_h u + (V_TF + V_xc + v) u.
//
// GPU work per iteration (FP64):
//   Ka  stencil pass on u: H u; totals <u,Hu>, <u,Lu>, <u,u>; eta on device
//   Kb  r = -2 (H u - eta u); totals <r,r>, <r,r_prev>
//   Kd  stencil pass on the new direction d = r + xi d_prev (formed while loading);
//       stores d; totals <u,d>, <d,d>, <u,Ld>, <d,Ld>, <Hu,d>
//   Ke  (per line-search probe) sum of (V_TF+V_xc+v)(rho_s) w (d - t w), w = u + s d
//   Kf  u <- sqrt(N_e) (u + s d) / ||u + s d||
// The line search finds the root of dE/ds with Brent's method; the von
// Weizsacker part of dE/ds is a quadratic in s built from the Kd/Ka totals, so
// each probe reads only u, d and v.
//
// Electrostatics inside (fixed_point 1, the paper's map U(V_LR)): v is the
// external potential and the functional also holds 1/2 h^3 sum (rho + b)
// phi[rho].  Its gradient keeps the form 2 (H u - eta u) with phi[rho] added
// to the potential.  Along the line, rho_s = c_s^2 (u + s d)^2 with
// c_s^2 = N_e / (h^3 ||u + s d||^2), so by linearity
//   phi_s = phi[b] + c_s^2 (Q0 + 2 s Q1 + s^2 Q2),
// Q0, Q1, Q2 the zero-mean fields of u^2, u d and d^2: two Poisson solves per
// iteration (Q1, Q2) make every probe a pointwise pass, and the accepted
// step updates Q0 by the same formula.  Q0 is solved afresh at entry.
//
// Device-driven form (the potential-mixing map, fixed_point 0): the same
// iteration with every scalar decision on the device (struct UDev): the
// residual test, the Polak-Ribiere coefficient and restarts, the slope at
// s = 0 and the line search (the same secant growth and Brent's method as
// the host form, one decision kernel per evaluation), within a budget of
// kProbes evaluations per iteration.  Every kernel returns at once when
// the update is over (or, for the line-search passes, when the step is
// chosen), so blocks of kBlockIters iterations are captured once in a HIP
// graph and replayed; the host reads the state once per block.  Profiled
// runs of the classes launch the same kernels one by one.
//
// Optional preconditioning (not in the paper; its conclusion calls for
// real-space preconditioners, Section 5.5): the steepest-descent direction r
// is replaced by z = M r projected onto the tangent space of the constraint,
// z~ = z - (<u,z>/<u,u>) u, with M one multigrid cycle of -Delta + 2 sigma /
// lambda, sigma = V_TF of the mean density (the scale of the local part of
// the energy's second derivative); Polak-Ribiere becomes
// xi = <r - r_prev, z~> / <r_prev, z~_prev>.  M is symmetric positive
// definite, so z~ is a descent direction and the minimiser is unchanged;
// the iteration count drops several-fold because M removes the h^-2 spread
// of the -(lambda/2) L_h part of the Hessian.
#include <algorithm>
#include <cmath>

#include "physics.hpp"
#include "scf.hpp"

namespace ofdft {

namespace {

// device scalar slots
enum {
    S_UHU = 0, S_ULU, S_UU, S_ETA, S_RR, S_RRP, S_UD, S_DD, S_ULD, S_DLD, S_EVAL, S_COUNT,
    S_DOTS = 24     // 5 slots: <u,z>, <r,z>, <r_prev,z>, <u,r>, <u,r_prev>
};

struct EpiHu {
    const double *__restrict__ v;
    double *__restrict__ Hu;
    double *dsc;
    double *partials;
    unsigned int *counter;
    double half_lam, inv_ne_dv;
    double a0, a1, a2;
    double vv[4];
    __device__ bool skip() const { return false; }
    __device__ void pre(int q, int64_t i) { vv[q] = v[i]; }
    __device__ void point(int q, int64_t i, double c, double s) {
        const double rho = c * c;
        const double vl = rho > 0.0 ? v_local(rho) : 0.0;
        const double hu = ::fma(-half_lam, s, (vl + vv[q]) * c);
        Hu[i] = hu;
        a0 = ::fma(c, hu, a0);
        a1 = ::fma(c, s, a1);
        a2 = ::fma(c, c, a2);
    }
    __device__ void finish(int block, int nblocks, double *scratch) {
        double x[3] = {a0, a1, a2};
        block_sum<3>(x, scratch);
        double t[3];
        if (reduce_grid<3>(x, partials, nblocks, block, counter, scratch, t)) {
            dsc[S_UHU] = t[0];
            dsc[S_ULU] = t[1];
            dsc[S_UU] = t[2];
            dsc[S_ETA] = t[0] * inv_ne_dv;          // eta = h^3 <u,Hu> / N_e
        }
    }
};

struct ResidOp {        // r = -2 (Hu - eta u); totals {<r,r>, <r,r_prev>}
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 32;
    const double *Hu, *u, *r_prev;
    double *r;
    const double *dsc;
    int have_prev;
    double eta;
    __device__ bool skip() const { return false; }
    __device__ void prepare() { eta = dsc[S_ETA]; }
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const double ri = -2.0 * (Hu[i] - eta * u[i]);
        r[i] = ri;
        acc[0] = ::fma(ri, ri, acc[0]);
        if (have_prev) acc[1] = ::fma(ri, r_prev[i], acc[1]);
    }
};

// d' = r + xi d_prev (xi = 0: steepest descent, with d_prev := r); with the
// preconditioner r is z, and the stored direction is d = d' - cu u (EpiLd).
struct LoadDir {
    const double *__restrict__ r;
    const double *__restrict__ d_prev;
    double xi;
    __device__ void prepare() {
        if (xi == 0.0) d_prev = r;
    }
    __device__ double operator()(int64_t i) const { return ::fma(xi, d_prev[i], r[i]); }
};

struct DotsOp {         // totals {<u,z>, <r,z>, <r_prev,z>, <u,r>, <u,r_prev>}
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 32;
    const double *u, *z, *r, *r_prev;
    int have_prev;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[5]) const {
        const double ui = u[i], zi = z[i], ri = r[i];
        acc[0] = ::fma(ui, zi, acc[0]);
        acc[1] = ::fma(ri, zi, acc[1]);
        acc[3] = ::fma(ui, ri, acc[3]);
        if (have_prev) {
            const double pi = r_prev[i];
            acc[2] = ::fma(pi, zi, acc[2]);
            acc[4] = ::fma(ui, pi, acc[4]);
        }
    }
};

// Stores d = d' - cu u (d' from the loader); totals of the loaded d':
// {<u,d'>, <d',d'>, <u,L d'>, <d',L d'>, <H u,d'>} (the host corrects them
// for the -cu u term with <u,u>, <u,L u>, <u,H u>, L being symmetric).
// The last gives the line-search slope at s = 0 without an evaluation pass:
// with u normalised, (V_loc + v) u = H u + (lambda/2) L u, and the lambda
// terms of dE/ds cancel, leaving dE/ds(0) ~ <H u, d> - t <u, H u>.
struct EpiLd {
    const double *__restrict__ u;
    const double *__restrict__ Hu;
    double *__restrict__ d;
    double *totals;
    double *partials;
    unsigned int *counter;
    double cu;
    double a0, a1, a2, a3, a4;
    double uv[4], hv[4];
    __device__ bool skip() const { return false; }
    __device__ void pre(int q, int64_t i) {
        uv[q] = u[i];
        hv[q] = Hu[i];
    }
    __device__ void point(int q, int64_t i, double c, double s) {
        const double ui = uv[q];
        d[i] = ::fma(-cu, ui, c);
        a0 = ::fma(ui, c, a0);
        a1 = ::fma(c, c, a1);
        a2 = ::fma(ui, s, a2);
        a3 = ::fma(c, s, a3);
        a4 = ::fma(hv[q], c, a4);
    }
    __device__ void finish(int block, int nblocks, double *scratch) {
        double x[5] = {a0, a1, a2, a3, a4};
        block_sum<5>(x, scratch);
        double t[5];
        if (reduce_grid<5>(x, partials, nblocks, block, counter, scratch, t)) {
            for (int k = 0; k < 5; ++k) totals[k] = t[k];
        }
    }
};

struct EvalOp {         // sum (V_loc(rho_s) + v) w (d - t w),  w = u + s d,  rho_s = c2 w^2
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 24;
    const double *u, *d, *v;
    double s, c2, t;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        const double w = ::fma(s, d[i], u[i]);
        const double rho = c2 * w * w;
        const double vl = rho > 0.0 ? v_local(rho) : 0.0;
        acc[0] = ::fma((vl + v[i]) * w, ::fma(-t, w, d[i]), acc[0]);
    }
};

struct StepOp {         // u <- c (u + s d)
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 24;
    double *u;
    const double *d;
    double s, c;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { u[i] = c * ::fma(s, d[i], u[i]); }
};

// electrostatics inside U ------------------------------------------------
struct SrcOp {          // g = 4 pi a b (the source of the field of a b)
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 24;
    const double *a, *b;
    double *g;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { g[i] = 4.0 * kPi * a[i] * b[i]; }
};

struct ZeroVecOp {
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 8;
    double *x;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { x[i] = 0.0; }
};

struct PotPrepOp {      // P = v + phi[b], V = P + Q0
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 40;
    const double *v, *pb, *q0;
    double *P, *V;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double p = v[i] + pb[i];
        P[i] = p;
        V[i] = p + q0[i];
    }
};

struct EvalHOp {        // EvalOp with the potential of the probe: P + c2 (Q0 + 2 s Q1 + s^2 Q2)
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 48;
    const double *u, *d, *P, *q0, *q1, *q2;
    double s, c2, t;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        const double w = ::fma(s, d[i], u[i]);
        const double rho = c2 * w * w;
        const double vl = rho > 0.0 ? v_local(rho) : 0.0;
        const double vs = ::fma(c2, ::fma(s, ::fma(s, q2[i], 2.0 * q1[i]), q0[i]), P[i]);
        acc[0] = ::fma((vl + vs) * w, ::fma(-t, w, d[i]), acc[0]);
    }
};

struct StepHOp {        // u <- c (u + s d); Q0 <- c^2 (Q0 + 2 s Q1 + s^2 Q2); V = P + Q0
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 72;
    double *u, *q0, *V;
    const double *d, *q1, *q2, *P;
    double s, c;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        u[i] = c * ::fma(s, d[i], u[i]);
        const double q = c * c * ::fma(s, ::fma(s, q2[i], 2.0 * q1[i]), q0[i]);
        q0[i] = q;
        V[i] = P[i] + q;
    }
};

template <class Load, class Epi>
int stencil_pass(const ofdft_grid &g, const Coef<double> &c, const Load &ld, const Epi &ep, hipStream_t s,
                 int bytes_per_point) {
    ProfScope ps(K_U_STENCIL, (double)npoints(g) * bytes_per_point, s);
    return launch_stencil<double>(g, c, ld, ep, s);
}

int fetch(ofdft_scf *s, int first, int count, hipStream_t st) {
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->hsc + first, s->dsc + first, sizeof(double) * count,
                                   hipMemcpyDeviceToHost, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    return OFDFT_OK;
}

// Brent's method for a root of f on [a, b] with f(a) f(b) <= 0 (Brent 1973:
// bisection safeguarding secant / inverse quadratic interpolation steps).
// Stops when the bracket is below tol or when |f| <= ftol at the iterate.
template <class F>
int brent_root(F &&f, double a, double b, double fa, double fb, double tol, double ftol, int maxit,
               double &root) {
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < maxit; ++it) {
        if ((fb > 0) == (fc > 0)) {
            c = a;
            fc = fa;
            d = e = b - a;
        }
        if (std::fabs(fc) < std::fabs(fb)) {
            a = b; b = c; c = a;
            fa = fb; fb = fc; fc = fa;
        }
        const double tol1 = 2.0 * 2.220446049250313e-16 * std::fabs(b) + 0.5 * tol;
        const double xm = 0.5 * (c - b);
        if (std::fabs(xm) <= tol1 || std::fabs(fb) <= ftol) {
            root = b;
            return OFDFT_OK;
        }
        if (std::fabs(e) >= tol1 && std::fabs(fa) > std::fabs(fb)) {
            double p, q, r;
            const double sr = fb / fa;
            if (a == c) {
                p = 2.0 * xm * sr;
                q = 1.0 - sr;
            } else {
                q = fa / fc;
                r = fb / fc;
                p = sr * (2.0 * xm * q * (q - r) - (b - a) * (r - 1.0));
                q = (q - 1.0) * (r - 1.0) * (sr - 1.0);
            }
            if (p > 0) q = -q;
            p = std::fabs(p);
            if (2.0 * p < std::min(3.0 * xm * q - std::fabs(tol1 * q), std::fabs(e * q))) {
                e = d;
                d = p / q;
            } else {
                d = xm;
                e = d;
            }
        } else {
            d = xm;
            e = d;
        }
        a = b;
        fa = fb;
        b += std::fabs(d) > tol1 ? d : (xm > 0 ? tol1 : -tol1);
        int st = f(b, fb);
        if (st != OFDFT_OK) return st;
    }
    root = b;
    return OFDFT_OK;
}

// ---- device-driven iteration ---------------------------------------------
constexpr int kProbes = 10;        // line-search evaluations per iteration
constexpr int kBlockIters = 4;     // iterations per captured block (even: r, d in A; odd: in B)

enum { U_RUN = 0, U_CONVERGED = 1, U_STOPPED = 2, U_NONFINITE = 3 };

struct UDev {
    double uhu, ulu, uu, eta, rr, rrp;          // Ka, Kb totals
    double dots[5], kd[5], eval;                // preconditioner dots, direction totals, probe total
    double res, xi, cu, rz, rz_prev, rr_prev;
    double ud, dd, uLd, dLd, dHu, f0, f0_prev, s_prev;
    double lo, flo, hi, fhi, s, ftol, sstar, c; // line search
    double ba, bb, bc, bfa, bfb, bfc, bd, be, btol;   // Brent's method inside the bracket
    int q, done, skipit, ls_done, phase, probes, restart;
    int n_ka, n_kb, n_dots, n_kd, n_eval, n_step;   // passes that did work
};

struct UPar {
    double ne, dv, lam, tol, sqn, ltol, stol;
    int maxit, nres, pre;
};

struct EpiHuD {          // EpiHu with the totals into UDev
    const double *__restrict__ v;
    double *__restrict__ Hu;
    UDev *U;
    double *partials;
    unsigned int *counter;
    double half_lam, inv_ne_dv;
    double a0, a1, a2;
    double vv[4];
    __device__ bool skip() const { return U->done != U_RUN; }
    __device__ void pre(int q, int64_t i) { vv[q] = v[i]; }
    __device__ void point(int q, int64_t i, double c, double s) {
        const double rho = c * c;
        const double vl = rho > 0.0 ? v_local(rho) : 0.0;
        const double hu = ::fma(-half_lam, s, (vl + vv[q]) * c);
        Hu[i] = hu;
        a0 = ::fma(c, hu, a0);
        a1 = ::fma(c, s, a1);
        a2 = ::fma(c, c, a2);
    }
    __device__ void finish(int block, int nblocks, double *scratch) {
        double x[3] = {a0, a1, a2};
        block_sum<3>(x, scratch);
        double t[3];
        if (reduce_grid<3>(x, partials, nblocks, block, counter, scratch, t)) {
            U->uhu = t[0];
            U->ulu = t[1];
            U->uu = t[2];
            U->eta = t[0] * inv_ne_dv;
            U->n_ka += 1;
        }
    }
};

struct ResidOpD {        // r = -2 (Hu - eta u); {<r,r>, <r,r_prev>}
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 0;     // counted from the passes that did work
    const double *Hu, *u, *r_prev;
    double *r;
    UDev *U;
    double eta;
    int have_prev;
    __device__ bool skip() const { return U->done != U_RUN; }
    __device__ void prepare() {
        eta = U->eta;
        have_prev = U->q > 0;
    }
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const double ri = -2.0 * (Hu[i] - eta * u[i]);
        r[i] = ri;
        acc[0] = ::fma(ri, ri, acc[0]);
        if (have_prev) acc[1] = ::fma(ri, r_prev[i], acc[1]);
    }
};
struct FinRR {
    UDev *U;
    __device__ void operator()(const double (&t)[2]) const {
        U->rr = t[0];
        U->rrp = t[1];
        U->n_kb += 1;
    }
};

struct DotsOpD {         // {<u,z>, <r,z>, <r_prev,z>, <u,r>, <u,r_prev>}
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 0;     // counted from the passes that did work
    const double *u, *z, *r, *r_prev;
    UDev *U;
    int have_prev;
    __device__ bool skip() const { return U->done != U_RUN; }
    __device__ void prepare() { have_prev = U->q > 0; }
    __device__ void operator()(int64_t i, double (&acc)[5]) const {
        const double ui = u[i], zi = z[i], ri = r[i];
        acc[0] = ::fma(ui, zi, acc[0]);
        acc[1] = ::fma(ri, zi, acc[1]);
        acc[3] = ::fma(ui, ri, acc[3]);
        if (have_prev) {
            const double pi = r_prev[i];
            acc[2] = ::fma(pi, zi, acc[2]);
            acc[4] = ::fma(ui, pi, acc[4]);
        }
    }
};
struct FinDots {
    UDev *U;
    __device__ void operator()(const double (&t)[5]) const {
        for (int k = 0; k < 5; ++k) U->dots[k] = t[k];
        U->n_dots += 1;
    }
};

struct LoadDirD {        // d' = r + xi d_prev, xi from the device state
    const double *__restrict__ r;
    const double *__restrict__ d_prev;
    const UDev *U;
    double xi;
    __device__ void prepare() {
        xi = U->xi;
        if (xi == 0.0) d_prev = r;
    }
    __device__ double operator()(int64_t i) const { return ::fma(xi, d_prev[i], r[i]); }
};

struct EpiLdD {          // EpiLd with cu and the totals in UDev
    const double *__restrict__ u;
    const double *__restrict__ Hu;
    double *__restrict__ d;
    UDev *U;
    double *partials;
    unsigned int *counter;
    double cu;
    double a0, a1, a2, a3, a4;
    double uv[4], hv[4];
    __device__ bool skip() const { return U->done != U_RUN; }
    __device__ void prepare() { cu = U->cu; }
    __device__ void pre(int q, int64_t i) {
        uv[q] = u[i];
        hv[q] = Hu[i];
    }
    __device__ void point(int q, int64_t i, double c, double s) {
        const double ui = uv[q];
        d[i] = ::fma(-cu, ui, c);
        a0 = ::fma(ui, c, a0);
        a1 = ::fma(c, c, a1);
        a2 = ::fma(ui, s, a2);
        a3 = ::fma(c, s, a3);
        a4 = ::fma(hv[q], c, a4);
    }
    __device__ void finish(int block, int nblocks, double *scratch) {
        double x[5] = {a0, a1, a2, a3, a4};
        block_sum<5>(x, scratch);
        double t[5];
        if (reduce_grid<5>(x, partials, nblocks, block, counter, scratch, t)) {
            for (int k = 0; k < 5; ++k) U->kd[k] = t[k];
            U->n_kd += 1;
        }
    }
};

struct EvalOpD {         // EvalOp at the probe point U->s
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 0;     // counted from the passes that did work
    const double *u, *d, *v;
    UDev *U;
    double ne_dv;
    double s, c2, t;
    __device__ bool skip() const { return U->done != U_RUN || U->skipit || U->ls_done; }
    __device__ void prepare() {
        s = U->s;
        const double ww = U->uu + s * (2.0 * U->ud + s * U->dd);
        t = (U->ud + s * U->dd) / ww;
        c2 = ne_dv / ww;
    }
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        const double w = ::fma(s, d[i], u[i]);
        const double rho = c2 * w * w;
        const double vl = rho > 0.0 ? v_local(rho) : 0.0;
        acc[0] = ::fma((vl + v[i]) * w, ::fma(-t, w, d[i]), acc[0]);
    }
};
struct FinEval {
    UDev *U;
    __device__ void operator()(const double (&t)[1]) const {
        U->eval = t[0];
        U->n_eval += 1;
    }
};

struct StepOpD {         // u <- c (u + s* d)
    static constexpr int kClass = K_U_VECTOR;
    static constexpr int kBytes = 0;     // counted from the passes that did work
    double *u;
    const double *d;
    UDev *U;
    double s, c;
    __device__ bool skip() const { return U->done != U_RUN || U->skipit; }
    __device__ void prepare() {
        s = U->sstar;
        c = U->c;
    }
    __device__ void operator()(int64_t i, double (&)[1]) const { u[i] = c * ::fma(s, d[i], u[i]); }
};
struct FinStep {
    UDev *U;
    __device__ void operator()(const double (&)[1]) const { U->n_step += 1; }
};

// residual test (after Ka, Kb)
__global__ void u_check(UDev *U, UPar P) {
    if (U->done != U_RUN) return;
    const double res = 0.5 * sqrt(U->rr / U->uu);
    U->res = res;
    if (!isfinite(res)) U->done = U_NONFINITE;
    else if (res <= P.tol) U->done = U_CONVERGED;
    else if (U->q >= P.maxit) U->done = U_STOPPED;
}

// Polak-Ribiere coefficient and the projection coefficient (after the dots)
__global__ void u_direction(UDev *U, UPar P) {
    if (U->done != U_RUN) return;
    double xi = 0.0, cu = 0.0, rz = 0.0;
    if (P.pre) {
        cu = U->dots[0] / U->uu;
        rz = U->dots[1] - cu * U->dots[3];
        if (U->q > 0) xi = (rz - (U->dots[2] - cu * U->dots[4])) / U->rz_prev;
        if (!isfinite(rz) || !(rz > 0.0)) {
            U->done = U_NONFINITE;
            return;
        }
    } else if (U->q > 0) {
        xi = (U->rr - U->rrp) / U->rr_prev;
    }
    if (U->q % P.nres == 0 || !(xi > 0.0) || U->restart) xi = 0.0;
    U->restart = 0;
    U->xi = xi;
    U->cu = cu;
    U->rz = rz;
}

__device__ inline void u_accept(UDev *U, const UPar &P, double x) {
    U->sstar = x;
    U->ls_done = 1;
    const double ww = U->uu + x * (2.0 * U->ud + x * U->dd);
    U->c = P.sqn / sqrt(P.dv * ww);
}

// slope at s = 0 from the direction totals; line-search start (after Kd)
__global__ void u_slope0(UDev *U, UPar P) {
    if (U->done != U_RUN) return;
    const double cu = U->cu, uu = U->uu, ulu = U->ulu, uhu = U->uhu;
    const double *t = U->kd;
    const double ud = t[0] - cu * uu, dd = t[1] - 2.0 * cu * t[0] + cu * cu * uu;
    const double uLd = t[2] - cu * ulu, dLd = t[3] - 2.0 * cu * t[2] + cu * cu * ulu;
    const double dHu = t[4] - cu * uhu;
    U->ud = ud;
    U->dd = dd;
    U->uLd = uLd;
    U->dLd = dLd;
    U->dHu = dHu;
    U->skipit = 0;
    U->ls_done = 0;
    if (!(dd > 0.0)) {
        U->done = U_STOPPED;
        return;
    }
    const double f0 = P.ne / (P.dv * uu) * (dHu - ud / uu * uhu);
    U->f0 = f0;
    if (!(f0 < 0.0)) {
        if (U->xi != 0.0) {          // not a descent direction: restart along r next iteration
            U->restart = 1;
            U->skipit = 1;
        } else {
            U->done = U_STOPPED;     // no descent possible at this precision
        }
        return;
    }
    const double sp = U->s_prev;
    double hi = sp > 0.0 ? sp : 1.0 / sqrt(fmax(dd * P.dv / P.ne, 1e-300));
    if (sp > 0.0 && U->f0_prev < 0.0) hi = sp * fmin(fmax(U->f0_prev / f0, 0.1), 10.0);
    U->lo = 0.0;
    U->flo = f0;
    U->hi = hi;
    U->s = hi;
    U->ftol = P.stol * fabs(f0);
    U->phase = 0;
    U->probes = 0;
}

// One step of Brent's method (Brent 1973: bisection safeguarding secant and
// inverse quadratic interpolation steps) on the state after f(b) is known,
// the same arithmetic as brent_root; true when b is accepted, else b is the
// next point to evaluate.
__device__ bool brent_decide(UDev *U) {
    double a = U->ba, b = U->bb, c = U->bc, fa = U->bfa, fb = U->bfb, fc = U->bfc, d = U->bd, e = U->be;
    if ((fb > 0) == (fc > 0)) {
        c = a;
        fc = fa;
        d = e = b - a;
    }
    if (fabs(fc) < fabs(fb)) {
        a = b; b = c; c = a;
        fa = fb; fb = fc; fc = fa;
    }
    const double tol1 = 2.0 * 2.220446049250313e-16 * fabs(b) + 0.5 * U->btol;
    const double xm = 0.5 * (c - b);
    bool accepted = false;
    if (fabs(xm) <= tol1 || fabs(fb) <= U->ftol) {
        accepted = true;
    } else {
        if (fabs(e) >= tol1 && fabs(fa) > fabs(fb)) {
            double p, q, r;
            const double sr = fb / fa;
            if (a == c) {
                p = 2.0 * xm * sr;
                q = 1.0 - sr;
            } else {
                q = fa / fc;
                r = fb / fc;
                p = sr * (2.0 * xm * q * (q - r) - (b - a) * (r - 1.0));
                q = (q - 1.0) * (r - 1.0) * (sr - 1.0);
            }
            if (p > 0) q = -q;
            p = fabs(p);
            if (2.0 * p < fmin(3.0 * xm * q - fabs(tol1 * q), fabs(e * q))) {
                e = d;
                d = p / q;
            } else {
                d = xm;
                e = d;
            }
        } else {
            d = xm;
            e = d;
        }
        a = b;
        fa = fb;
        b += fabs(d) > tol1 ? d : (xm > 0 ? tol1 : -tol1);
    }
    U->ba = a; U->bb = b; U->bc = c;
    U->bfa = fa; U->bfb = fb; U->bfc = fc;
    U->bd = d; U->be = e;
    return accepted;
}

// one line-search decision after a probe: grow the bracket (secant past the
// estimated root, 1.1x to 8x) while the slope stays negative, then Brent's
// method inside it (the host form's search, one evaluation per probe)
__global__ void u_linesearch(UDev *U, UPar P) {
    if (U->done != U_RUN || U->skipit || U->ls_done) return;
    const double sv = U->s;
    const double ww = U->uu + sv * (2.0 * U->ud + sv * U->dd);
    const double t = (U->ud + sv * U->dd) / ww;
    const double c2 = P.ne / (P.dv * ww);
    const double vw = U->uLd + sv * U->dLd - t * (U->ulu + sv * (2.0 * U->uLd + sv * U->dLd));
    const double f = c2 * (U->eval - 0.5 * P.lam * vw);
    U->probes += 1;
    if (!isfinite(f)) {
        U->done = U_NONFINITE;
        return;
    }
    if (U->phase == 0) {
        if (fabs(f) <= U->ftol) {
            u_accept(U, P, sv);
            return;
        }
        const double lo = U->lo, flo = U->flo, hi = U->hi, fhi = f;
        if (fhi < 0.0) {
            double next = 2.0 * hi;
            if (fhi > flo) {
                const double sec = hi + (hi - lo) * (-fhi) / (fhi - flo);
                next = fmin(fmax(1.1 * sec, 1.1 * hi), 8.0 * hi);
            }
            U->lo = hi;
            U->flo = fhi;
            U->hi = next;
            U->s = next;
            return;
        }
        // bracketed: Brent from (lo, hi)
        U->phase = 1;
        U->ba = lo;
        U->bfa = flo;
        U->bb = hi;
        U->bfb = fhi;
        U->bc = lo;
        U->bfc = flo;
        U->bd = U->be = hi - lo;
        U->btol = P.ltol * hi;
    } else {
        U->bfb = f;
    }
    if (brent_decide(U)) u_accept(U, P, U->bb);
    else U->s = U->bb;
}

// budget spent without acceptance: the last point of negative slope while
// still growing, else Brent's current point inside the bracket
__global__ void u_linesearch_end(UDev *U, UPar P) {
    if (U->done != U_RUN || U->skipit || U->ls_done) return;
    u_accept(U, P, U->phase == 0 ? U->lo : U->bb);
}

// end of an iteration
__global__ void u_end(UDev *U) {
    if (U->done != U_RUN) return;
    if (!U->skipit) {
        U->s_prev = fabs(U->sstar);
        U->f0_prev = U->f0;
        U->rr_prev = U->rr;
        U->rz_prev = U->rz;
        U->q += 1;
    }
    U->skipit = 0;
}

// one iteration; parity 0 keeps r and d in rA/dA (previous in rB/dB), 1 the reverse
int u_iteration(ofdft_scf *s, const double *v, double *u, int parity, const UPar &P, hipStream_t st) {
    const ofdft_grid &g = s->g;
    const int64_t n = s->n;
    UDev *U = (UDev *)s->udev;
    double *r_cur = parity ? s->rB : s->rA, *r_prev = parity ? s->rA : s->rB;
    double *d_cur = parity ? s->dB : s->dA, *d_prev = parity ? s->dA : s->dB;
    {
        ProfScope ps(K_U_STENCIL, 0.0, st);
        OFDFT_TRY(launch_stencil<double>(g, s->coef, LoadPlain<double>{u},
                                         EpiHuD{v, s->Hu, U, s->rb.partials, s->rb.counter, 0.5 * P.lam,
                                                P.dv / P.ne, 0, 0, 0, {}},
                                         st));
    }
    OFDFT_TRY((launch_reduce<2>(n, ResidOpD{s->Hu, u, r_prev, r_cur, U, 0.0, 0}, FinRR{U}, s->rb, st)));
    hipLaunchKernelGGL(u_check, dim3(1), dim3(1), 0, st, U, P);
    OFDFT_CHECK_HIP(hipGetLastError());
    const double *base = r_cur;
    if (P.pre) {
        OFDFT_TRY(mg_apply_run(*s->umg, r_cur, s->z, st, s->u_kappa, &U->done));
        OFDFT_TRY((launch_reduce<5>(n, DotsOpD{u, s->z, r_cur, r_prev, U, 0}, FinDots{U}, s->rb, st)));
        base = s->z;
    }
    hipLaunchKernelGGL(u_direction, dim3(1), dim3(1), 0, st, U, P);
    OFDFT_CHECK_HIP(hipGetLastError());
    {
        ProfScope ps(K_U_STENCIL, 0.0, st);
        OFDFT_TRY(launch_stencil<double>(g, s->coef, LoadDirD{base, d_prev, U, 0.0},
                                         EpiLdD{u, s->Hu, d_cur, U, s->rb.partials, s->rb.counter, 0.0, 0, 0, 0, 0,
                                                0, {}, {}},
                                         st));
    }
    hipLaunchKernelGGL(u_slope0, dim3(1), dim3(1), 0, st, U, P);
    OFDFT_CHECK_HIP(hipGetLastError());
    for (int k = 0; k < kProbes; ++k) {
        OFDFT_TRY((launch_reduce<1>(n, EvalOpD{u, d_cur, v, U, P.ne / P.dv, 0.0, 0.0, 0.0}, FinEval{U}, s->rb, st)));
        hipLaunchKernelGGL(u_linesearch, dim3(1), dim3(1), 0, st, U, P);
        OFDFT_CHECK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(u_linesearch_end, dim3(1), dim3(1), 0, st, U, P);
    OFDFT_CHECK_HIP(hipGetLastError());
    OFDFT_TRY((launch_reduce<1>(n, StepOpD{u, d_cur, U, 0.0, 0.0}, FinStep{U}, s->rb, st)));
    hipLaunchKernelGGL(u_end, dim3(1), dim3(1), 0, st, U);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

int u_graph_get(ofdft_scf *s, const double *v, double *u, const UPar &P) {
    const void *key[3] = {v, u, s->udev};
    if (s->ugraph && std::equal(key, key + 3, s->ugraph_key)) return OFDFT_OK;
    if (s->ugraph) {
        (void)hipGraphExecDestroy(s->ugraph);
        s->ugraph = nullptr;
    }
    if (!s->ucap) OFDFT_CHECK_HIP(hipStreamCreateWithFlags(&s->ucap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    OFDFT_CHECK_HIP(hipStreamBeginCapture(s->ucap, hipStreamCaptureModeThreadLocal));
    prof_suspend(true);
    int rc = OFDFT_OK;
    for (int k = 0; k < kBlockIters && rc == OFDFT_OK; ++k) rc = u_iteration(s, v, u, k & 1, P, s->ucap);
    prof_suspend(false);
    const hipError_t e = hipStreamEndCapture(s->ucap, &graph);
    if (rc != OFDFT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    OFDFT_CHECK_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&s->ugraph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    OFDFT_CHECK_HIP(ei);
    for (int i = 0; i < 3; ++i) s->ugraph_key[i] = key[i];
    return OFDFT_OK;
}

int density_update_dev(ofdft_scf *s, const double *v, double *u, int &iters, double &res, double &eta,
                       hipStream_t st) {
    if (!s->udev) {
        OFDFT_CHECK_HIP(hipMalloc(&s->udev, sizeof(UDev)));
        OFDFT_CHECK_HIP(hipHostMalloc(&s->udev_h, sizeof(UDev), hipHostMallocDefault));
    }
    UDev *Uh = (UDev *)s->udev_h;
    UPar P{};
    P.ne = s->p.n_electrons;
    P.dv = s->dv;
    P.lam = s->p.lambda;
    P.tol = s->p.u_tol;
    P.sqn = std::sqrt(P.ne);
    P.ltol = s->p.line_tol > 0.0 ? s->p.line_tol : 1e-8;
    P.stol = s->p.line_slope_tol > 0.0 ? s->p.line_slope_tol : 1e-6;
    P.maxit = s->p.u_max_iter > 0 ? s->p.u_max_iter : 20000;
    P.nres = s->p.n_restart > 0 ? s->p.n_restart : 50;
    P.pre = s->umg != nullptr;
    *Uh = UDev{};
    Uh->s_prev = s->s_prev;
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->udev, Uh, sizeof(UDev), hipMemcpyHostToDevice, st));
    const bool eager = prof_timed(K_U_STENCIL) || prof_timed(K_U_VECTOR) || (P.pre && prof_timed(K_MULTIGRID));
    auto read_state = [&]() -> int {
        OFDFT_CHECK_HIP(hipMemcpyAsync(Uh, s->udev, sizeof(UDev), hipMemcpyDeviceToHost, st));
        OFDFT_CHECK_HIP(hipStreamSynchronize(st));
        return OFDFT_OK;
    };
    // every iteration either steps (q grows) or restarts once; the cap is a guard
    const int64_t cap = 2 * (int64_t)P.maxit + 8;
    if (eager) {
        for (int64_t k = 0; k < cap; ++k) {
            OFDFT_TRY(u_iteration(s, v, u, (int)(k & 1), P, st));
            OFDFT_TRY(read_state());
            if (Uh->done != U_RUN) break;
        }
    } else {
        OFDFT_TRY(u_graph_get(s, v, u, P));
        for (int64_t k = 0; k < cap; k += kBlockIters) {
            OFDFT_CHECK_HIP(hipGraphLaunch(s->ugraph, st));
            OFDFT_TRY(read_state());
            if (Uh->done != U_RUN) break;
        }
    }
    if (Uh->done == U_RUN) {
        set_error("ofdft_density_update: iteration guard reached");
        return OFDFT_HIP_ERROR;
    }
    // algorithmic bytes of the passes that did work (the early exits move none)
    const double nd = (double)s->n;
    const int64_t nst = Uh->n_ka + Uh->n_kd, nvec = Uh->n_kb + Uh->n_dots + Uh->n_eval + Uh->n_step;
    prof_add(K_U_STENCIL, nd * (24.0 * Uh->n_ka + 40.0 * Uh->n_kd), eager ? 0 : nst);
    prof_add(K_U_VECTOR, nd * (32.0 * Uh->n_kb + 32.0 * Uh->n_dots + 24.0 * Uh->n_eval + 24.0 * Uh->n_step),
             eager ? 0 : nvec);
    if (P.pre) prof_add(K_MULTIGRID, mg_cycle_bytes(*s->umg) * Uh->n_dots, eager ? 0 : Uh->n_dots);
    s->s_prev = Uh->s_prev;
    iters = Uh->q;
    res = Uh->res;
    eta = Uh->eta;
    if (Uh->done == U_NONFINITE) return OFDFT_NONFINITE;
    return Uh->done == U_CONVERGED ? OFDFT_OK : OFDFT_NOT_CONVERGED;
}

}  // namespace

void density_free(ofdft_scf *s) {
    if (s->ugraph) (void)hipGraphExecDestroy(s->ugraph);
    if (s->ucap) (void)hipStreamDestroy(s->ucap);
    if (s->udev) (void)hipFree(s->udev);
    if (s->udev_h) (void)hipHostFree(s->udev_h);
    s->ugraph = nullptr;
    s->ucap = nullptr;
    s->udev = s->udev_h = nullptr;
}

int density_update(ofdft_scf *s, const double *v, double *u, int &iters, double &res, double &eta,
                   hipStream_t st) {
    // the potential-mixing map runs device-driven; with the electrostatics
    // inside (Poisson solves between the passes) the host drives the loop
    if (s->p.fixed_point == 0) return density_update_dev(s, v, u, iters, res, eta, st);
    const ofdft_grid &g = s->g;
    const int64_t n = s->n;
    const double ne = s->p.n_electrons, dv = s->dv, lam = s->p.lambda;
    const double sqn = std::sqrt(ne);
    double *r_cur = s->rA, *r_prev = s->rB, *d_cur = s->dA, *d_prev = s->dB;
    double *tot = s->dsc + 16;          // Kd totals
    const bool pre = s->umg != nullptr;
    int q = 0;
    double rr_prev = 0.0, rz_prev = 0.0;
    res = INFINITY;
    eta = 0.0;
    double s_prev = s->s_prev;
    double f0_prev = 0.0;                        // slope at s = 0 of the previous iteration
    const int maxit = s->p.u_max_iter > 0 ? s->p.u_max_iter : 20000;
    const int nres = s->p.n_restart > 0 ? s->p.n_restart : 50;
    // electrostatics inside: the field of a b into x by the context's Poisson solver
    const bool hart = s->p.fixed_point == 1;
    int worst = OFDFT_OK;
    s->u_pois_it = 0;
    auto field = [&](const double *a, const double *b, double *x, bool zero) -> int {
        OFDFT_TRY((launch_reduce<1>(n, SrcOp{a, b, s->g4}, NoFin{}, s->rb, st)));
        if (zero) OFDFT_TRY((launch_reduce<1>(n, ZeroVecOp{x}, NoFin{}, s->rb, st)));
        ofdft_solve_stats ps{};
        const int pst = poisson_solve(s->pois, s->g4, x, s->p.poisson_tol, s->p.max_iter, ps, st);
        if (pst < 0) return pst;
        s->u_pois_it += ps.iters;
        worst = std::max(worst, pst);
        return OFDFT_OK;
    };
    if (hart) {
        OFDFT_TRY(field(u, u, s->hQ0, false));          // warm start: the previous field
        OFDFT_TRY((launch_reduce<1>(n, PotPrepOp{v, s->hPb, s->hQ0, s->hP, s->hV}, NoFin{}, s->rb, st)));
    }
    const double *vtot = hart ? s->hV : v;
    for (;;) {
        // Ka: H u
        OFDFT_TRY(stencil_pass(g, s->coef, LoadPlain<double>{u},
                               EpiHu{vtot, s->Hu, s->dsc, s->rb.partials, s->rb.counter, 0.5 * lam,
                                     dv / ne, 0, 0, 0},
                               st, 24));
        // Kb: r
        ResidOp ro{s->Hu, u, r_prev, r_cur, s->dsc, q > 0, 0.0};
        OFDFT_TRY((launch_reduce<2>(n, ro, StoreTotals<2>{s->dsc + S_RR}, s->rb, st)));
        OFDFT_TRY(fetch(s, 0, S_COUNT, st));
        const double *h = s->hsc;
        eta = h[S_ETA];
        const double rr = h[S_RR], uu = h[S_UU];
        res = 0.5 * std::sqrt(rr / uu);
        if (!std::isfinite(res)) return OFDFT_NONFINITE;
        if (res <= s->p.u_tol || q >= maxit) break;
        double xi = 0.0, cu = 0.0, rz = 0.0;
        const double *base = r_cur;
        if (pre) {
            // z = M r, then the Polak-Ribiere terms of the projected z~ = z - cu u
            OFDFT_TRY(mg_apply(*s->umg, r_cur, s->z, st, s->u_kappa));
            DotsOp dop{u, s->z, r_cur, r_prev, q > 0};
            OFDFT_TRY((launch_reduce<5>(n, dop, StoreTotals<5>{s->dsc + S_DOTS}, s->rb, st)));
            OFDFT_TRY(fetch(s, S_DOTS, 5, st));
            const double *t = s->hsc + S_DOTS;
            cu = t[0] / uu;
            rz = t[1] - cu * t[3];                                   // <r, z~>
            if (q > 0) xi = (rz - (t[2] - cu * t[4])) / rz_prev;     // <r - r_prev, z~> / <r_prev, z~_prev>
            if (!std::isfinite(rz) || !(rz > 0.0)) return OFDFT_NONFINITE;
            base = s->z;
        } else if (q > 0) {
            xi = (rr - h[S_RRP]) / rr_prev;    // <r - r_prev, r> / <r_prev, r_prev>
        }
        if (q % nres == 0 || !(xi > 0.0)) xi = 0.0;
        // Kd: d = r + xi d_prev (or z~ + xi d_prev), L d
        auto make_dir = [&](double xiv) -> int {
            OFDFT_TRY(stencil_pass(g, s->coef, LoadDir{base, d_prev, xiv},
                                   EpiLd{u, s->Hu, d_cur, tot, s->rb.partials, s->rb.counter, cu, 0, 0, 0, 0, 0},
                                   st, 40));
            OFDFT_CHECK_HIP(hipMemcpyAsync(s->hsc + 16, tot, sizeof(double) * 5, hipMemcpyDeviceToHost, st));
            OFDFT_CHECK_HIP(hipStreamSynchronize(st));
            return OFDFT_OK;
        };
        const double uLu = h[S_ULU], uHu = h[S_UHU];
        double ud, dd, uLd, dLd, dHu;
        // totals of d = d' - cu u from those of the loaded d'
        auto read_dir = [&]() {
            const double *t = s->hsc + 16;
            ud = t[0] - cu * uu;
            dd = t[1] - 2.0 * cu * t[0] + cu * cu * uu;
            uLd = t[2] - cu * uLu;
            dLd = t[3] - 2.0 * cu * t[2] + cu * cu * uLu;
            dHu = t[4] - cu * uHu;
        };
        OFDFT_TRY(make_dir(xi));
        read_dir();
        // slope at s = 0 from the direction pass (u is normalised, so c2 = N_e / (h^3 <u,u>))
        auto slope0 = [&]() { return ne / (dv * uu) * (dHu - ud / uu * uHu); };
        if (!(dd > 0.0)) break;
        // dE/ds (up to the positive factor 2 h^3)
        auto slope = [&](double sv, double &out) -> int {
            const double ww = uu + sv * (2.0 * ud + sv * dd);
            const double t = (ud + sv * dd) / ww;
            const double c2 = ne / (dv * ww);
            if (hart) {
                EvalHOp ev{u, d_cur, s->hP, s->hQ0, s->hQ1, s->hQ2, sv, c2, t};
                OFDFT_TRY((launch_reduce<1>(n, ev, StoreTotals<1>{s->dsc + S_EVAL}, s->rb, st)));
            } else {
                EvalOp ev{u, d_cur, v, sv, c2, t};
                OFDFT_TRY((launch_reduce<1>(n, ev, StoreTotals<1>{s->dsc + S_EVAL}, s->rb, st)));
            }
            OFDFT_TRY(fetch(s, S_EVAL, 1, st));
            const double vw = uLd + sv * dLd - t * (uLu + sv * (2.0 * uLd + sv * dLd));
            out = c2 * (s->hsc[S_EVAL] - 0.5 * lam * vw);
            return OFDFT_OK;
        };
        double f0 = slope0();
        if (!(f0 < 0.0) && xi != 0.0) {          // not a descent direction: restart along r
            xi = 0.0;
            OFDFT_TRY(make_dir(0.0));
            read_dir();
            f0 = slope0();
        }
        if (!(f0 < 0.0)) break;                  // no descent possible at this precision
        if (hart) {                              // the fields of u d and d^2 along this direction
            OFDFT_TRY(field(u, d_cur, s->hQ1, true));
            OFDFT_TRY(field(d_cur, d_cur, s->hQ2, true));
        }
        double lo = 0.0, flo = f0;
        // first probe: the previous step scaled by the ratio of the slopes at
        // s = 0 (the first-order decrease of the last step, repeated), kept
        // within 0.1x..10x of that step; with no history, the previous step
        // or a step of the size of u
        double hi = s_prev > 0 ? s_prev : 1.0 / std::sqrt(std::max(dd * dv / ne, 1e-300));
        if (s_prev > 0 && f0_prev < 0.0) hi = s_prev * std::min(std::max(f0_prev / f0, 0.1), 10.0);
        const double ltol = s->p.line_tol > 0.0 ? s->p.line_tol : 1e-8;
        const double stol = s->p.line_slope_tol > 0.0 ? s->p.line_slope_tol : 1e-6;
        const double ftol = stol * std::fabs(f0);
        double fhi;
        OFDFT_TRY(slope(hi, fhi));
        // Bracket the root of dE/ds: while the slope is still negative, step
        // just past the secant estimate of its zero (at least 1.1x, at most
        // 8x further), which the nearly linear slope usually brackets at once.
        // A probe whose slope is already within ftol is the accepted step.
        int grow = 0;
        while (fhi < 0.0 && std::fabs(fhi) > ftol && grow < 80) {
            double next = 2.0 * hi;
            if (fhi > flo) {
                const double sec = hi + (hi - lo) * (-fhi) / (fhi - flo);
                next = std::min(std::max(1.1 * sec, 1.1 * hi), 8.0 * hi);
            }
            lo = hi;
            flo = fhi;
            hi = next;
            OFDFT_TRY(slope(hi, fhi));
            ++grow;
        }
        if (!std::isfinite(fhi)) return OFDFT_NONFINITE;
        double sstar = hi;
        // the slope is reduced by stol at the accepted step (by default a
        // million-fold: an exact line search for NLCG purposes), or the
        // bracket is below ltol
        if (std::fabs(fhi) > ftol)
            OFDFT_TRY(brent_root(slope, lo, hi, flo, fhi, ltol * hi, ftol, 200, sstar));
        const double ww = uu + sstar * (2.0 * ud + sstar * dd);
        const double c = sqn / std::sqrt(dv * ww);
        if (hart) {
            StepHOp so{u, s->hQ0, s->hV, d_cur, s->hQ1, s->hQ2, s->hP, sstar, c};
            OFDFT_TRY((launch_reduce<1>(n, so, NoFin{}, s->rb, st)));
        } else {
            StepOp so{u, d_cur, sstar, c};
            OFDFT_TRY((launch_reduce<1>(n, so, NoFin{}, s->rb, st)));
        }
        s_prev = std::fabs(sstar);
        f0_prev = f0;
        rr_prev = rr;
        rz_prev = rz;
        std::swap(r_cur, r_prev);
        std::swap(d_cur, d_prev);
        ++q;
    }
    s->s_prev = s_prev;
    iters = q;
    // stopped by the iteration cap or by the lack of a descent direction
    // before the tolerance (or a Poisson solve inside missed its own): the
    // result is written, the status says so
    return std::max(res <= s->p.u_tol ? OFDFT_OK : OFDFT_NOT_CONVERGED, worst);
}

}  // namespace ofdft
