// ofdft_scf_step: one step of the fixed-point iteration (Section 3.3 and its
// flowchart; Appendix D), with mixing variable v = phi + mu V_LR:
//   u = U(v); phi = Poisson(4 pi (u^2 + b)); V_LR from the 8 K_00 shifted solves
//   (mu = 1); vhat = phi + mu V_LR; f = vhat - v; v <- Anderson(v, f).
// Kernel-term constants: K_00 row of the Appendix A table (r = 1, 3 printed;
// r = 2, 4 their complex conjugates), alpha = 5/6 + sqrt(5)/6,
// beta = 5/6 - sqrt(5)/6 (Section 5), kF = (3 pi^2 N_e / |Omega|)^{1/3}.
// With m = n = 0 the right-hand side of each shifted equation is
// P_r (-L_h rho^p) after multiplying through by (2 kF)^2, and
// kappa_r = (2 kF)^2 Q_r.  V_{beta,r} (solution for rho^beta) multiplies
// alpha rho^{alpha-1} in V_LR and V_{alpha,r} multiplies beta rho^{beta-1}.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "physics.hpp"
#include "scf.hpp"

namespace ofdft {

namespace {

const double kAlpha = 5.0 / 6.0 + 0.37267799624996495;   // sqrt(5)/6
const double kBeta = 5.0 / 6.0 - 0.37267799624996495;
const double kP00[4][2] = {{0.108403, 0.079657}, {0.108403, -0.079657},
                           {-0.908403, 0.439708}, {-0.908403, -0.439708}};
const double kQ00[4][2] = {{-0.470923, -0.465392}, {-0.470923, 0.465392},
                           {0.066051, -0.259678}, {0.066051, 0.259678}};

struct PoissonRhsOp {   // g = 4 pi (u^2 + b)
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24;
    const double *u, *b;
    double *g;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double ui = u[i];
        g[i] = 4.0 * kPi * ::fma(ui, ui, b[i]);
    }
};

struct PowersOp {       // rho^alpha, rho^beta
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24;
    const double *u;
    double *ra, *rb;
    double a, bb;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double rho = u[i] * u[i];
        ra[i] = rho > 0.0 ? pow(rho, a) : 0.0;
        rb[i] = rho > 0.0 ? pow(rho, bb) : 0.0;
    }
};

// The K_00 row of Appendix A lists r = 2, 4 as the complex conjugates of
// r = 1, 3 (both P and Q).  With a real density the right-hand sides of
// systems r = 2, 4 are then the conjugates of those of r = 1, 3, and so are
// their solutions: only systems 0, 2, 4, 6 (r = 1, 3 for beta and alpha) are
// solved; 1, 3, 5, 7 are their conjugates.
struct ShiftRhsOp {     // F_j = P_r f_beta (j = 0, 2), P_r f_alpha (j = 4, 6), r = j % 4
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 80;
    const double *fa, *fb;
    double2 *F0, *F2, *F4, *F6;
    double pr[4], pi[4];
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double b_ = fb[i], a_ = fa[i];
        F0[i] = make_double2(pr[0] * b_, pi[0] * b_);
        F2[i] = make_double2(pr[2] * b_, pi[2] * b_);
        F4[i] = make_double2(pr[0] * a_, pi[0] * a_);
        F6[i] = make_double2(pr[2] * a_, pi[2] * a_);
    }
};

struct BaseRhsOp {      // complex128 copies of the base right-hand sides f_beta, f_alpha
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 48;
    const double *fa, *fb;
    double2 *Fb, *Fa;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        Fb[i] = make_double2(fb[i], 0.0);
        Fa[i] = make_double2(fa[i], 0.0);
    }
};

struct ScaleConjOp {    // V_j = P_r U_j in place (r = j % 4), V_{j+1} = conj(V_j), j = 0, 2, 4, 6
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 192;
    double2 *V0, *V2, *V4, *V6;
    double2 *V1, *V3, *V5, *V7;
    double2 P0, P2;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double2 a = cmul(P0, V0[i]), b = cmul(P2, V2[i]), c = cmul(P0, V4[i]), d = cmul(P2, V6[i]);
        V0[i] = a;
        V2[i] = b;
        V4[i] = c;
        V6[i] = d;
        V1[i] = make_double2(a.x, -a.y);
        V3[i] = make_double2(b.x, -b.y);
        V5[i] = make_double2(c.x, -c.y);
        V7[i] = make_double2(d.x, -d.y);
    }
};

struct ConjOp {         // V_{j+1} = conj(V_j), j = 0, 2, 4, 6
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 128;
    const double2 *V0, *V2, *V4, *V6;
    double2 *V1, *V3, *V5, *V7;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double2 a = V0[i], b = V2[i], c = V4[i], d = V6[i];
        V1[i] = make_double2(a.x, -a.y);
        V3[i] = make_double2(b.x, -b.y);
        V5[i] = make_double2(c.x, -c.y);
        V7[i] = make_double2(d.x, -d.y);
    }
};

// V_LR = C_F Re sum_r [alpha rho^(alpha-1) V_beta,r + beta rho^(beta-1) V_alpha,r];
// Re V_{r=2} = Re V_{r=1} and Re V_{r=4} = Re V_{r=3} (conjugate pairs).
struct VlrOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 80;
    const double *u;
    const double2 *V0, *V2, *V4, *V6;
    double *vlr;
    double floor_rho, a, bb;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double rho = fmax(u[i] * u[i], floor_rho);
        const double vb = 2.0 * (V0[i].x + V2[i].x);
        const double va = 2.0 * (V4[i].x + V6[i].x);
        vlr[i] = kCF * (a * pow(rho, a - 1.0) * vb + bb * pow(rho, bb - 1.0) * va);
    }
};

// ---------------------------------------------------------------------------
// Order-2 kernel terms (Section 2, the Taylor expansion of the density-
// dependent kernel about rho_bar with C_mnpq = (-1)^(p+q) / (m! n!)
// binom(m,p) binom(n,q) rho_bar^(p+q-m-n); Section 3.1, the local form;
// Appendix A, P and Q of K_00, K_10, K_20, K_11 for r = 1, 3, with
// P_mn = P_nm, Q_mn = Q_nm and r = 2, 4 the conjugates).  The pairs with
// m + n <= 2 are the ones the table covers.  Q_11 for r = 1 is printed with an
// imaginary part of -0.0266195, one digit more than every other entry; it is
// read as -0.266195, next to K_20's -0.233840 (the smaller value would place
// the shift almost on the real axis inside the spectrum of -L_h).
// K_mn rho^a = sum_r V_r with (-L_h + kappa_r) V_r = (2 kF)^2 P_r rho^a for
// m + n > 0 and P_r (-L_h rho^a) for K_00, kappa_r = (2 kF)^2 Q_r; with a
// real rho the r = 2, 4 solutions are conjugates of r = 1, 3, so the sum is
// W = 2 Re(V_1 + V_3).
//   V_LR = C_F sum_{m,n,p,q} C_mnpq [ (m-p+alpha) rho^(m-p+alpha-1) K_mn rho^(n-q+beta)
//                                   + (n-q+beta) rho^(n-q+beta-1) K_mn rho^(m-p+alpha) ].
struct LrKernel {
    int m, n;
    double P[2][2], Q[2][2];     // r = 1, 3: {re, im}
};
const LrKernel kLrTable[4] = {
    {0, 0, {{0.108403, 0.079657}, {-0.908403, 0.439708}}, {{-0.470923, -0.465392}, {0.066051, -0.259678}}},
    {1, 0, {{-0.030515, 0.015027}, {0.028915, -0.008817}}, {{-0.597793, -0.294130}, {-0.087917, -0.164937}}},
    {2, 0, {{0.008907, -0.032841}, {-0.034974, 0.009116}}, {{-0.537986, -0.233840}, {-0.041565, -0.196662}}},
    {1, 1, {{0.012423, -0.034421}, {-0.031907, 0.007392}}, {{-0.511699, -0.266195}, {-0.034031, -0.188927}}},
};

double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}
double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }

// The distinct convolutions and the V_LR terms of the order-L expansion
// (L = 0 or 2), in the documented order.
// eterms: the kernel energy C_F sum C_mnpq <rho^(m-p+alpha), K_mn rho^(n-q+beta)>
// as coef <rho^e, W_conv> terms.
void lr_setup(int L, double rho_bar, std::vector<LrConv> &conv, std::vector<LrTerm> &terms,
              std::vector<LrTerm> &eterms) {
    conv.clear();
    terms.clear();
    eterms.clear();
    auto conv_index = [&](int m, int n, double a) {
        const int km = std::max(m, n), kn = std::min(m, n);
        for (size_t c = 0; c < conv.size(); ++c)
            if (conv[c].m == km && conv[c].n == kn && std::fabs(conv[c].a - a) < 1e-12) return (int)c;
        LrConv e{km, kn, a, {}, {}};
        for (const LrKernel &k : kLrTable)
            if (k.m == km && k.n == kn)
                for (int r = 0; r < 2; ++r) {
                    e.P[r] = make_double2(k.P[r][0], k.P[r][1]);
                    e.Q[r] = make_double2(k.Q[r][0], k.Q[r][1]);
                }
        conv.push_back(e);
        return (int)conv.size() - 1;
    };
    for (int m = 0; m <= L; ++m)
        for (int n = 0; n <= L; ++n) {
            if (m + n > L) continue;
            for (int p = 0; p <= m; ++p)
                for (int q = 0; q <= n; ++q) {
                    const double a = m - p + kAlpha, b = n - q + kBeta;
                    const int cb = conv_index(m, n, b), ca = conv_index(m, n, a);
                    const double c = ((p + q) % 2 ? -1.0 : 1.0) / (fact(m) * fact(n)) * binom(m, p) * binom(n, q) *
                                     std::pow(rho_bar, p + q - m - n);
                    terms.push_back(LrTerm{kCF * c * a, a - 1.0, cb});
                    terms.push_back(LrTerm{kCF * c * b, b - 1.0, ca});
                    eterms.push_back(LrTerm{kCF * c, a, cb});
                }
        }
}

// Right-hand sides of one round of solved systems: F_k = c_k g_k with g the
// power rho^a (or -L_h rho^a for K_00, from the precomputed fa / fb).
struct LrRhsOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 8 + 16 * kLrRound;
    const double *u, *fa, *fb;
    double2 *F[kLrRound];
    double cre[kLrRound], cim[kLrRound], a[kLrRound];
    int lap[kLrRound];          // 0: rho^a; 1: fa (-L_h rho^alpha); 2: fb (-L_h rho^beta)
    int count;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double rho = u[i] * u[i];
        const double lr = rho > 0.0 ? log(rho) : 0.0;
        for (int k = 0; k < count; ++k) {
            const double g = lap[k] == 1 ? fa[i] : (lap[k] == 2 ? fb[i] : (rho > 0.0 ? exp(a[k] * lr) : 0.0));
            F[k][i] = make_double2(cre[k] * g, cim[k] * g);
        }
    }
};

struct LrBaseOp {        // F = g (complex128), the shared right-hand side of one group
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24;
    const double *u, *fa, *fb;
    double2 *F;
    double a;
    int lap;                    // 0: rho^a; 1: fa (-L_h rho^alpha); 2: fb (-L_h rho^beta)
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        double g;
        if (lap == 1) {
            g = fa[i];
        } else if (lap == 2) {
            g = fb[i];
        } else {
            const double rho = u[i] * u[i];
            g = rho > 0.0 ? exp(a * log(rho)) : 0.0;
        }
        F[i] = make_double2(g, 0.0);
    }
};

struct LrScaleOp {       // V *= c (the factor (2 kF)^2 P_r of the system's right-hand side)
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 32;
    double2 *V;
    double2 c;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { V[i] = cmul(c, V[i]); }
};

// W_c = 2 Re(V_{2c} + V_{2c+1}) for the convolutions of one round
struct LrSumOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 16 * kLrRound + 8 * kLrRound / 2;
    const double2 *V[kLrRound];
    double *W[kLrRound / 2];
    int count;                  // convolutions in the round
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        for (int c = 0; c < count; ++c) W[c][i] = 2.0 * (V[2 * c][i].x + V[2 * c + 1][i].x);
    }
};

// V_LR = sum_t coef_t max(rho, floor)^e_t W_{conv_t}
struct LrVlrOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 16 + 8 * kLrMaxConv;
    const double *u;
    const double *W[kLrMaxConv];
    double *vlr;
    double coef[kLrMaxTerms], e[kLrMaxTerms];
    int conv[kLrMaxTerms];
    int nterms;
    double floor_rho;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        const double lr = log(fmax(u[i] * u[i], floor_rho));
        double v = 0.0;
        for (int t = 0; t < nterms; ++t) v = ::fma(coef[t] * exp(e[t] * lr), W[conv[t]][i], v);
        vlr[i] = v;
    }
};

// With autotune, the batch's schedule is timed on its first batched solve
// (8 iterations from the current warm starts, on copies).
int tune_batch_once(ofdft_scf *s, const double *kap, const void *const *rhs, void *const *xs, hipStream_t st) {
    if (!s->p.autotune || s->batch_tuned) return OFDFT_OK;
    s->batch_tuned = true;
    return ofdft_batch_tune(s->batch, kap, rhs, (const void *const *)xs, 8, nullptr, st);
}

// The order-2 kernel potential: rounds of kLrRound solved systems.
int lr2_potential(ofdft_scf *s, hipStream_t st, int &helm_it, double &helm_res) {
    const int64_t n = s->n;
    OFDFT_TRY((launch_reduce<1>(n, PowersOp{s->u, s->rho_a, s->rho_b, kAlpha, kBeta}, NoFin{}, s->rb, st)));
    OFDFT_TRY(fd_laplacian_apply(&s->g, s->p.radius, OFDFT_F64, s->rho_a, s->f_a, -1.0, 0.0, st));
    OFDFT_TRY(fd_laplacian_apply(&s->g, s->p.radius, OFDFT_F64, s->rho_b, s->f_b, -1.0, 0.0, st));
    const double volume = (double)n * s->dv;
    const double kf = std::cbrt(3.0 * kPi * kPi * s->p.n_electrons / volume);
    const double k2 = 4.0 * kf * kf;
    const int nsys = 2 * (int)s->lr_conv.size();
    const bool ms = s->ms && !s->kernel_warm;
    int worst = OFDFT_OK;       // worst non-negative status of the solves
    if (ms) {
        // no warm start: one multi-shift solve of (-L_h + kappa_r) U = g per group
        // of systems sharing g (from zero), then V = c_r U with the system's factor
        // c_r = P_r (K_00, g = -L_h rho^a) or (2 kF)^2 P_r (g = rho^a)
        for (const std::vector<int> &grp : s->lr_groups) {
            const int cnt = (int)grp.size();
            const LrConv &c0 = s->lr_conv[grp[0] / 2];
            const bool k00 = c0.m == 0 && c0.n == 0;
            const int lap = !k00 ? 0 : (std::fabs(c0.a - kAlpha) < 1e-12 ? 1 : 2);
            OFDFT_TRY((launch_reduce<1>(n, LrBaseOp{s->u, s->f_a, s->f_b, s->lr_F[0], c0.a, lap}, NoFin{}, s->rb,
                                        st)));
            void *xs[kMsGroupMax];
            double kap[2 * kMsGroupMax];
            for (int k = 0; k < cnt; ++k) {
                const LrConv &c = s->lr_conv[grp[k] / 2];
                const int r = grp[k] % 2;
                xs[k] = s->lr_V[grp[k]];
                kap[2 * k] = k2 * c.Q[r].x;
                kap[2 * k + 1] = k2 * c.Q[r].y;
            }
            ofdft_solve_stats hs[kMsGroupMax];
            const int hst = cocg_multishift_solve(s->ms, cnt, kap, -1, s->lr_F[0], xs, s->p.helmholtz_tol,
                                                  s->p.max_iter, hs, nullptr, st);
            if (hst < 0) return hst;
            worst = std::max(worst, hst);
            const double sc = k00 ? 1.0 : k2;
            for (int k = 0; k < cnt; ++k) {
                helm_it += hs[k].iters;
                helm_res = std::max(helm_res, hs[k].rel_res);
                const LrConv &c = s->lr_conv[grp[k] / 2];
                const int r = grp[k] % 2;
                LrScaleOp so{s->lr_V[grp[k]], make_double2(sc * c.P[r].x, sc * c.P[r].y)};
                OFDFT_TRY((launch_reduce<1>(n, so, NoFin{}, s->rb, st)));
            }
        }
    }
    for (int j0 = 0; j0 < nsys; j0 += kLrRound) {
        if (ms) {               // solved above: only the round's sums
            LrSumOp so{};
            so.count = kLrRound / 2;
            for (int k = 0; k < kLrRound; ++k) so.V[k] = s->lr_V[j0 + k];
            for (int c = 0; c < kLrRound / 2; ++c) so.W[c] = s->lr_W[j0 / 2 + c];
            OFDFT_TRY((launch_reduce<1>(n, so, NoFin{}, s->rb, st)));
            continue;
        }
        const int cnt = std::min(kLrRound, nsys - j0);
        LrRhsOp ro{};
        ro.u = s->u;
        ro.fa = s->f_a;
        ro.fb = s->f_b;
        ro.count = cnt;
        const void *rhs[kLrRound];
        void *xs[kLrRound];
        double kap[2 * kLrRound];
        for (int k = 0; k < cnt; ++k) {
            const int j = j0 + k;
            const LrConv &c = s->lr_conv[j / 2];
            const int r = j % 2;
            const bool k00 = c.m == 0 && c.n == 0;
            const double sc = k00 ? 1.0 : k2;
            ro.F[k] = s->lr_F[k];
            ro.cre[k] = sc * c.P[r].x;
            ro.cim[k] = sc * c.P[r].y;
            ro.a[k] = c.a;
            ro.lap[k] = !k00 ? 0 : (std::fabs(c.a - kAlpha) < 1e-12 ? 1 : 2);
            rhs[k] = s->lr_F[k];
            xs[k] = s->lr_V[j];
            kap[2 * k] = k2 * c.Q[r].x;
            kap[2 * k + 1] = k2 * c.Q[r].y;
        }
        if (cnt < kLrRound) {        // lr_setup gives 32 systems for L = 2
            set_error("kernel terms: the number of solved systems must be a multiple of %d", kLrRound);
            return OFDFT_INVALID_ARG;
        }
        OFDFT_TRY((launch_reduce<1>(n, ro, NoFin{}, s->rb, st)));
        ofdft_solve_stats hs[kLrRound];
        OFDFT_TRY(tune_batch_once(s, kap, rhs, xs, st));
        int hst = cg_helmholtz_solve_batched(s->batch, kap, rhs, xs, s->p.helmholtz_tol, s->p.max_iter, hs, st);
        if (hst < 0) return hst;
        worst = std::max(worst, hst);
        for (int k = 0; k < cnt; ++k) {
            helm_it += hs[k].iters;
            helm_res = std::max(helm_res, hs[k].rel_res);
        }
        LrSumOp so{};
        so.count = cnt / 2;
        for (int k = 0; k < cnt; ++k) so.V[k] = s->lr_V[j0 + k];
        for (int c = 0; c < cnt / 2; ++c) so.W[c] = s->lr_W[j0 / 2 + c];
        OFDFT_TRY((launch_reduce<1>(n, so, NoFin{}, s->rb, st)));
    }
    LrVlrOp vo{};
    vo.u = s->u;
    vo.vlr = s->vlr;
    for (size_t c = 0; c < s->lr_W.size(); ++c) vo.W[c] = s->lr_W[c];
    vo.nterms = (int)s->lr_terms.size();
    for (int t = 0; t < vo.nterms; ++t) {
        vo.coef[t] = s->lr_terms[t].coef;
        vo.e[t] = s->lr_terms[t].e;
        vo.conv[t] = s->lr_terms[t].conv;
    }
    vo.floor_rho = 1e-12 * s->p.n_electrons / volume;
    OFDFT_TRY((launch_reduce<1>(n, vo, NoFin{}, s->rb, st)));
    s->kernel_warm = true;
    return worst;
}

struct MixResidOp {     // vhat = phi + mu vlr (kernel_only: mu vlr); f = vhat - v; totals {|f|^2, |v|^2}
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 32;
    const double *phi, *vlr, *v;
    double *f;
    double mu;
    int kernel_only;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const double vh = kernel_only ? mu * vlr[i] : (mu != 0.0 ? ::fma(mu, vlr[i], phi[i]) : phi[i]);
        const double vi = v[i];
        const double fi = vh - vi;
        f[i] = fi;
        acc[0] = ::fma(fi, fi, acc[0]);
        acc[1] = ::fma(vi, vi, acc[1]);
    }
};

struct CopyOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 16;
    const double *a;
    double *b;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { b[i] = a[i]; }
};

struct SubOp {          // y = a - b
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24;
    const double *a, *b;
    double *y;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { y[i] = a[i] - b[i]; }
};

struct BRhsOp {         // g = 4 pi b (the source of phi[b]); x = 0
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24;
    const double *b;
    double *g, *x;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const {
        g[i] = 4.0 * kPi * b[i];
        x[i] = 0.0;
    }
};

template <typename P_>
int salloc(ofdft_scf *s, P_ **p, size_t bytes) {
    void *q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
        set_error("ofdft_scf: out of device memory (%zu bytes)", bytes);
        return OFDFT_NO_MEMORY;
    }
    s->allocs.push_back(q);
    *p = (P_ *)q;
    return OFDFT_OK;
}

void scf_free(ofdft_scf *s) {
    density_free(s);
    if (s->pois) ofdft_poisson_destroy(s->pois);
    if (s->batch) ofdft_batch_destroy(s->batch);
    if (s->ms) ofdft_multishift_destroy(s->ms);
    if (s->mix) ofdft_anderson_destroy(s->mix);
    if (s->umg) {
        mg_free(*s->umg);
        delete s->umg;
        s->umg = nullptr;
    }
    for (void *p : s->allocs)
        if (p) (void)hipFree(p);
    s->allocs.clear();
    if (s->hsc) (void)hipHostFree(s->hsc);
    redbuf_free(s->rb);
}

// vhat -> s->fres (phi and the shifted solutions are updated as warm starts).
// Returns the worst status of the solves: an error (< 0) at once, else
// NOT_CONVERGED if any solve missed its tolerance (the map is still formed).
int potential_map(ofdft_scf *s, hipStream_t st, double &pois_res, int &pois_it, int &helm_it,
                  double &helm_res) {
    const int64_t n = s->n;
    OFDFT_TRY((launch_reduce<1>(n, PoissonRhsOp{s->u, s->b, s->g4}, NoFin{}, s->rb, st)));
    ofdft_solve_stats ps{};
    int pst = poisson_solve(s->pois, s->g4, s->phi, s->p.poisson_tol, s->p.max_iter, ps, st);
    if (pst < 0) return pst;
    int worst = pst;
    pois_res = ps.rel_res;
    pois_it = ps.iters;
    helm_it = 0;
    helm_res = 0.0;
    if (s->p.mu && s->p.lr_order == 2) {
        const int lst = lr2_potential(s, st, helm_it, helm_res);
        return lst < 0 ? lst : std::max(worst, lst);
    }
    if (s->p.mu && s->ms && !s->kernel_warm) {
        // No warm start yet: the systems of one power share the right-hand side
        // up to P_r, so one multi-shift solve of (-L_h + kappa_r) U_r = f per
        // power for r = 1, 3 (from zero), then V_r = P_r U_r and the conjugates.
        OFDFT_TRY((launch_reduce<1>(n, PowersOp{s->u, s->rho_a, s->rho_b, kAlpha, kBeta}, NoFin{}, s->rb, st)));
        OFDFT_TRY(fd_laplacian_apply(&s->g, s->p.radius, OFDFT_F64, s->rho_a, s->f_a, -1.0, 0.0, st));
        OFDFT_TRY(fd_laplacian_apply(&s->g, s->p.radius, OFDFT_F64, s->rho_b, s->f_b, -1.0, 0.0, st));
        OFDFT_TRY((launch_reduce<1>(n, BaseRhsOp{s->f_a, s->f_b, (double2 *)s->Fr[0], (double2 *)s->Fr[4]},
                                    NoFin{}, s->rb, st)));
        const double kap[4] = {s->kappa[0], s->kappa[1], s->kappa[4], s->kappa[5]};
        for (int q = 0; q < 2; ++q) {          // q = 0: f_beta (V_0, V_2), q = 1: f_alpha (V_4, V_6)
            void *xs[2] = {s->Vr[4 * q], s->Vr[4 * q + 2]};
            ofdft_solve_stats hs[2];
            const int hst = cocg_multishift_solve(s->ms, 2, kap, -1, s->Fr[4 * q], xs, s->p.helmholtz_tol,
                                                  s->p.max_iter, hs, nullptr, st);
            if (hst < 0) return hst;
            worst = std::max(worst, hst);
            for (int k = 0; k < 2; ++k) {
                helm_it += hs[k].iters;
                helm_res = std::max(helm_res, hs[k].rel_res);
            }
        }
        ScaleConjOp sc{(double2 *)s->Vr[0], (double2 *)s->Vr[2], (double2 *)s->Vr[4], (double2 *)s->Vr[6],
                       (double2 *)s->Vr[1], (double2 *)s->Vr[3], (double2 *)s->Vr[5], (double2 *)s->Vr[7],
                       make_double2(kP00[0][0], kP00[0][1]), make_double2(kP00[2][0], kP00[2][1])};
        OFDFT_TRY((launch_reduce<1>(n, sc, NoFin{}, s->rb, st)));
        const double rho_bar = s->p.n_electrons / ((double)n * s->dv);
        VlrOp vo{s->u, s->Vr[0], s->Vr[2], s->Vr[4], s->Vr[6], s->vlr, 1e-12 * rho_bar, kAlpha, kBeta};
        OFDFT_TRY((launch_reduce<1>(n, vo, NoFin{}, s->rb, st)));
        s->kernel_warm = true;
    } else if (s->p.mu) {
        OFDFT_TRY((launch_reduce<1>(n, PowersOp{s->u, s->rho_a, s->rho_b, kAlpha, kBeta}, NoFin{}, s->rb, st)));
        OFDFT_TRY(fd_laplacian_apply(&s->g, s->p.radius, OFDFT_F64, s->rho_a, s->f_a, -1.0, 0.0, st));
        OFDFT_TRY(fd_laplacian_apply(&s->g, s->p.radius, OFDFT_F64, s->rho_b, s->f_b, -1.0, 0.0, st));
        ShiftRhsOp sr{s->f_a, s->f_b, s->Fr[0], s->Fr[2], s->Fr[4], s->Fr[6], {}, {}};
        for (int r = 0; r < 4; ++r) {
            sr.pr[r] = kP00[r][0];
            sr.pi[r] = kP00[r][1];
        }
        OFDFT_TRY((launch_reduce<1>(n, sr, NoFin{}, s->rb, st)));
        const void *rhs[4];
        void *xs[4];
        double kap[8];
        for (int q = 0; q < 4; ++q) {
            rhs[q] = s->Fr[2 * q];
            xs[q] = s->Vr[2 * q];
            kap[2 * q] = s->kappa[4 * q];
            kap[2 * q + 1] = s->kappa[4 * q + 1];
        }
        ofdft_solve_stats hs[4];
        OFDFT_TRY(tune_batch_once(s, kap, rhs, xs, st));
        int hst = cg_helmholtz_solve_batched(s->batch, kap, rhs, xs, s->p.helmholtz_tol,
                                             s->p.max_iter, hs, st);
        if (hst < 0) return hst;
        worst = std::max(worst, hst);
        for (int q = 0; q < 4; ++q) {
            helm_it += hs[q].iters;
            helm_res = std::max(helm_res, hs[q].rel_res);
        }
        ConjOp co{(const double2 *)s->Vr[0], (const double2 *)s->Vr[2], (const double2 *)s->Vr[4],
                  (const double2 *)s->Vr[6], (double2 *)s->Vr[1], (double2 *)s->Vr[3],
                  (double2 *)s->Vr[5], (double2 *)s->Vr[7]};
        OFDFT_TRY((launch_reduce<1>(n, co, NoFin{}, s->rb, st)));
        const double rho_bar = s->p.n_electrons / ((double)n * s->dv);
        VlrOp vo{s->u, s->Vr[0], s->Vr[2], s->Vr[4], s->Vr[6], s->vlr, 1e-12 * rho_bar, kAlpha, kBeta};
        OFDFT_TRY((launch_reduce<1>(n, vo, NoFin{}, s->rb, st)));
        s->kernel_warm = true;
    }
    return worst;
}

}  // namespace

}  // namespace ofdft

using namespace ofdft;

extern "C" int ofdft_scf_create(const ofdft_scf_params *p, const double *b, const double *u0,
                                ofdft_scf **out, void *stream) {
    if (!p || !b || !u0 || !out) {
        set_error("ofdft_scf_create: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    OFDFT_TRY(check_grid(&p->grid, p->radius));
    if (!(p->n_electrons > 0) || p->lambda < 0 || (p->mu != 0 && p->mu != 1) || p->history < 0 ||
        !(p->u_tol > 0) || !(p->poisson_tol > 0) || (p->mu && !(p->helmholtz_tol > 0)) ||
        (p->lr_order != 0 && p->lr_order != 2) || !(p->line_slope_tol >= 0.0 && p->line_slope_tol < 1.0) ||
        (p->helmholtz_multishift != 0 && p->helmholtz_multishift != 1) ||
        (p->autotune != 0 && p->autotune != 1) || (p->fixed_point != 0 && p->fixed_point != 1)) {
        set_error("ofdft_scf_create: invalid parameters");
        return OFDFT_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    ofdft_scf *s = new (std::nothrow) ofdft_scf();
    if (!s) return OFDFT_NO_MEMORY;
    s->p = *p;
    if (s->p.max_iter <= 0) s->p.max_iter = 100000;
    s->g = p->grid;
    s->n = npoints(p->grid);
    s->dv = p->grid.hx * p->grid.hy * p->grid.hz;
    s->coef = make_coef(p->grid, p->radius);
    auto fail = [&](int code) {
        scf_free(s);
        delete s;
        return code;
    };
    const size_t b8 = sizeof(double) * s->n;
    int rc = OFDFT_OK;
    double **vecs[] = {&s->b, &s->u, &s->v, &s->phi, &s->vlr, &s->fres, &s->g4, &s->Hu,
                       &s->rA, &s->rB, &s->dA, &s->dB};
    for (double **q : vecs)
        if ((rc = salloc(s, q, b8))) return fail(rc);
    if (p->fixed_point == 1) {
        double **hv[] = {&s->hPb, &s->hP, &s->hQ0, &s->hQ1, &s->hQ2, &s->hV};
        for (double **q : hv)
            if ((rc = salloc(s, q, b8))) return fail(rc);
    }
    const bool u_mg = p->u_precond == OFDFT_PRECOND_MULTIGRID || p->u_precond == OFDFT_PRECOND_MULTIGRID_F64;
    if (u_mg && p->lambda > 0) {
        // preconditioner of the density update: -Delta + 2 sigma / lambda,
        // sigma = V_TF(mean density)
        if ((rc = salloc(s, &s->z, b8))) return fail(rc);
        s->umg = new (std::nothrow) Multigrid();
        if (!s->umg) return fail(OFDFT_NO_MEMORY);
        if ((rc = mg_create(*s->umg, p->grid, 8, p->u_precond == OFDFT_PRECOND_MULTIGRID))) return fail(rc);
        const double rho_bar = p->n_electrons / ((double)s->n * s->dv);
        const double sigma = p->u_precond_sigma > 0.0 ? p->u_precond_sigma
                                                       : (5.0 / 3.0) * kCF * std::cbrt(rho_bar * rho_bar);
        s->u_kappa = 2.0 * sigma / p->lambda;
    } else if (p->u_precond != OFDFT_PRECOND_NONE && !u_mg) {
        set_error("ofdft_scf_create: unknown u_precond %d", p->u_precond);
        return fail(OFDFT_INVALID_ARG);
    }
    if ((rc = salloc(s, &s->dsc, sizeof(double) * 64))) return fail(rc);
    if (hipHostMalloc(&s->hsc, sizeof(double) * 64, hipHostMallocDefault) != hipSuccess) return fail(OFDFT_NO_MEMORY);
    if ((rc = redbuf_alloc(s->rb))) return fail(rc);
    if (p->mu && p->lr_order == 2) {
        if ((rc = salloc(s, &s->rho_a, b8)) || (rc = salloc(s, &s->rho_b, b8)) ||
            (rc = salloc(s, &s->f_a, b8)) || (rc = salloc(s, &s->f_b, b8)))
            return fail(rc);
        const double rho_bar = p->n_electrons / ((double)s->n * s->dv);
        lr_setup(2, rho_bar, s->lr_conv, s->lr_terms, s->lr_eterms);
        if ((int)s->lr_conv.size() > kLrMaxConv || (int)s->lr_terms.size() > kLrMaxTerms ||
            (2 * s->lr_conv.size()) % kLrRound) {
            set_error("ofdft_scf_create: kernel-term tables exceed their limits");
            return fail(OFDFT_INVALID_ARG);
        }
        s->lr_V.assign(2 * s->lr_conv.size(), nullptr);
        s->lr_W.assign(s->lr_conv.size(), nullptr);
        for (double2 *&q : s->lr_V) {
            if ((rc = salloc(s, &q, 2 * b8))) return fail(rc);
            if (hipMemsetAsync(q, 0, 2 * b8, st) != hipSuccess) return fail(OFDFT_HIP_ERROR);
        }
        for (double *&q : s->lr_W)
            if ((rc = salloc(s, &q, b8))) return fail(rc);
        for (double2 *&q : s->lr_F)
            if ((rc = salloc(s, &q, 2 * b8))) return fail(rc);
        ofdft_grid grids[kLrRound];
        for (int q = 0; q < kLrRound; ++q) grids[q] = p->grid;
        if (p->helmholtz_multishift) {
            // group the systems by their shared right-hand side: rho^a (the same
            // power in several kernels) or -L_h rho^a (K_00), up to kMsGroupMax
            std::vector<std::pair<double, bool>> keys;
            int gmax = 0;
            for (int j = 0; j < 2 * (int)s->lr_conv.size(); ++j) {
                const LrConv &c = s->lr_conv[j / 2];
                const bool k00 = c.m == 0 && c.n == 0;
                size_t g = 0;
                while (g < keys.size() && !(std::fabs(keys[g].first - c.a) < 1e-12 && keys[g].second == k00 &&
                                            (int)s->lr_groups[g].size() < kMsGroupMax))
                    ++g;
                if (g == keys.size()) {
                    keys.emplace_back(c.a, k00);
                    s->lr_groups.emplace_back();
                }
                s->lr_groups[g].push_back(j);
                gmax = std::max(gmax, (int)s->lr_groups[g].size());
            }
            if ((rc = ofdft_multishift_create(&p->grid, p->radius, gmax, &s->ms))) return fail(rc);
        }
        if ((rc = ofdft_batch_create(kLrRound, grids, p->radius,
                                     p->helmholtz_dtype == OFDFT_C64 ? OFDFT_C64 : OFDFT_C128, &s->batch)))
            return fail(rc);
        if (p->helmholtz_precond != OFDFT_PRECOND_NONE &&
            (rc = ofdft_batch_set_preconditioner(s->batch, p->helmholtz_precond)))
            return fail(rc);
    } else if (p->mu) {
        if ((rc = salloc(s, &s->rho_a, b8)) || (rc = salloc(s, &s->rho_b, b8)) ||
            (rc = salloc(s, &s->f_a, b8)) || (rc = salloc(s, &s->f_b, b8)))
            return fail(rc);
        for (int j = 0; j < 8; ++j)
            if ((j % 2 == 0 && (rc = salloc(s, &s->Fr[j], 2 * b8))) || (rc = salloc(s, &s->Vr[j], 2 * b8)))
                return fail(rc);
        const double volume = (double)s->n * s->dv;
        const double kf = std::cbrt(3.0 * kPi * kPi * p->n_electrons / volume);
        const double k2 = 4.0 * kf * kf;
        for (int j = 0; j < 8; ++j) {
            s->kappa[2 * j] = k2 * kQ00[j % 4][0];
            s->kappa[2 * j + 1] = k2 * kQ00[j % 4][1];
        }
        ofdft_grid grids[4];
        for (int q = 0; q < 4; ++q) grids[q] = p->grid;
        if (p->helmholtz_multishift && (rc = ofdft_multishift_create(&p->grid, p->radius, 2, &s->ms)))
            return fail(rc);
        if ((rc = ofdft_batch_create(4, grids, p->radius,
                                     p->helmholtz_dtype == OFDFT_C64 ? OFDFT_C64 : OFDFT_C128, &s->batch)))
            return fail(rc);
        if (p->helmholtz_precond != OFDFT_PRECOND_NONE &&
            (rc = ofdft_batch_set_preconditioner(s->batch, p->helmholtz_precond)))
            return fail(rc);
        for (int j = 0; j < 8; ++j)
            if (hipMemsetAsync(s->Vr[j], 0, 2 * b8, st) != hipSuccess) return fail(OFDFT_HIP_ERROR);
    }
    const int pmode = (p->poisson_mode == OFDFT_REFINED_F32 || p->poisson_mode == OFDFT_MULTIGRID ||
                       p->poisson_mode == OFDFT_MULTIGRID_F64)
                          ? p->poisson_mode
                          : OFDFT_PLAIN_F64;
    if ((rc = ofdft_poisson_create(&p->grid, p->radius, pmode, &s->pois))) return fail(rc);
    if ((rc = ofdft_anderson_create(s->n, p->history, p->zeta, &s->mix))) return fail(rc);
    if (hipMemcpyAsync(s->b, b, b8, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(s->u, u0, b8, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemsetAsync(s->phi, 0, b8, st) != hipSuccess || hipMemsetAsync(s->vlr, 0, b8, st) != hipSuccess ||
        hipMemsetAsync(s->v, 0, b8, st) != hipSuccess)
        return fail(OFDFT_HIP_ERROR);
    if (p->autotune) {
        // the fused stencil passes (density update, CG, residuals) and the
        // apply (kernel right-hand sides) on this grid
        if ((rc = ofdft_tune_stencil(&p->grid, p->radius, OFDFT_F64, OFDFT_TUNE_PASS, 5, nullptr, st)) ||
            (rc = ofdft_tune_stencil(&p->grid, p->radius, OFDFT_F64, OFDFT_TUNE_APPLY, 5, nullptr, st)))
            return fail(rc);
    }
    // v_0 = phi[u_0] + mu V_LR[u_0] (fixed_point 1: V_LR[u_0], and phi[b] for U)
    double pr, hr;
    int pit, hit;
    int bst = OFDFT_OK;
    if (p->fixed_point == 1) {
        if ((rc = launch_reduce<1>(s->n, BRhsOp{s->b, s->g4, s->hPb}, NoFin{}, s->rb, st)) < 0) return fail(rc);
        ofdft_solve_stats ps{};
        bst = poisson_solve(s->pois, s->g4, s->hPb, p->poisson_tol, s->p.max_iter, ps, st);
        if (bst < 0) return fail(bst);
    }
    int mst = potential_map(s, st, pr, pit, hit, hr);
    if (mst < 0) return fail(mst);
    mst = std::max(mst, bst);
    if (p->fixed_point == 1 &&
        (rc = launch_reduce<1>(s->n, SubOp{s->phi, s->hPb, s->hQ0}, NoFin{}, s->rb, st)) < 0)
        return fail(rc);
    // the multi-shift context serves only this first kernel potential (the
    // steps warm-start the batched solver): release its vectors
    if (s->ms) {
        ofdft_multishift_destroy(s->ms);
        s->ms = nullptr;
    }
    if ((rc = launch_reduce<2>(s->n, MixResidOp{s->phi, s->vlr, s->v, s->fres, (double)p->mu, p->fixed_point},
                               NoFin{}, s->rb, st)) < 0)
        return fail(rc);
    // v = 0 + f  (MixResidOp wrote f = vhat - 0)
    if ((rc = launch_reduce<1>(s->n, CopyOp{s->fres, s->v}, NoFin{}, s->rb, st)) < 0) return fail(rc);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(OFDFT_HIP_ERROR);
    *out = s;
    return mst;         // NOT_CONVERGED if a solve of v_0 missed its tolerance
}

extern "C" int ofdft_scf_destroy(ofdft_scf *s) {
    if (!s) return OFDFT_OK;
    scf_free(s);
    delete s;
    return OFDFT_OK;
}

extern "C" int ofdft_scf_step(ofdft_scf *s, double *fp_residual, void *stream) {
    if (!s) {
        set_error("ofdft_scf_step: NULL context");
        return OFDFT_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    int uit = 0;
    double ures = 0, eta = 0;
    const int ust = density_update(s, s->v, s->u, uit, ures, eta, st);
    if (ust < 0) return ust;
    double pr = 0, hr = 0;
    int pit = 0, hit = 0;
    const int mst = potential_map(s, st, pr, pit, hit, hr);
    if (mst < 0) return mst;
    if (s->p.fixed_point == 1) {
        // the field of u^2 for the next U (its warm start) and the Poisson
        // iterations inside this one
        OFDFT_TRY((launch_reduce<1>(s->n, SubOp{s->phi, s->hPb, s->hQ0}, NoFin{}, s->rb, st)));
        pit += (int)s->u_pois_it;
    }
    OFDFT_TRY((launch_reduce<2>(s->n, MixResidOp{s->phi, s->vlr, s->v, s->fres, (double)s->p.mu, s->p.fixed_point},
                                StoreTotals<2>{s->dsc + 40}, s->rb, st)));
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->hsc + 40, s->dsc + 40, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    OFDFT_TRY(anderson_mix(s->mix, s->v, s->fres, s->v, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    const double f2 = s->hsc[40], v2 = s->hsc[41];
    const double res = v2 > 0 ? std::sqrt(f2 / v2) : std::sqrt(f2);
    if (fp_residual) *fp_residual = res;
    s->last[0] = uit;
    s->last[1] = pit;
    s->last[2] = hit;
    s->last[3] = ures;
    s->last[4] = pr;
    s->last[5] = hr;
    s->last[6] = eta;
    if (!std::isfinite(res)) return OFDFT_NONFINITE;
    return std::max(ust, mst);      // NOT_CONVERGED if U(v) or a solve missed its tolerance
}

// State vectors: 0 v, 1 u, 2 phi, 3 V_LR (n doubles); 4.. the shifted-solve
// solutions (complex128, 2n doubles; mu = 1 only): 4..11 the K_00 systems,
// or 4..35 the solved systems of the order-2 terms.
static double *state_ptr(ofdft_scf *s, int which, size_t &count) {
    count = (size_t)s->n;
    switch (which) {
        case 0: return s->v;
        case 1: return s->u;
        case 2: return s->phi;
        case 3: return s->vlr;
        default:
            if (which >= 4 && which - 4 < (int)s->lr_V.size()) {
                count = 2 * (size_t)s->n;
                return (double *)s->lr_V[which - 4];
            }
            if (which >= 4 && which < 12 && s->Vr[which - 4]) {
                count = 2 * (size_t)s->n;
                return (double *)s->Vr[which - 4];
            }
            return nullptr;
    }
}

// Checkpoint file: a header (magic, version, grid, spacings, radius, kernel
// settings, history length, number of state arrays, the line-search memory,
// whether the kernel solutions are warm), every state array of
// ofdft_scf_get in order, then the Anderson history.
namespace {
constexpr char kCkMagic[8] = {'O', 'F', 'D', 'F', 'T', 'C', 'K', '2'};
struct CkHeader {
    char magic[8];
    int64_t nx, ny, nz, radius, mu, lr_order, history, nstate, kernel_warm, fixed_point;
    double hx, hy, hz, n_electrons, s_prev;
};

int64_t state_count(ofdft_scf *s) {
    int64_t k = 0;
    size_t c = 0;
    while (state_ptr(s, (int)k, c)) ++k;
    return k;
}
}  // namespace

extern "C" int ofdft_scf_save(ofdft_scf *s, const char *path, void *stream) {
    if (!s || !path) {
        set_error("ofdft_scf_save: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    OFDFT_CHECK_HIP(hipStreamSynchronize((hipStream_t)stream));
    std::FILE *f = std::fopen(path, "wb");
    if (!f) {
        set_error("ofdft_scf_save: cannot open %s", path);
        return OFDFT_INVALID_ARG;
    }
    CkHeader h{};
    std::memcpy(h.magic, kCkMagic, 8);
    h.nx = s->g.nx;
    h.ny = s->g.ny;
    h.nz = s->g.nz;
    h.radius = s->p.radius;
    h.mu = s->p.mu;
    h.lr_order = s->p.lr_order;
    h.history = s->p.history;
    h.fixed_point = s->p.fixed_point;
    h.nstate = state_count(s);
    h.kernel_warm = s->kernel_warm ? 1 : 0;
    h.hx = s->g.hx;
    h.hy = s->g.hy;
    h.hz = s->g.hz;
    h.n_electrons = s->p.n_electrons;
    h.s_prev = s->s_prev;
    int rc = ck_write(f, &h, sizeof h);
    for (int64_t k = 0; rc == OFDFT_OK && k < h.nstate; ++k) {
        size_t c = 0;
        const double *p = state_ptr(s, (int)k, c);
        rc = ck_write_dev(f, p, sizeof(double) * c);
    }
    if (rc == OFDFT_OK) rc = anderson_write(s->mix, f);
    if (std::fclose(f) != 0 && rc == OFDFT_OK) {
        set_error("ofdft_scf_save: closing %s failed", path);
        rc = OFDFT_INVALID_ARG;
    }
    return rc;
}

extern "C" int ofdft_scf_load(ofdft_scf *s, const char *path, void *stream) {
    if (!s || !path) {
        set_error("ofdft_scf_load: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    OFDFT_CHECK_HIP(hipStreamSynchronize((hipStream_t)stream));
    std::FILE *f = std::fopen(path, "rb");
    if (!f) {
        set_error("ofdft_scf_load: cannot open %s", path);
        return OFDFT_INVALID_ARG;
    }
    CkHeader h{};
    int rc = ck_read(f, &h, sizeof h);
    if (rc == OFDFT_OK &&
        (std::memcmp(h.magic, kCkMagic, 8) != 0 || h.nx != s->g.nx || h.ny != s->g.ny || h.nz != s->g.nz ||
         h.hx != s->g.hx || h.hy != s->g.hy || h.hz != s->g.hz || h.radius != s->p.radius || h.mu != s->p.mu ||
         h.lr_order != s->p.lr_order || h.history != s->p.history || h.fixed_point != s->p.fixed_point ||
         h.n_electrons != s->p.n_electrons ||
         h.nstate != state_count(s))) {
        set_error("ofdft_scf_load: %s is not a checkpoint of a context with these grid and kernel settings", path);
        rc = OFDFT_INVALID_ARG;
    }
    for (int64_t k = 0; rc == OFDFT_OK && k < h.nstate; ++k) {
        size_t c = 0;
        double *p = state_ptr(s, (int)k, c);
        rc = ck_read_dev(f, p, sizeof(double) * c);
    }
    if (rc == OFDFT_OK) rc = anderson_read(s->mix, f);
    std::fclose(f);
    if (rc == OFDFT_OK) {
        s->kernel_warm = h.kernel_warm != 0;
        s->s_prev = h.s_prev;
    }
    return rc;
}

extern "C" int ofdft_scf_get(ofdft_scf *s, int which, double *dst, void *stream) {
    size_t count = 0;
    double *p = s ? state_ptr(s, which, count) : nullptr;
    if (!p || !dst) {
        set_error("ofdft_scf_get: bad context, index or destination");
        return OFDFT_INVALID_ARG;
    }
    OFDFT_CHECK_HIP(hipMemcpyAsync(dst, p, sizeof(double) * count, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return OFDFT_OK;
}

extern "C" int ofdft_scf_set(ofdft_scf *s, int which, const double *src, void *stream) {
    size_t count = 0;
    double *p = s ? state_ptr(s, which, count) : nullptr;
    if (!p || !src) {
        set_error("ofdft_scf_set: bad context, index or source");
        return OFDFT_INVALID_ARG;
    }
    OFDFT_CHECK_HIP(hipMemcpyAsync(p, src, sizeof(double) * count, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return OFDFT_OK;
}

extern "C" int ofdft_scf_reset_history(ofdft_scf *s) {
    if (!s) {
        set_error("ofdft_scf_reset_history: NULL context");
        return OFDFT_INVALID_ARG;
    }
    s->s_prev = 0.0;
    return ofdft_anderson_reset(s->mix);
}

extern "C" int ofdft_scf_kernel_shifts(ofdft_scf *s, double *kappa8, double *factor8) {
    if (!s || !kappa8) {
        set_error("ofdft_scf_kernel_shifts: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    const double volume = (double)s->n * s->dv;
    const double kf = std::cbrt(3.0 * kPi * kPi * s->p.n_electrons / volume);
    const double k2 = 4.0 * kf * kf;
    for (int r = 0; r < 4; ++r) {
        kappa8[2 * r] = k2 * kQ00[r][0];
        kappa8[2 * r + 1] = k2 * kQ00[r][1];
        if (factor8) {
            factor8[2 * r] = kP00[r][0];
            factor8[2 * r + 1] = kP00[r][1];
        }
    }
    return OFDFT_OK;
}

extern "C" int ofdft_scf_stats(ofdft_scf *s, double *out7) {
    if (!s || !out7) return OFDFT_INVALID_ARG;
    for (int k = 0; k < 7; ++k) out7[k] = s->last[k];
    return OFDFT_OK;
}

extern "C" int ofdft_density_update(ofdft_scf *s, const double *v, double *u, int *iters,
                                    double *residual, double *eta, void *stream) {
    if (!s || !v || !u) {
        set_error("ofdft_density_update: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    int it = 0;
    double res = 0, e = 0;
    const int ust = density_update(s, v, u, it, res, e, (hipStream_t)stream);
    if (ust < 0) return ust;
    if (iters) *iters = it;
    if (residual) *residual = res;
    if (eta) *eta = e;
    return ust;
}
