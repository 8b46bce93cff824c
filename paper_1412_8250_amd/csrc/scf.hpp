// Fixed-point (SCF-type) context: state vectors, solver contexts and the
// density-update workspace.
#pragma once

#include "poisson.hpp"

struct ofdft_batch;
struct ofdft_multishift;
struct ofdft_anderson;

namespace ofdft {

// One distinct convolution K_mn rho^a of the order-2 kernel terms (solved as
// the shifted systems r = 1, 3; r = 2, 4 are their conjugates).
struct LrConv {
    int m, n;                // kernel, m >= n
    double a;                // power of rho
    double2 P[2], Q[2];      // r = 1, 3
};

// One term of V_LR: coef rho^e (K rho^a of convolution conv).
struct LrTerm {
    double coef, e;
    int conv;
};

constexpr int kLrMaxConv = 16;
constexpr int kLrMaxTerms = 32;
constexpr int kLrRound = 8;        // shifted systems per batched solve
constexpr int kMsGroupMax = 16;    // shifts per multi-shift solve (the solver's maximum)

}  // namespace ofdft

struct ofdft_scf {
    ofdft_scf_params p{};
    ofdft_grid g{};
    int64_t n = 0;
    double dv = 0;                       // h_x h_y h_z (quadrature weight, Section 4)
    ofdft::Coef<double> coef{};
    // state
    double *b = nullptr, *u = nullptr, *v = nullptr, *phi = nullptr, *vlr = nullptr;
    double *fres = nullptr, *g4 = nullptr;
    // kernel-term work (mu = 1)
    double *rho_a = nullptr, *rho_b = nullptr, *f_a = nullptr, *f_b = nullptr;
    double2 *Fr[8] = {}, *Vr[8] = {};
    double kappa[16] = {};
    // order-2 kernel terms (lr_order 2): distinct convolutions, V_LR terms,
    // the solved systems' solutions (2 per convolution, kept as warm starts),
    // each convolution's real sum W = 2 Re(V_1 + V_3), a round's right-hand sides
    std::vector<ofdft::LrConv> lr_conv;
    // multi-shift form (helmholtz_multishift): the kernel potential without a
    // warm start (the context's first) solves the systems grouped by their
    // shared right-hand side, one multi-shift solve per group; later ones use
    // the batched solver warm-started from the previous solutions
    std::vector<std::vector<int>> lr_groups;
    bool kernel_warm = false;
    bool batch_tuned = false;     // autotune: the batch's schedule has been timed
    std::vector<ofdft::LrTerm> lr_terms, lr_eterms;
    std::vector<double2 *> lr_V;
    std::vector<double *> lr_W;
    double2 *lr_F[ofdft::kLrRound] = {};
    // density update workspace; with the preconditioner, z = M r and the
    // multigrid hierarchy of -Delta + u_kappa
    double *Hu = nullptr, *rA = nullptr, *rB = nullptr, *dA = nullptr, *dB = nullptr, *z = nullptr;
    ofdft::Multigrid *umg = nullptr;
    double u_kappa = 0;
    double s_prev = 0;
    // electrostatics inside U (fixed_point 1): phi[b]; the external potential
    // plus phi[b] (P); the fields of u^2, u d and d^2 (Q0, Q1, Q2); the total
    // potential at the current u (V = P + Q0); Poisson iterations inside U
    double *hPb = nullptr, *hP = nullptr, *hQ0 = nullptr, *hQ1 = nullptr, *hQ2 = nullptr, *hV = nullptr;
    int64_t u_pois_it = 0;
    // device-driven density update: iteration state (device and pinned host
    // copies), the captured block of iterations and the pointers it was
    // captured with
    void *udev = nullptr, *udev_h = nullptr;
    hipGraphExec_t ugraph = nullptr;
    hipStream_t ucap = nullptr;
    const void *ugraph_key[3] = {};
    // solver contexts
    ofdft_poisson *pois = nullptr;
    ofdft_batch *batch = nullptr;
    ofdft_multishift *ms = nullptr;   // multi-shift solver of the K_00 term (helmholtz_multishift)
    ofdft_anderson *mix = nullptr;
    ofdft::RedBuf rb{};
    double *dsc = nullptr, *hsc = nullptr;   // device / pinned host scalars
    double last[8] = {};                     // statistics of the last step
    std::vector<void *> allocs;
};

namespace ofdft {

// Anderson history in checkpoint files (anderson.hip).
int anderson_write(ofdft_anderson *a, std::FILE *f);
int anderson_read(ofdft_anderson *a, std::FILE *f);

// U(v): Algorithm 1 from the current s->u; v is a device array.
int density_update(ofdft_scf *s, const double *v, double *u, int &iters, double &res, double &eta,
                   hipStream_t st);
// Releases the density update's device-driven state (graph, stream, buffers).
void density_free(ofdft_scf *s);

}  // namespace ofdft
