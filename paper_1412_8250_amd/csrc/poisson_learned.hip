// Learned form of the Poisson solve: a network initial guess and flexible CG
// with the network as preconditioner (the paper calls for real-space
// preconditioners to make iteration counts size-independent, Section 5.5).
// The learned-refined form continues from the corrected guess with FP32 CG
// inside FP64 residual refinement instead.
//
//   M(r) = h^2 rms(r) N(r / rms(r)), projected to zero mean
//   x_0 = x + M(g - A x);  r_0 = g - A x_0;  z_0 = M(r_0);  p_0 = z_0
//   flexible CG (truncation 1, Polak-Ribiere form):
//     alpha = <r,z> / <p,Ap>;  x += alpha p;  r_new = r - alpha Ap
//     z_new = M(r_new);  beta = <z_new, r_new - r> / <z, r>;  p = z_new + beta p
// All vectors FP64.  Plain FP64 CG from the best iterate takes over if the
// residual has not dropped 10x after 20 iterations, or on NaN/Inf.
#include <algorithm>
#include <cmath>

#include "fcg.hpp"
#include "nn.hpp"

namespace ofdft {


int poisson_solve_learned(ofdft_poisson *s, double *x, double rel_tol, int max_iter,
                          ofdft_solve_stats &stats, hipStream_t st) {
    if (!s->net) {
        set_error("cg_poisson_solve: learned mode needs a network (ofdft_poisson_set_network)");
        return OFDFT_INVALID_ARG;
    }
    const ofdft_grid &g = s->g;
    const int64_t n = npoints(g);
    const double h2 = std::cbrt(g.hx * g.hy * g.hz) * std::cbrt(g.hx * g.hy * g.hz);
    double *r = s->r, *p = s->pA, *r_old = s->pB, *Ap = s->Ap, *z = s->z, *xb = s->xbest;
    double *tot = s->totals + 8, *th = s->totals_host + 8;
    auto sync_tot = [&](int count) -> int {
        OFDFT_CHECK_HIP(hipMemcpyAsync(th, tot, sizeof(double) * count, hipMemcpyDeviceToHost, st));
        OFDFT_CHECK_HIP(hipStreamSynchronize(st));
        return OFDFT_OK;
    };
    auto residual = [&](double &r2) -> int {      // r = gp + L x, totals {sum r, sum r^2}
        OFDFT_TRY(residual_pass<double>(g, s->coef, x, s->gp, r, tot, s->rb, st));
        OFDFT_TRY(sync_tot(2));
        r2 = th[1];
        return OFDFT_OK;
    };
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->totals_host, s->totals, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    const double g2 = s->totals_host[3];
    const double tol2 = rel_tol * rel_tol * g2;
    int applies = 0, iters = 0;
    double r2;
    OFDFT_TRY(residual(r2));
    if (!std::isfinite(r2)) return OFDFT_NONFINITE;
    // Network correction of the starting guess: z = N(r), then the step a
    // along z that minimises the energy-norm error, a = z.r / z.Az (a
    // correction can only lower that error; a useless one gets a ~ 0).
    if (r2 > tol2) {
        OFDFT_TRY(nn::net_apply(s->net, g, r, z, h2, true, st));
        ++applies;
        OFDFT_TRY(pass64(g, s->coef, LoadPlain<double>{z}, EpiAp{Ap, tot, s->rb.partials, s->rb.counter, 0.0},
                         st, 16.0, K_CG_STENCIL));
        OFDFT_TRY((launch_reduce<2>(n, FcgDotsOp{z, r, r}, StoreTotals<2>{tot + 1}, s->rb, st)));
        OFDFT_TRY(sync_tot(3));
        const double zAz = th[0], zr = th[2];
        if (std::isfinite(zAz) && std::isfinite(zr) && zAz > 0.0)
            OFDFT_TRY((launch_reduce<1>(n, AxpyOp{x, z, zr / zAz}, NoFin{}, s->rb, st)));
        OFDFT_TRY(residual(r2));
    }
    stats.nn_applies = applies;
    if (s->mode == OFDFT_LEARNED_REFINED) {      // the refined form from the corrected guess
        ofdft_solve_stats rest{};
        const int status = solve_refined(s, x, rel_tol, max_iter, rest, st);
        stats.iters = rest.iters;
        stats.outer_iters = rest.outer_iters;
        stats.fell_back = 0;
        return status;
    }
    if (!s->learned_fcg) {
        ofdft_solve_stats rest{};
        const int status = solve_plain(s, x, rel_tol, max_iter, rest, st);
        stats.iters = rest.iters;
        stats.fell_back = 0;
        return status;
    }
    double best = r2;
    OFDFT_TRY((launch_reduce<1>(n, CopyOp2{xb, x}, NoFin{}, s->rb, st)));
    const double r2_start = r2;
    bool fall_back = !std::isfinite(r2);
    if (!fall_back && r2 > tol2) {
        OFDFT_TRY(nn::net_apply(s->net, g, r, z, h2, true, st));
        ++applies;
        OFDFT_TRY((launch_reduce<2>(n, FcgDotsOp{z, r, r}, StoreTotals<2>{tot}, s->rb, st)));
        OFDFT_TRY(sync_tot(2));
        double rz = th[1];
        OFDFT_TRY((launch_reduce<1>(n, CopyOp2{p, z}, NoFin{}, s->rb, st)));
        while (iters < max_iter) {
            OFDFT_TRY(pass64(g, s->coef, LoadPlain<double>{p},
                             EpiAp{Ap, tot, s->rb.partials, s->rb.counter, 0.0}, st, 16.0, K_CG_STENCIL));
            OFDFT_TRY(sync_tot(1));
            const double pAp = th[0];
            if (!std::isfinite(pAp) || !(pAp > 0) || !std::isfinite(rz)) {
                fall_back = true;
                break;
            }
            const double a = rz / pAp;
            OFDFT_TRY((launch_reduce<1>(n, FcgStepOp{x, r, r_old, p, Ap, a}, StoreTotals<1>{tot}, s->rb, st)));
            OFDFT_TRY(sync_tot(1));
            r2 = th[0];
            ++iters;
            if (!std::isfinite(r2)) {
                fall_back = true;
                break;
            }
            if (r2 < best) {
                best = r2;
                OFDFT_TRY((launch_reduce<1>(n, CopyOp2{xb, x}, NoFin{}, s->rb, st)));
            }
            if (r2 <= tol2) break;
            if (iters >= 20 && best > 0.01 * r2_start) {   // less than 10x in residual norm
                fall_back = true;
                break;
            }
            OFDFT_TRY(nn::net_apply(s->net, g, r, z, h2, true, st));
            ++applies;
            OFDFT_TRY((launch_reduce<2>(n, FcgDotsOp{z, r, r_old}, StoreTotals<2>{tot}, s->rb, st)));
            OFDFT_TRY(sync_tot(2));
            const double b = th[0] / rz;
            rz = th[1];
            OFDFT_TRY((launch_reduce<1>(n, DirOp{p, z, std::isfinite(b) ? b : 0.0}, NoFin{}, s->rb, st)));
        }
    }
    stats.nn_applies = applies;
    stats.fell_back = fall_back ? 1 : 0;
    int status = OFDFT_OK;
    if (fall_back) {
        OFDFT_TRY((launch_reduce<1>(n, CopyOp2{x, xb}, NoFin{}, s->rb, st)));
        ofdft_solve_stats rest{};
        status = solve_plain(s, x, rel_tol, std::max(1, max_iter - iters), rest, st);
        iters += rest.iters;
    } else if (r2 > tol2) {
        status = OFDFT_NOT_CONVERGED;
    }
    stats.iters = iters;
    return status;
}

}  // namespace ofdft

using namespace ofdft;

extern "C" int ofdft_poisson_set_learned_mode(ofdft_poisson *s, int precondition) {
    if (!s || s->mode != OFDFT_LEARNED || precondition < 0 || precondition > 1) {
        set_error("ofdft_poisson_set_learned_mode: learned solver and 0/1 expected");
        return OFDFT_INVALID_ARG;
    }
    s->learned_fcg = precondition;
    return OFDFT_OK;
}

extern "C" int ofdft_poisson_set_network(ofdft_poisson *s, ofdft_nn *net) {
    if (!s || (s->mode != OFDFT_LEARNED && s->mode != OFDFT_LEARNED_REFINED)) {
        set_error("ofdft_poisson_set_network: solver must be created with OFDFT_LEARNED(_REFINED)");
        return OFDFT_INVALID_ARG;
    }
    if (!net) {
        s->net = nullptr;
        return OFDFT_OK;
    }
    OFDFT_TRY(nn::net_reserve(net, s->g));
    if (!s->z) {
        const size_t b8 = sizeof(double) * npoints(s->g);
        OFDFT_CHECK_HIP(hipMalloc(&s->z, b8));
        OFDFT_CHECK_HIP(hipMalloc(&s->xbest, b8));
    }
    s->net = net;
    return OFDFT_OK;
}
