// Poisson solver context shared by the plain, refined and learned forms.
#pragma once

#include "cg.hpp"
#include "multigrid.hpp"

struct ofdft_nn;
namespace ofdft {
struct CgGraph;
}

struct ofdft_poisson {
    ofdft_grid g{};
    int radius = 6;
    int mode = OFDFT_PLAIN_F64;
    ofdft::Coef<double> coef{};
    ofdft::Coef<float> coef32{};
    double *gp = nullptr, *r = nullptr, *pA = nullptr, *pB = nullptr, *Ap = nullptr;
    float *r32 = nullptr, *d32 = nullptr, *qA = nullptr, *qB = nullptr, *Aq = nullptr;
    ofdft::CgState *st = nullptr, *st_host = nullptr;
    double *totals = nullptr, *totals_host = nullptr;
    ofdft::RedBuf rb{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // captured iteration blocks (FP64 and FP32 loops)
    ofdft::CgGraph *graph64 = nullptr, *graph32 = nullptr;
    bool use_graphs = true;
    double inner_min = 1e-5, inner_max = 1e-1;    // FP32 inner tolerance bounds (refined form)
    // learned form
    ofdft_nn *net = nullptr;
    double *z = nullptr, *zprev = nullptr, *xbest = nullptr;
    int learned_fcg = 0;     // 0: network correction + plain CG; 1: + network-preconditioned FCG
    // multigrid form; its iteration state on the device (and a pinned host
    // copy) and the captured block of iterations
    ofdft::Multigrid *mg = nullptr;
    void *pdev = nullptr, *pdev_h = nullptr;
    hipGraphExec_t mggraph = nullptr;
    hipStream_t mgcap = nullptr;
};

namespace ofdft {

// CG preconditioned by the multigrid V-cycle (s->mg), from the iterate x.
int poisson_solve_mg(ofdft_poisson *s, double *x, double rel_tol, int max_iter,
                     ofdft_solve_stats &stats, hipStream_t st);

// Plain FP64 CG from the iterate x (residual recomputed first); stats.iters set.
int solve_plain(ofdft_poisson *s, double *x, double rel_tol, int max_iter,
                ofdft_solve_stats &stats, hipStream_t st);
// FP32 CG inside FP64 residual refinement from the current x (needs the FP32
// workspace of the refined forms).
int solve_refined(ofdft_poisson *s, double *x, double rel_tol, int max_iter,
                ofdft_solve_stats &stats, hipStream_t st);

template <typename T>
int cg_k1(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, const T *r, const T *p_old,
          T *p_new, T *Ap, CgState *st, const RedBuf &rb, hipStream_t s);
template <typename T>
int residual_pass(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, const T *x,
                  const double *gp, T *r, double *totals, const RedBuf &rb, hipStream_t s);
template <typename T>
int cg_iterate(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, T *x, T *r, T *pA, T *pB,
               T *Ap, CgState *st, CgState *st_host, const RedBuf &rb, hipStream_t s, int &iters,
               int &done, CgGraph *graph = nullptr);
int status_from_done(int done);
int poisson_solve(ofdft_poisson *s, const double *rhs, double *x, double rel_tol, int max_iter,
                  ofdft_solve_stats &stats, hipStream_t st);
int poisson_solve_learned(ofdft_poisson *s, double *x, double rel_tol, int max_iter,
                          ofdft_solve_stats &stats, hipStream_t st);

}  // namespace ofdft
