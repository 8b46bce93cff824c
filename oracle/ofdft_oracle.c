/*
 * Plain FP64 CPU oracle of the periodic higher-order finite-difference
 * Laplacian and of the Krylov solves built on it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it shares no code with the GPU library.  It is written for
 * obviousness, not speed: direct loops with modulo index wrapping, no
 * blocking, no fusion.  OpenMP only splits the outermost loop.
 *
 * Layout: arrays are [nz][ny][nx], x fastest; complex arrays interleave
 * (re, im) doubles.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Weights of the 2N-th order central second difference (Section 4, FD
 * Laplacian equation and its weight formulas):
 *   w_0 = -(1/h^2) sum_{q=1}^{N} 1/q^2
 *   w_p = 2 (-1)^{p+1} (N!)^2 / (h^2 p^2 (N-p)! (N+p)!),  p = 1..N      */
void orc_fd_weights(int N, double h, double *w)
{
    double fact[32];
    fact[0] = 1.0;
    for (int i = 1; i < 32; ++i) fact[i] = fact[i - 1] * (double)i;
    double s = 0.0;
    for (int q = 1; q <= N; ++q) s += 1.0 / ((double)q * (double)q);
    w[0] = -s / (h * h);
    for (int p = 1; p <= N; ++p) {
        double sign = (p % 2 == 1) ? 1.0 : -1.0;
        w[p] = 2.0 * sign * fact[N] * fact[N] /
               (h * h * (double)p * (double)p * fact[N - p] * fact[N + p]);
    }
}

/* Periodic image of an index (Section 4: an index outside the grid maps to
 * its periodic image; repeated wrapping for offsets larger than n). */
static long wrap(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

/* y = L_h x.  Each axis a contributes sum_{p=0}^{N} w_p^{(a)} (f_{+p} + f_{-p}),
 * so the centre carries 2 w_0^{(a)} per axis (6 w_0 for equal spacings). */
void orc_laplacian(int nx, int ny, int nz, double hx, double hy, double hz, int N,
                   const double *x, double *y)
{
    double wx[16], wy[16], wz[16];
    orc_fd_weights(N, hx, wx);
    orc_fd_weights(N, hy, wy);
    orc_fd_weights(N, hz, wz);
    const long sx = 1, sy = nx, sz = (long)nx * ny;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                double s = 2.0 * (wx[0] + wy[0] + wz[0]) * x[k * sz + j * sy + i * sx];
                for (int p = 1; p <= N; ++p) {
                    s += wx[p] * (x[k * sz + j * sy + wrap(i + p, nx)] +
                                  x[k * sz + j * sy + wrap(i - p, nx)]);
                    s += wy[p] * (x[k * sz + wrap(j + p, ny) * sy + i] +
                                  x[k * sz + wrap(j - p, ny) * sy + i]);
                    s += wz[p] * (x[wrap(k + p, nz) * sz + j * sy + i] +
                                  x[wrap(k - p, nz) * sz + j * sy + i]);
                }
                y[k * sz + j * sy + i] = s;
            }
}

/* Complex version: L_h is real, so it acts on real and imaginary parts alike. */
void orc_laplacian_z(int nx, int ny, int nz, double hx, double hy, double hz, int N,
                     const double *x, double *y)
{
    long n = (long)nx * ny * nz;
    double *re = malloc(sizeof(double) * n), *im = malloc(sizeof(double) * n);
    double *lre = malloc(sizeof(double) * n), *lim = malloc(sizeof(double) * n);
    for (long i = 0; i < n; ++i) { re[i] = x[2 * i]; im[i] = x[2 * i + 1]; }
    orc_laplacian(nx, ny, nz, hx, hy, hz, N, re, lre);
    orc_laplacian(nx, ny, nz, hx, hy, hz, N, im, lim);
    for (long i = 0; i < n; ++i) { y[2 * i] = lre[i]; y[2 * i + 1] = lim[i]; }
    free(re); free(im); free(lre); free(lim);
}

static double dot(long n, const double *a, const double *b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Textbook conjugate gradients for  -L_h x = g  (g must have zero mean; the
 * operator -L_h is symmetric positive semi-definite with the constants as its
 * null space, Section 3.3).  Stops when ||g + L_h x|| <= tol ||g|| on the
 * recursively updated residual; afterwards x is shifted to zero mean
 * (Section 4: the free constant is fixed by a zero integral).
 * Returns the iteration count; *relres gets the true final residual. */
int orc_cg_poisson(int nx, int ny, int nz, double hx, double hy, double hz, int N,
                   const double *g, double *x, double tol, int maxit, double *relres)
{
    long n = (long)nx * ny * nz;
    double *r = malloc(sizeof(double) * n), *p = malloc(sizeof(double) * n);
    double *Ap = malloc(sizeof(double) * n);
    orc_laplacian(nx, ny, nz, hx, hy, hz, N, x, Ap);
    for (long i = 0; i < n; ++i) r[i] = g[i] + Ap[i];      /* r = g - (-L x) */
    memcpy(p, r, sizeof(double) * n);
    double gnorm = sqrt(dot(n, g, g));
    double rr = dot(n, r, r);
    int it = 0;
    while (it < maxit && sqrt(rr) > tol * gnorm) {
        orc_laplacian(nx, ny, nz, hx, hy, hz, N, p, Ap);
        for (long i = 0; i < n; ++i) Ap[i] = -Ap[i];        /* Ap = (-L) p */
        double alpha = rr / dot(n, p, Ap);
        for (long i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
        double rr_new = dot(n, r, r);
        double beta = rr_new / rr;
        rr = rr_new;
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        ++it;
    }
    double mean = 0.0;
    for (long i = 0; i < n; ++i) mean += x[i];
    mean /= (double)n;
    for (long i = 0; i < n; ++i) x[i] -= mean;
    orc_laplacian(nx, ny, nz, hx, hy, hz, N, x, Ap);
    for (long i = 0; i < n; ++i) r[i] = g[i] + Ap[i];
    *relres = sqrt(dot(n, r, r)) / gnorm;
    free(r); free(p); free(Ap);
    return it;
}

/* Unconjugated bilinear form sum a_i b_i of two interleaved complex vectors. */
static void zdotu(long n, const double *a, const double *b, double *re, double *im)
{
    double sr = 0.0, si = 0.0;
#pragma omp parallel for reduction(+ : sr, si) schedule(static)
    for (long i = 0; i < n; ++i) {
        sr += a[2 * i] * b[2 * i] - a[2 * i + 1] * b[2 * i + 1];
        si += a[2 * i] * b[2 * i + 1] + a[2 * i + 1] * b[2 * i];
    }
    *re = sr; *im = si;
}

static double znorm(long n, const double *a)
{
    return sqrt(dot(2 * n, a, a));
}

/* Textbook COCG (conjugate gradients with the unconjugated bilinear form) for
 * the complex-symmetric shifted system (-L_h + kappa) u = f (Section 3.1,
 * Helmholtz equations, multiplied through by (2 k_F)^2).  Stops when
 * ||f - A u|| <= tol ||f|| on the recursive residual.  Returns iterations;
 * *relres gets the true final residual.  Returns -1 on breakdown. */
int orc_cocg(int nx, int ny, int nz, double hx, double hy, double hz, int N,
             double kre, double kim, const double *f, double *u, double tol, int maxit,
             double *relres)
{
    long n = (long)nx * ny * nz;
    double *r = malloc(sizeof(double) * 2 * n), *p = malloc(sizeof(double) * 2 * n);
    double *Ap = malloc(sizeof(double) * 2 * n);
    int it = 0, status = 0;
    /* r = f - A u,  A u = -L u + kappa u */
    orc_laplacian_z(nx, ny, nz, hx, hy, hz, N, u, Ap);
    for (long i = 0; i < n; ++i) {
        double ar = -Ap[2 * i] + kre * u[2 * i] - kim * u[2 * i + 1];
        double ai = -Ap[2 * i + 1] + kre * u[2 * i + 1] + kim * u[2 * i];
        r[2 * i] = f[2 * i] - ar;
        r[2 * i + 1] = f[2 * i + 1] - ai;
    }
    memcpy(p, r, sizeof(double) * 2 * n);
    double fnorm = znorm(n, f);
    double rr_re, rr_im;
    zdotu(n, r, r, &rr_re, &rr_im);
    while (it < maxit && znorm(n, r) > tol * fnorm) {
        orc_laplacian_z(nx, ny, nz, hx, hy, hz, N, p, Ap);
        for (long i = 0; i < n; ++i) {
            double ar = -Ap[2 * i] + kre * p[2 * i] - kim * p[2 * i + 1];
            double ai = -Ap[2 * i + 1] + kre * p[2 * i + 1] + kim * p[2 * i];
            Ap[2 * i] = ar;
            Ap[2 * i + 1] = ai;
        }
        double pa_re, pa_im;
        zdotu(n, p, Ap, &pa_re, &pa_im);
        double den = pa_re * pa_re + pa_im * pa_im;
        if (den == 0.0) { status = -1; break; }
        /* alpha = (r.r) / (p.Ap) */
        double al_re = (rr_re * pa_re + rr_im * pa_im) / den;
        double al_im = (rr_im * pa_re - rr_re * pa_im) / den;
        for (long i = 0; i < n; ++i) {
            u[2 * i] += al_re * p[2 * i] - al_im * p[2 * i + 1];
            u[2 * i + 1] += al_re * p[2 * i + 1] + al_im * p[2 * i];
            r[2 * i] -= al_re * Ap[2 * i] - al_im * Ap[2 * i + 1];
            r[2 * i + 1] -= al_re * Ap[2 * i + 1] + al_im * Ap[2 * i];
        }
        double nr_re, nr_im;
        zdotu(n, r, r, &nr_re, &nr_im);
        double d2 = rr_re * rr_re + rr_im * rr_im;
        if (d2 == 0.0) { status = -1; break; }
        double be_re = (nr_re * rr_re + nr_im * rr_im) / d2;
        double be_im = (nr_im * rr_re - nr_re * rr_im) / d2;
        rr_re = nr_re; rr_im = nr_im;
        for (long i = 0; i < n; ++i) {
            double pr = p[2 * i], pi = p[2 * i + 1];
            p[2 * i] = r[2 * i] + be_re * pr - be_im * pi;
            p[2 * i + 1] = r[2 * i + 1] + be_re * pi + be_im * pr;
        }
        ++it;
    }
    orc_laplacian_z(nx, ny, nz, hx, hy, hz, N, u, Ap);
    for (long i = 0; i < n; ++i) {
        double ar = -Ap[2 * i] + kre * u[2 * i] - kim * u[2 * i + 1];
        double ai = -Ap[2 * i + 1] + kre * u[2 * i + 1] + kim * u[2 * i];
        r[2 * i] = f[2 * i] - ar;
        r[2 * i + 1] = f[2 * i + 1] - ai;
    }
    *relres = znorm(n, r) / fnorm;
    free(r); free(p); free(Ap);
    return status < 0 ? status : it;
}

/* Number of OpenMP threads the oracle runs with (for reporting). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads of later calls (n >= 1), for timing the
 * oracle on one core and on all of them. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
