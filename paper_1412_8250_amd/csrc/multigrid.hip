// Geometric multigrid V-cycle (see multigrid.hpp) and the Poisson form that
// uses it as the preconditioner of CG.
#include <algorithm>
#include <cmath>
#include <utility>

#include "fcg.hpp"
#include "multigrid.hpp"
#include "profile.hpp"

namespace ofdft {

namespace {

constexpr int kMgThreads = 256;

struct MgDims {
    int nx, ny, nz;
    double cx, cy, cz, diag;
    double kre, kim;          // shift kappa of A = -Delta_h + kappa
    int64_t n;
};

MgDims dims_of(const MgLevel &L, double2 kappa) {
    return MgDims{L.nx, L.ny, L.nz, L.cx, L.cy, L.cz, 2.0 * (L.cx + L.cy + L.cz), kappa.x, kappa.y, L.n};
}

// Launch geometry: 64 x 4 threads over (x, y), one z plane per block row of
// the grid, so point coordinates come from the launch indices (no divisions).
constexpr int kMgBX = 64, kMgBY = 4;
static_assert(kMgBX * kMgBY == kMgThreads, "block shape");

dim3 mg_grid(int nx, int ny, int nz) { return dim3((nx + kMgBX - 1) / kMgBX, (ny + kMgBY - 1) / kMgBY, nz); }

struct MgPt {
    int x, y, z;
    int64_t i;
};

__device__ inline bool mg_point(int nx, int ny, MgPt &p) {
    p.x = blockIdx.x * kMgBX + threadIdx.x;
    p.y = blockIdx.y * kMgBY + threadIdx.y;
    p.z = blockIdx.z;
    p.i = ((int64_t)p.z * ny + p.y) * nx + p.x;
    return p.x < nx && p.y < ny;
}

// Element arithmetic for real (Poisson) and complex (shifted) levels.
__device__ inline double mg_scale(double2 s, double v) { return s.x * v; }
__device__ inline double2 mg_scale(double2 s, double2 v) {
    return make_double2(s.x * v.x - s.y * v.y, s.x * v.y + s.y * v.x);
}
__device__ inline double mg_axpy(double a, double x, double y) { return ::fma(a, x, y); }
__device__ inline double2 mg_axpy(double a, double2 x, double2 y) {
    return make_double2(::fma(a, x.x, y.x), ::fma(a, x.y, y.y));
}

// (A u) at p for the periodic 7-point operator A = -Delta_h + kappa (second order).
template <typename T>
__device__ inline T apply7(const T *__restrict__ u, const MgDims &d, const MgPt &p) {
    using V = VT<T>;
    const int64_t i = p.i, nxy = (int64_t)d.nx * d.ny;
    const int64_t xp = p.x + 1 == d.nx ? i - p.x : i + 1;
    const int64_t xm = p.x == 0 ? i + d.nx - 1 : i - 1;
    const int64_t yp = p.y + 1 == d.ny ? i - (int64_t)p.y * d.nx : i + d.nx;
    const int64_t ym = p.y == 0 ? i + (int64_t)(d.ny - 1) * d.nx : i - d.nx;
    const int64_t zp = p.z + 1 == d.nz ? i - (int64_t)p.z * nxy : i + nxy;
    const int64_t zm = p.z == 0 ? i + (int64_t)(d.nz - 1) * nxy : i - nxy;
    const T c = u[i];
    T a = V::mul(d.diag, c);
    a = mg_axpy(-d.cx, V::add(u[xp], u[xm]), a);
    a = mg_axpy(-d.cy, V::add(u[yp], u[ym]), a);
    a = mg_axpy(-d.cz, V::add(u[zp], u[zm]), a);
    return V::add(a, mg_scale(make_double2(d.kre, d.kim), c));
}

// Per-launch shift source: when `kap` is given, kappa is read from device
// memory (so a captured launch follows the current shift); when `run` is
// given the kernel returns at once unless *run == 0 (a converged system of a
// batch).
struct MgShift {
    const double *kap;
    const int *run;
};

// Returns false when the launch is to be skipped; otherwise sets d's shift.
__device__ inline bool take_shift(const MgShift &sh, MgDims &d) {
    if (sh.run && *sh.run != 0) return false;
    if (sh.kap) {
        d.kre = sh.kap[0];
        d.kim = sh.kap[1];
    }
    return true;
}

// omega / (diag + kappa)
__device__ inline double2 jacobi_factor(const MgDims &d, double w) {
    const double re = d.diag + d.kre, im = d.kim, den = re * re + im * im;
    return make_double2(w * re / den, -w * im / den);
}

// The two pre-smoothing sweeps from u = 0 in one pass: with the Jacobi factor
// s = omega / (diag + kappa), u1 = s f and u2 = u1 + s (f - A u1) = s (2 f - s A f).
template <typename T>
__global__ void __launch_bounds__(kMgThreads) mg_pre2(MgDims d, double w, const T *__restrict__ f,
                                                      T *__restrict__ u, MgShift sh) {
    if (!take_shift(sh, d)) return;
    MgPt p;
    if (!mg_point(d.nx, d.ny, p)) return;
    using V = VT<T>;
    const double2 s = jacobi_factor(d, w);
    const T af = apply7(f, d, p);
    const T two_f = V::add(f[p.i], f[p.i]);
    u[p.i] = mg_scale(s, V::sub(two_f, mg_scale(s, af)));
}

// t = u + omega (f - A u) / (diag + kappa)
template <typename T>
__global__ void __launch_bounds__(kMgThreads) mg_smooth(MgDims d, double w, const T *__restrict__ f,
                                                        const T *__restrict__ u, T *__restrict__ t,
                                                        MgShift sh) {
    if (!take_shift(sh, d)) return;
    MgPt p;
    if (!mg_point(d.nx, d.ny, p)) return;
    using V = VT<T>;
    const double2 s = jacobi_factor(d, w);
    t[p.i] = V::add(u[p.i], mg_scale(s, V::sub(f[p.i], apply7(u, d, p))));
}

// r = f - A u
template <typename T>
__global__ void __launch_bounds__(kMgThreads) mg_residual(MgDims d, const T *__restrict__ f,
                                                          const T *__restrict__ u, T *__restrict__ r,
                                                          MgShift sh) {
    if (!take_shift(sh, d)) return;
    MgPt p;
    if (!mg_point(d.nx, d.ny, p)) return;
    r[p.i] = VT<T>::sub(f[p.i], apply7(u, d, p));
}

// Full weighting: fc[I] = sum over the 27 fine points around 2I of
// (1/8) w(dx) w(dy) w(dz) r, w(0) = 1, w(+-1) = 1/2 (= P^T / 8).
template <typename T>
__global__ void __launch_bounds__(kMgThreads) mg_restrict(MgDims fd, MgDims cd, const T *__restrict__ r,
                                                          T *__restrict__ fc, MgShift sh) {
    if (sh.run && *sh.run != 0) return;
    MgPt P;
    if (!mg_point(cd.nx, cd.ny, P)) return;
    using V = VT<T>;
    const int64_t fnxy = (int64_t)fd.nx * fd.ny;
    int xs[3], ys[3], zs[3];
    xs[0] = P.x == 0 ? fd.nx - 1 : 2 * P.x - 1;
    xs[1] = 2 * P.x;
    xs[2] = 2 * P.x + 1;         // fine axes are even, so 2X + 1 < n
    ys[0] = P.y == 0 ? fd.ny - 1 : 2 * P.y - 1;
    ys[1] = 2 * P.y;
    ys[2] = 2 * P.y + 1;
    zs[0] = P.z == 0 ? fd.nz - 1 : 2 * P.z - 1;
    zs[1] = 2 * P.z;
    zs[2] = 2 * P.z + 1;
    T acc = V::zero();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double wz = c == 1 ? 1.0 : 0.5;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double wy = b == 1 ? wz : 0.5 * wz;
            const int64_t row = (int64_t)zs[c] * fnxy + (int64_t)ys[b] * fd.nx;
#pragma unroll
            for (int a = 0; a < 3; ++a) acc = mg_axpy(a == 1 ? wy : 0.5 * wy, r[row + xs[a]], acc);
        }
    }
    fc[P.i] = V::mul(0.125, acc);
}

// Trilinear prolongation added to u: fine index i takes coarse i/2 (even i)
// or the mean of coarse (i-1)/2 and (i+1)/2 (odd i), per axis.
template <typename T>
__global__ void __launch_bounds__(kMgThreads) mg_prolong_add(MgDims fd, MgDims cd, const T *__restrict__ uc,
                                                             T *__restrict__ u, MgShift sh) {
    if (sh.run && *sh.run != 0) return;
    MgPt p;
    if (!mg_point(fd.nx, fd.ny, p)) return;
    const int64_t cnxy = (int64_t)cd.nx * cd.ny;
    const int x0 = p.x >> 1, y0 = p.y >> 1, z0 = p.z >> 1;
    const int x1 = (p.x & 1) ? (x0 + 1 == cd.nx ? 0 : x0 + 1) : x0;
    const int y1 = (p.y & 1) ? (y0 + 1 == cd.ny ? 0 : y0 + 1) : y0;
    const int z1 = (p.z & 1) ? (z0 + 1 == cd.nz ? 0 : z0 + 1) : z0;
    const int64_t r00 = (int64_t)z0 * cnxy + (int64_t)y0 * cd.nx, r01 = (int64_t)z0 * cnxy + (int64_t)y1 * cd.nx;
    const int64_t r10 = (int64_t)z1 * cnxy + (int64_t)y0 * cd.nx, r11 = (int64_t)z1 * cnxy + (int64_t)y1 * cd.nx;
    // the 8 corner weights are 1/8 each; duplicated corners (even indices)
    // add up to the weights 1, 1/2, 1/4 of fewer distinct points
    using V = VT<T>;
    T acc = V::zero();
    acc = V::add(acc, V::add(uc[r00 + x0], uc[r00 + x1]));
    acc = V::add(acc, V::add(uc[r01 + x0], uc[r01 + x1]));
    acc = V::add(acc, V::add(uc[r10 + x0], uc[r10 + x1]));
    acc = V::add(acc, V::add(uc[r11 + x0], uc[r11 + x1]));
    u[p.i] = mg_axpy(0.125, acc, u[p.i]);
}

// Exact solve on the coarsest grid (at most 16^3 points, one workgroup):
// A is diagonalised by the DFT, eigenvalue sum_a c_a (2 - 2 cos(2 pi k_a / n_a))
// + kappa; with kappa = 0 the k = 0 (constant) component is set to zero.
__device__ void dft_axis(const double2 *in, double2 *out, int nx, int ny, int nz, int axis, double sign) {
    const int n = nx * ny * nz;
    const int len = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const int stride = axis == 0 ? 1 : (axis == 1 ? nx : nx * ny);
    for (int o = threadIdx.x; o < n; o += blockDim.x) {
        const int x = o % nx, y = (o / nx) % ny, z = o / (nx * ny);
        const int k = axis == 0 ? x : (axis == 1 ? y : z);
        const int base = o - k * stride;
        double re = 0.0, im = 0.0;
        for (int j = 0; j < len; ++j) {
            double sn, cs;
            sincospi(2.0 * (double)((j * k) % len) / (double)len, &sn, &cs);
            sn *= sign;
            const double2 v = in[base + j * stride];
            re += v.x * cs - v.y * sn;
            im += v.x * sn + v.y * cs;
        }
        out[o] = make_double2(re, im);
    }
}

__device__ inline double2 mg_to_c(double v) { return make_double2(v, 0.0); }
__device__ inline double2 mg_to_c(double2 v) { return v; }
__device__ inline void mg_from_c(double2 v, double &o) { o = v.x; }
__device__ inline void mg_from_c(double2 v, double2 &o) { o = v; }

template <typename T>
__global__ void __launch_bounds__(kMgThreads) mg_coarse_solve(MgDims d, const T *__restrict__ f,
                                                              T *__restrict__ u, MgShift sh) {
    if (!take_shift(sh, d)) return;
    __shared__ double2 a[kMgCoarseMax * kMgCoarseMax * kMgCoarseMax];
    __shared__ double2 b[kMgCoarseMax * kMgCoarseMax * kMgCoarseMax];
    const int n = (int)d.n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = mg_to_c(f[i]);
    __syncthreads();
    dft_axis(a, b, d.nx, d.ny, d.nz, 0, -1.0);
    __syncthreads();
    dft_axis(b, a, d.nx, d.ny, d.nz, 1, -1.0);
    __syncthreads();
    dft_axis(a, b, d.nx, d.ny, d.nz, 2, -1.0);
    __syncthreads();
    for (int o = threadIdx.x; o < n; o += blockDim.x) {
        const int x = o % d.nx, y = (o / d.nx) % d.ny, z = o / (d.nx * d.ny);
        const double lr = d.cx * (2.0 - 2.0 * cospi(2.0 * x / d.nx)) +
                          d.cy * (2.0 - 2.0 * cospi(2.0 * y / d.ny)) +
                          d.cz * (2.0 - 2.0 * cospi(2.0 * z / d.nz)) + d.kre;
        const double li = d.kim, den = lr * lr + li * li;
        double2 v = b[o];
        if (den == 0.0) {
            v = make_double2(0.0, 0.0);
        } else {   // v / (lr + i li) / n
            const double sr = lr / (den * n), si = -li / (den * n);
            v = make_double2(v.x * sr - v.y * si, v.x * si + v.y * sr);
        }
        b[o] = v;
    }
    __syncthreads();
    dft_axis(b, a, d.nx, d.ny, d.nz, 0, 1.0);
    __syncthreads();
    dft_axis(a, b, d.nx, d.ny, d.nz, 1, 1.0);
    __syncthreads();
    dft_axis(b, a, d.nx, d.ny, d.nz, 2, 1.0);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) mg_from_c(a[i], u[i]);
}

template <typename T>
int vcycle(Multigrid &mg, int l, double2 kappa, MgShift sh, hipStream_t s) {
    MgLevel &L = mg.lv[l];
    const MgDims d = dims_of(L, kappa);
    T *f = (T *)L.f;
    if (l + 1 == (int)mg.lv.size()) {
        hipLaunchKernelGGL(mg_coarse_solve<T>, dim3(1), dim3(kMgThreads), 0, s, d, f, (T *)L.u, sh);
        OFDFT_CHECK_HIP(hipGetLastError());
        return OFDFT_OK;
    }
    const dim3 grid = mg_grid(L.nx, L.ny, L.nz), block(kMgBX, kMgBY);
    // V(2,2): both pre-sweeps in one pass into u, residual, coarse
    // correction added to u, two post-sweeps (u -> t -> u)
    T *u = (T *)L.u, *t = (T *)L.t;
    hipLaunchKernelGGL(mg_pre2<T>, grid, block, 0, s, d, mg.omega, f, u, sh);
    hipLaunchKernelGGL(mg_residual<T>, grid, block, 0, s, d, f, u, (T *)L.r, sh);
    MgLevel &C = mg.lv[l + 1];
    const MgDims cd = dims_of(C, kappa);
    hipLaunchKernelGGL(mg_restrict<T>, mg_grid(C.nx, C.ny, C.nz), block, 0, s, d, cd, (const T *)L.r,
                       (T *)C.f, sh);
    OFDFT_CHECK_HIP(hipGetLastError());
    OFDFT_TRY(vcycle<T>(mg, l + 1, kappa, sh, s));
    hipLaunchKernelGGL(mg_prolong_add<T>, grid, block, 0, s, d, cd, (const T *)C.u, u, sh);
    hipLaunchKernelGGL(mg_smooth<T>, grid, block, 0, s, d, mg.omega, f, u, t, sh);
    hipLaunchKernelGGL(mg_smooth<T>, grid, block, 0, s, d, mg.omega, f, t, u, sh);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

}  // namespace

int mg_create(Multigrid &mg, const ofdft_grid &g, int elem_bytes) {
    mg_free(mg);
    if (elem_bytes != 8 && elem_bytes != 16) return OFDFT_INVALID_ARG;
    if (g.nz > 65535) {             // one z plane per grid row of the launches
        set_error("multigrid: nz = %d exceeds 65535", g.nz);
        return OFDFT_INVALID_ARG;
    }
    mg.elem = elem_bytes;
    MgLevel L;
    L.nx = g.nx;
    L.ny = g.ny;
    L.nz = g.nz;
    L.cx = 1.0 / (g.hx * g.hx);
    L.cy = 1.0 / (g.hy * g.hy);
    L.cz = 1.0 / (g.hz * g.hz);
    for (;;) {
        L.n = (int64_t)L.nx * L.ny * L.nz;
        mg.lv.push_back(L);
        const bool small = L.nx <= kMgCoarseMax && L.ny <= kMgCoarseMax && L.nz <= kMgCoarseMax;
        if (small) break;
        if (L.nx % 2 || L.ny % 2 || L.nz % 2) {
            set_error("multigrid: grid %dx%dx%d cannot be halved down to %d per axis", g.nx, g.ny, g.nz,
                      kMgCoarseMax);
            mg.lv.clear();
            return OFDFT_INVALID_ARG;
        }
        L.nx /= 2;
        L.ny /= 2;
        L.nz /= 2;
        L.cx /= 4.0;
        L.cy /= 4.0;
        L.cz /= 4.0;
    }
    for (size_t l = 0; l < mg.lv.size(); ++l) {
        MgLevel &M = mg.lv[l];
        const size_t b = (size_t)elem_bytes * (size_t)M.n;
        void **own[4] = {&M.t, &M.r, &M.u, &M.f};
        const int count = l == 0 ? 2 : 4;          // level 0 uses the caller's r and z
        for (int k = 0; k < count; ++k) {
            void *p = nullptr;
            if (hipMalloc(&p, b) != hipSuccess) {
                mg_free(mg);
                set_error("multigrid: out of device memory");
                return OFDFT_NO_MEMORY;
            }
            mg.allocs.push_back(p);
            *own[k] = p;
        }
    }
    return OFDFT_OK;
}

void mg_free(Multigrid &mg) {
    for (void *p : mg.allocs) (void)hipFree(p);
    mg.allocs.clear();
    mg.lv.clear();
}

int mg_apply(Multigrid &mg, const double *r, double *z, hipStream_t s, double kappa) {
    if (mg.lv.empty() || mg.elem != 8) return OFDFT_INVALID_ARG;
    MgLevel &L0 = mg.lv[0];
    L0.f = const_cast<double *>(r);
    L0.u = z;
    ProfScope ps(K_MULTIGRID, mg_cycle_bytes(mg), s);
    return vcycle<double>(mg, 0, make_double2(kappa, 0.0), MgShift{nullptr, nullptr}, s);
}

int mg_apply_shifted(Multigrid &mg, const double2 *r, double2 *z, const double *kappa, const int *run,
                     hipStream_t s) {
    if (mg.lv.empty() || mg.elem != 16 || !kappa) return OFDFT_INVALID_ARG;
    MgLevel &L0 = mg.lv[0];
    L0.f = const_cast<double2 *>(r);
    L0.u = z;
    return vcycle<double2>(mg, 0, make_double2(0.0, 0.0), MgShift{kappa, run}, s);
}

// Algorithmic bytes of one cycle on the fine level (the coarser levels add
// about 1/7): pre-smoothing reads f and writes u, the residual and each
// post-sweep read f, u and write one array, restriction reads r and writes
// an eighth, prolongation reads and writes u.
double mg_cycle_bytes(const Multigrid &mg) {
    if (mg.lv.empty()) return 0.0;
    const double e = (double)mg.elem;
    return (double)mg.lv[0].n * e * (2.0 + 3.0 * 3 + 1.125 + 2.0) * 8.0 / 7.0;
}

// CG on the projected Poisson system preconditioned by the V-cycle (flexible
// CG form, which equals preconditioned CG for this fixed SPD operator).
int poisson_solve_mg(ofdft_poisson *s, double *x, double rel_tol, int max_iter, ofdft_solve_stats &stats,
                     hipStream_t st) {
    const ofdft_grid &g = s->g;
    const int64_t n = npoints(g);
    double *r = s->r, *p = s->pA, *r_old = s->pB, *Ap = s->Ap, *z = s->z;
    double *tot = s->totals + 8, *th = s->totals_host + 8;
    auto sync_tot = [&](int count) -> int {
        OFDFT_CHECK_HIP(hipMemcpyAsync(th, tot, sizeof(double) * count, hipMemcpyDeviceToHost, st));
        OFDFT_CHECK_HIP(hipStreamSynchronize(st));
        return OFDFT_OK;
    };
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->totals_host, s->totals, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    const double g2 = s->totals_host[3];
    const double tol2 = rel_tol * rel_tol * g2;
    OFDFT_TRY(residual_pass<double>(g, s->coef, x, s->gp, r, tot, s->rb, st));
    OFDFT_TRY(sync_tot(2));
    double r2 = th[1];
    int iters = 0;
    stats.iters = 0;
    if (!std::isfinite(r2)) return OFDFT_NONFINITE;
    if (r2 <= tol2) return OFDFT_OK;
    if (max_iter <= 0) return OFDFT_NOT_CONVERGED;
    OFDFT_TRY(mg_apply(*s->mg, r, z, st));
    OFDFT_TRY((launch_reduce<2>(n, FcgDotsOp{z, r, r}, StoreTotals<2>{tot}, s->rb, st)));
    OFDFT_TRY(sync_tot(2));
    double rz = th[1];
    OFDFT_TRY((launch_reduce<1>(n, CopyOp2{p, z}, NoFin{}, s->rb, st)));
    int status = OFDFT_NOT_CONVERGED;
    while (iters < max_iter) {
        OFDFT_TRY(pass64(g, s->coef, LoadPlain<double>{p}, EpiAp{Ap, tot, s->rb.partials, s->rb.counter, 0.0},
                         st, 16.0, K_CG_STENCIL));
        OFDFT_TRY(sync_tot(1));
        const double pAp = th[0];
        if (!std::isfinite(pAp) || !std::isfinite(rz)) {
            status = OFDFT_NONFINITE;
            break;
        }
        if (!(pAp > 0.0) || !(rz > 0.0)) {
            status = OFDFT_BREAKDOWN;
            break;
        }
        const double a = rz / pAp;
        OFDFT_TRY((launch_reduce<1>(n, FcgStepOp{x, r, r_old, p, Ap, a}, StoreTotals<1>{tot}, s->rb, st)));
        OFDFT_TRY(sync_tot(1));
        r2 = th[0];
        ++iters;
        if (!std::isfinite(r2)) {
            status = OFDFT_NONFINITE;
            break;
        }
        if (r2 <= tol2) {
            status = OFDFT_OK;
            break;
        }
        OFDFT_TRY(mg_apply(*s->mg, r, z, st));
        OFDFT_TRY((launch_reduce<2>(n, FcgDotsOp{z, r, r_old}, StoreTotals<2>{tot}, s->rb, st)));
        OFDFT_TRY(sync_tot(2));
        const double b = th[0] / rz;
        rz = th[1];
        OFDFT_TRY((launch_reduce<1>(n, DirOp{p, z, std::isfinite(b) ? b : 0.0}, NoFin{}, s->rb, st)));
    }
    stats.iters = iters;
    return status;
}

}  // namespace ofdft

using namespace ofdft;

// z = M r for a multigrid solver (for inspection and for callers that build
// their own Krylov loop around the preconditioner).
extern "C" int ofdft_poisson_apply_preconditioner(ofdft_poisson *s, const double *r, double *z,
                                                  void *stream) {
    if (!s || !r || !z || r == z || s->mode != OFDFT_MULTIGRID || !s->mg) {
        set_error("ofdft_poisson_apply_preconditioner: multigrid solver and distinct r, z required");
        return OFDFT_INVALID_ARG;
    }
    return mg_apply(*s->mg, r, z, (hipStream_t)stream);
}
