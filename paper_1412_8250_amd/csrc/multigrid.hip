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

// Launch geometry: 64 x 4 threads over (x, y); each thread runs down a
// column of kMgKZ consecutive z planes (grid z = chunks), keeping the column's
// values in registers so that the z neighbours are loaded once.  Point
// coordinates come from the launch indices (no divisions).
constexpr int kMgBX = 64, kMgBY = 4, kMgKZ = 4;
static_assert(kMgBX * kMgBY == kMgThreads, "block shape");

// z chunks of one system; the systems of a launch are stacked along grid z
__host__ __device__ inline int mg_zch(int nz) { return (nz + kMgKZ - 1) / kMgKZ; }

dim3 mg_grid(int nx, int ny, int nz, int count = 1) {
    return dim3((nx + kMgBX - 1) / kMgBX, (ny + kMgBY - 1) / kMgBY, mg_zch(nz) * count);
}

struct MgPt {
    int x, y, z;     // z: first plane of the thread's column chunk
    int64_t i;       // index of (x, y, z)
};

// System of the workgroup within its launch (grid z = system * chunks + chunk).
__device__ inline int mg_sys(int nz) { return blockIdx.z / mg_zch(nz); }

__device__ inline bool mg_point(int nx, int ny, int nz, MgPt &p) {
    p.x = blockIdx.x * kMgBX + threadIdx.x;
    p.y = blockIdx.y * kMgBY + threadIdx.y;
    p.z = (blockIdx.z - mg_sys(nz) * mg_zch(nz)) * kMgKZ;
    p.i = ((int64_t)p.z * ny + p.y) * nx + p.x;
    return p.x < nx && p.y < ny;
}

// Element types: the cycle's input f and output z are FP64 (real or complex);
// the levels' arrays are stored, and their arithmetic done, in S (FP64 or
// FP32, real or complex).  R is S's real type, C the complex scalar of that
// precision (the Jacobi factor and the shift).
template <typename S> struct MgT;
template <> struct MgT<double> { using R = double; using C = double2; };
template <> struct MgT<float> { using R = float; using C = float2; };
template <> struct MgT<double2> { using R = double; using C = double2; };
template <> struct MgT<float2> { using R = float; using C = float2; };

template <typename To> __device__ inline To cv(double v);
template <typename To> __device__ inline To cv(float v);
template <typename To> __device__ inline To cv(double2 v);
template <typename To> __device__ inline To cv(float2 v);
template <> __device__ inline double cv<double>(double v) { return v; }
template <> __device__ inline float cv<float>(double v) { return (float)v; }
template <> __device__ inline double cv<double>(float v) { return (double)v; }
template <> __device__ inline float cv<float>(float v) { return v; }
template <> __device__ inline double2 cv<double2>(double2 v) { return v; }
template <> __device__ inline float2 cv<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ inline double2 cv<double2>(float2 v) { return make_double2(v.x, v.y); }
template <> __device__ inline float2 cv<float2>(float2 v) { return v; }

__device__ inline double mg_scale(double2 s, double v) { return s.x * v; }
__device__ inline float mg_scale(float2 s, float v) { return s.x * v; }
__device__ inline double2 mg_scale(double2 s, double2 v) {
    return make_double2(s.x * v.x - s.y * v.y, s.x * v.y + s.y * v.x);
}
__device__ inline float2 mg_scale(float2 s, float2 v) {
    return make_float2(s.x * v.x - s.y * v.y, s.x * v.y + s.y * v.x);
}
__device__ inline double mg_axpy(double a, double x, double y) { return ::fma(a, x, y); }
__device__ inline float mg_axpy(float a, float x, float y) { return fmaf(a, x, y); }
__device__ inline double2 mg_axpy(double a, double2 x, double2 y) {
    return make_double2(::fma(a, x.x, y.x), ::fma(a, x.y, y.y));
}
__device__ inline float2 mg_axpy(float a, float2 x, float2 y) {
    return make_float2(fmaf(a, x.x, y.x), fmaf(a, x.y, y.y));
}

template <typename C> __device__ inline C mk_c(double a, double b);
template <> __device__ inline double2 mk_c<double2>(double a, double b) { return make_double2(a, b); }
template <> __device__ inline float2 mk_c<float2>(double a, double b) { return make_float2((float)a, (float)b); }

// A u on the thread's column chunk for the periodic 7-point operator
// A = -Delta_h + kappa (second order), u of element type TI, computed in S:
// au[k] and the centre values cen[k] for planes p.z + k, k < kMgKZ (planes
// at or beyond nz are left unset).
template <typename S, typename TI>
__device__ inline void apply7_col(const TI *__restrict__ u, const MgDims &d, const MgPt &p, S (&cen)[kMgKZ],
                                  S (&au)[kMgKZ]) {
    using V = VT<S>;
    using R = typename MgT<S>::R;
    using C = typename MgT<S>::C;
    const int64_t nxy = (int64_t)d.nx * d.ny;
    const int64_t row = (int64_t)p.y * d.nx + p.x;
    const int dxp = p.x + 1 == d.nx ? -p.x : 1, dxm = p.x == 0 ? d.nx - 1 : -1;
    const int64_t dyp = p.y + 1 == d.ny ? -(int64_t)p.y * d.nx : d.nx;
    const int64_t dym = p.y == 0 ? (int64_t)(d.ny - 1) * d.nx : -(int64_t)d.nx;
    S col[kMgKZ + 2];
#pragma unroll
    for (int k = 0; k < kMgKZ + 2; ++k) {
        int z = p.z - 1 + k;
        z = z < 0 ? z + d.nz : (z >= d.nz ? z - d.nz : z);
        z = z >= d.nz ? d.nz - 1 : z;        // chunk tail past nz: any valid plane
        col[k] = cv<S>(u[(int64_t)z * nxy + row]);
    }
    const C kap = mk_c<C>(d.kre, d.kim);
#pragma unroll
    for (int k = 0; k < kMgKZ; ++k) {
        if (p.z + k < d.nz) {
            const int64_t i = (int64_t)(p.z + k) * nxy + row;
            const S c = col[k + 1];
            S a = V::mul((R)d.diag, c);
            a = mg_axpy((R)-d.cx, V::add(cv<S>(u[i + dxp]), cv<S>(u[i + dxm])), a);
            a = mg_axpy((R)-d.cy, V::add(cv<S>(u[i + dyp]), cv<S>(u[i + dym])), a);
            a = mg_axpy((R)-d.cz, V::add(col[k], col[k + 2]), a);
            cen[k] = c;
            au[k] = V::add(a, mg_scale(kap, c));
        }
    }
}

// Per-launch shift source: when `kap` is given, kappa is read from device
// memory (so a captured launch follows the current shift); when `run` is
// given the kernel returns at once unless *run == 0 (a converged system of a
// batch).  System q of a launch reads kap + q kstride and run + q rstride.
struct MgShift {
    const double *kap;
    const int *run;
    int kstride, rstride;
    __device__ bool skip(int q) const { return run && run[(int64_t)q * rstride] != 0; }
};

// An array of every system of a launch: system q's part starts at
// base + q stride, or at tab[q] (a device table of the callers' arrays).
template <typename P>
struct MgArr {
    P *base;
    int64_t stride;
    P *const *tab;
    __device__ P *at(int q) const { return tab ? tab[q] : (base ? base + (int64_t)q * stride : nullptr); }
};

// Returns false when system q is to be skipped; otherwise sets d's shift.
__device__ inline bool take_shift(const MgShift &sh, MgDims &d, int q) {
    if (sh.skip(q)) return false;
    if (sh.kap) {
        d.kre = sh.kap[(int64_t)q * sh.kstride];
        d.kim = sh.kap[(int64_t)q * sh.kstride + 1];
    }
    return true;
}

// omega / (diag + kappa)
template <typename C>
__device__ inline C jacobi_factor(const MgDims &d, double w) {
    const double re = d.diag + d.kre, im = d.kim, den = re * re + im * im;
    return mk_c<C>(w * re / den, -w * im / den);
}

// The two pre-smoothing sweeps from u = 0 in one pass: with the Jacobi factor
// s = omega / (diag + kappa), u1 = s f and u2 = u1 + s (f - A u1) = s (2 f - s A f).
// When fl is given, f is also stored there in S (the fine level's later
// passes then read the narrower copy).
template <typename TF, typename S>
__global__ void __launch_bounds__(kMgThreads) mg_pre2(MgDims d, double w, MgArr<const TF> fa, MgArr<S> ua,
                                                      MgArr<S> fla, MgShift sh) {
    const int q = mg_sys(d.nz);
    if (!take_shift(sh, d, q)) return;
    MgPt p;
    if (!mg_point(d.nx, d.ny, d.nz, p)) return;
    const TF *__restrict__ f = fa.at(q);
    S *__restrict__ u = ua.at(q);
    S *__restrict__ fl = fla.at(q);
    using V = VT<S>;
    const auto s = jacobi_factor<typename MgT<S>::C>(d, w);
    S fc[kMgKZ], af[kMgKZ];
    apply7_col(f, d, p, fc, af);
    const int64_t nxy = (int64_t)d.nx * d.ny;
#pragma unroll
    for (int k = 0; k < kMgKZ; ++k)
        if (p.z + k < d.nz) {
            const int64_t i = p.i + k * nxy;
            u[i] = mg_scale(s, V::sub(V::add(fc[k], fc[k]), mg_scale(s, af[k])));
            if (fl) fl[i] = fc[k];
        }
}

// t = u + omega (f - A u) / (diag + kappa), computed in S, stored as TO
template <typename TF, typename S, typename TO>
__global__ void __launch_bounds__(kMgThreads) mg_smooth(MgDims d, double w, MgArr<const TF> fa,
                                                        MgArr<const S> ua, MgArr<TO> ta, MgShift sh) {
    const int q = mg_sys(d.nz);
    if (!take_shift(sh, d, q)) return;
    MgPt p;
    if (!mg_point(d.nx, d.ny, d.nz, p)) return;
    const TF *__restrict__ f = fa.at(q);
    const S *__restrict__ u = ua.at(q);
    TO *__restrict__ t = ta.at(q);
    using V = VT<S>;
    const auto s = jacobi_factor<typename MgT<S>::C>(d, w);
    S uc[kMgKZ], au[kMgKZ];
    apply7_col(u, d, p, uc, au);
    const int64_t nxy = (int64_t)d.nx * d.ny;
#pragma unroll
    for (int k = 0; k < kMgKZ; ++k)
        if (p.z + k < d.nz) {
            const int64_t i = p.i + k * nxy;
            t[i] = cv<TO>(V::add(uc[k], mg_scale(s, V::sub(cv<S>(f[i]), au[k]))));
        }
}

// r = f - A u
template <typename TF, typename S>
__global__ void __launch_bounds__(kMgThreads) mg_residual(MgDims d, MgArr<const TF> fa, MgArr<const S> ua,
                                                          MgArr<S> ra, MgShift sh) {
    const int q = mg_sys(d.nz);
    if (!take_shift(sh, d, q)) return;
    MgPt p;
    if (!mg_point(d.nx, d.ny, d.nz, p)) return;
    const TF *__restrict__ f = fa.at(q);
    const S *__restrict__ u = ua.at(q);
    S *__restrict__ r = ra.at(q);
    S uc[kMgKZ], au[kMgKZ];
    apply7_col(u, d, p, uc, au);
    const int64_t nxy = (int64_t)d.nx * d.ny;
#pragma unroll
    for (int k = 0; k < kMgKZ; ++k)
        if (p.z + k < d.nz) {
            const int64_t i = p.i + k * nxy;
            r[i] = VT<S>::sub(cv<S>(f[i]), au[k]);
        }
}

// Full weighting: fc[I] = sum over the 27 fine points around 2I of
// (1/8) w(dx) w(dy) w(dz) r, w(0) = 1, w(+-1) = 1/2 (= P^T / 8).  A thread
// runs down kMgKZ coarse planes; each fine plane's 9-point (x, y) sum is
// formed once and shared by the coarse planes it touches.
template <typename S>
__global__ void __launch_bounds__(kMgThreads) mg_restrict(MgDims fd, MgDims cd, MgArr<const S> ra,
                                                          MgArr<S> fca, MgShift sh) {
    const int qs = mg_sys(cd.nz);
    if (sh.skip(qs)) return;
    MgPt P;
    if (!mg_point(cd.nx, cd.ny, cd.nz, P)) return;
    const S *__restrict__ r = ra.at(qs);
    S *__restrict__ fc = fca.at(qs);
    using V = VT<S>;
    using R = typename MgT<S>::R;
    const int64_t fnxy = (int64_t)fd.nx * fd.ny, cnxy = (int64_t)cd.nx * cd.ny;
    int xs[3];
    int64_t ys[3];
    xs[0] = P.x == 0 ? fd.nx - 1 : 2 * P.x - 1;
    xs[1] = 2 * P.x;
    xs[2] = 2 * P.x + 1;         // fine axes are even, so 2X + 1 < n
    ys[0] = (int64_t)(P.y == 0 ? fd.ny - 1 : 2 * P.y - 1) * fd.nx;
    ys[1] = (int64_t)(2 * P.y) * fd.nx;
    ys[2] = (int64_t)(2 * P.y + 1) * fd.nx;
    // plane sums q[j] for fine planes 2 Z0 - 1 + j, j = 0 .. 2 kMgKZ
    S q[2 * kMgKZ + 1];
#pragma unroll
    for (int j = 0; j < 2 * kMgKZ + 1; ++j) {
        int z = 2 * P.z - 1 + j;
        z = z < 0 ? z + fd.nz : (z >= fd.nz ? fd.nz - 1 : z);    // past the end: unused, any valid plane
        const int64_t base = (int64_t)z * fnxy;
        S acc = V::zero();
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const R wy = b == 1 ? (R)1 : (R)0.5;
            const S rowsum = V::add(mg_axpy((R)0.5, V::add(r[base + ys[b] + xs[0]], r[base + ys[b] + xs[2]]),
                                            V::zero()),
                                    r[base + ys[b] + xs[1]]);
            acc = mg_axpy(wy, rowsum, acc);
        }
        q[j] = acc;
    }
#pragma unroll
    for (int k = 0; k < kMgKZ; ++k)
        if (P.z + k < cd.nz) {
            const S sz = V::add(mg_axpy((R)0.5, V::add(q[2 * k], q[2 * k + 2]), V::zero()), q[2 * k + 1]);
            fc[P.i + k * cnxy] = V::mul((R)0.125, sz);
        }
}

// Coarse correction (P uc) on fine plane z + K (K = -1 .. kMgKZ) from the
// corner sums cs[j][c] of coarse block plane j (coarse plane z / 2 - 1 + j)
// for the fine column c: 1/4 of one plane's sum (even fine plane) or 1/8 of
// two (odd fine plane).
template <int K, int CI, typename S, int NZC>
__device__ __forceinline__ S mg_corr(const S (&cs)[NZC][5]) {
    using V = VT<S>;
    using R = typename MgT<S>::R;
    constexpr int J = (K + 2) >> 1;              // block plane of coarse plane (z + K) >> 1
    if constexpr (K & 1)
        return mg_axpy((R)0.125, V::add(cs[J][CI], cs[J + 1][CI]), V::zero());
    else
        return V::mul((R)0.25, cs[J][CI]);
}

// The first post-smoothing sweep with the coarse correction folded in:
// t = v + omega (f - A v) / (diag + kappa), v = u + P uc, with P the
// trilinear prolongation (per axis, fine index i takes coarse i/2 when i is
// even and the mean of coarse (i-1)/2 and (i+1)/2 when odd), formed in
// registers; v is never stored: it is the corrected u that the two
// post-sweeps start from.  The thread's column needs v on planes z - 1 ..
// z + kMgKZ at (x, y) and on planes z .. z + kMgKZ - 1 at the four (x, y)
// neighbours; their coarse corners lie in a 3 x 3 block of coarse columns
// around (x / 2, y / 2) on coarse planes z / 2 - 1 .. z / 2 + kMgKZ / 2, each
// loaded once.
template <typename TF, typename S>
__global__ void __launch_bounds__(kMgThreads) mg_prolong_smooth(MgDims d, MgDims cd, double w,
                                                                MgArr<const TF> fa, MgArr<const S> ua,
                                                                MgArr<const S> uca, MgArr<S> ta, MgShift sh) {
    const int q = mg_sys(d.nz);
    if (!take_shift(sh, d, q)) return;
    MgPt p;
    if (!mg_point(d.nx, d.ny, d.nz, p)) return;
    const TF *__restrict__ f = fa.at(q);
    const S *__restrict__ u = ua.at(q);
    const S *__restrict__ uc = uca.at(q);
    S *__restrict__ t = ta.at(q);
    using V = VT<S>;
    using R = typename MgT<S>::R;
    using C = typename MgT<S>::C;
    static_assert(kMgKZ % 2 == 0, "chunks start on even planes");
    constexpr int NZC = kMgKZ / 2 + 2;             // coarse planes z/2 - 1 .. z/2 + kMgKZ/2
    const int64_t nxy = (int64_t)d.nx * d.ny, cnxy = (int64_t)cd.nx * cd.ny;
    const int cx0 = p.x >> 1, cy0 = p.y >> 1;
    int64_t cxo[3], cyo[3];                        // block columns cx0 - 1 .. cx0 + 1, likewise y
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        int X = cx0 - 1 + m, Y = cy0 - 1 + m;
        X = X < 0 ? X + cd.nx : (X >= cd.nx ? X - cd.nx : X);
        Y = Y < 0 ? Y + cd.ny : (Y >= cd.ny ? Y - cd.ny : Y);
        cxo[m] = X;
        cyo[m] = (int64_t)Y * cd.nx;
    }
    // Corner sums of the fine columns c = 0: (x, y), 1: (x + 1, y), 2: (x - 1, y),
    // 3: (x, y + 1), 4: (x, y - 1) on each block plane j.  Per axis the fine
    // column at x + dx takes block columns (x0, x1) = (0, 1), (1, 1), (1, 2)
    // for dx = -1, 0, 1 when x is even and (1, 1), (1, 2), (2, 2) when odd
    // (grids are even, so the parity survives the periodic wrap); a corner sum
    // is (x0 + x1 on row y0) + (x0 + x1 on row y1).  The row sums are formed
    // for every candidate pair and the parity selects among the values.
    const bool px = p.x & 1, py = p.y & 1;
    S cs[NZC][5];
#pragma unroll
    for (int j = 0; j < NZC; ++j) {
        int Z = (p.z >> 1) - 1 + j;
        Z = Z < 0 ? Z + cd.nz : (Z >= cd.nz ? Z - cd.nz : Z);
        Z = Z >= cd.nz ? cd.nz - 1 : Z;            // chunk tail past the end: unused, any valid plane
        const int64_t b = (int64_t)Z * cnxy;
        S rm[3], r0[3], rp[3];                     // row sums for dx = -1, 0, +1 on block rows 0..2
#pragma unroll
        for (int my = 0; my < 3; ++my) {
            const S c0 = uc[b + cyo[my] + cxo[0]], c1 = uc[b + cyo[my] + cxo[1]], c2 = uc[b + cyo[my] + cxo[2]];
            const S s01 = V::add(c0, c1), s11 = V::add(c1, c1), s12 = V::add(c1, c2), s22 = V::add(c2, c2);
            rm[my] = px ? s11 : s01;
            r0[my] = px ? s12 : s11;
            rp[my] = px ? s22 : s12;
        }
        // rows (y0, y1): dy = 0 -> (1, 1) even / (1, 2) odd; +1 -> (1, 2) / (2, 2); -1 -> (0, 1) / (1, 1)
        cs[j][0] = py ? V::add(r0[1], r0[2]) : V::add(r0[1], r0[1]);
        cs[j][1] = py ? V::add(rp[1], rp[2]) : V::add(rp[1], rp[1]);
        cs[j][2] = py ? V::add(rm[1], rm[2]) : V::add(rm[1], rm[1]);
        cs[j][3] = py ? V::add(r0[2], r0[2]) : V::add(r0[1], r0[2]);
        cs[j][4] = py ? V::add(r0[1], r0[1]) : V::add(r0[0], r0[1]);
    }
    const int64_t row = (int64_t)p.y * d.nx + p.x;
    const int dxp = p.x + 1 == d.nx ? -p.x : 1, dxm = p.x == 0 ? d.nx - 1 : -1;
    const int64_t dyp = p.y + 1 == d.ny ? -(int64_t)p.y * d.nx : d.nx;
    const int64_t dym = p.y == 0 ? (int64_t)(d.ny - 1) * d.nx : -(int64_t)d.nx;
    // v on the centre column, planes z - 1 .. z + kMgKZ
    S col[kMgKZ + 2];
    static_for<0, kMgKZ + 2>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        int z = p.z - 1 + k;
        z = z < 0 ? z + d.nz : (z >= d.nz ? z - d.nz : z);
        z = z >= d.nz ? d.nz - 1 : z;              // chunk tail past nz: any valid plane
        col[k] = V::add(u[(int64_t)z * nxy + row], mg_corr<k - 1, 0>(cs));
    });
    const C kap = mk_c<C>(d.kre, d.kim);
    const auto s = jacobi_factor<C>(d, w);
    static_for<0, kMgKZ>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        if (p.z + k < d.nz) {
            const int64_t i = (int64_t)(p.z + k) * nxy + row;
            const S c = col[k + 1];
            const S vxp = V::add(u[i + dxp], mg_corr<k, 1>(cs));
            const S vxm = V::add(u[i + dxm], mg_corr<k, 2>(cs));
            const S vyp = V::add(u[i + dyp], mg_corr<k, 3>(cs));
            const S vym = V::add(u[i + dym], mg_corr<k, 4>(cs));
            S a = V::mul((R)d.diag, c);
            a = mg_axpy((R)-d.cx, V::add(vxp, vxm), a);
            a = mg_axpy((R)-d.cy, V::add(vyp, vym), a);
            a = mg_axpy((R)-d.cz, V::add(col[k], col[k + 2]), a);
            const S av = V::add(a, mg_scale(kap, c));
            t[i] = V::add(c, mg_scale(s, V::sub(cv<S>(f[i]), av)));
        }
    });
}

// Exact solve on the coarsest grid (at most 16^3 points, one workgroup, FP64):
// A is diagonalised by the DFT, eigenvalue sum_a c_a (2 - 2 cos(2 pi k_a / n_a))
// + kappa; with kappa = 0 the k = 0 (constant) component is set to zero.
// tw[m] = (cos, sin)(2 pi m / len) for m < len, one table per axis.
__device__ void dft_axis(const double2 *in, double2 *out, int nx, int ny, int nz, int axis, double sign,
                         const double2 *tw) {
    const int n = nx * ny * nz;
    const int len = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const int stride = axis == 0 ? 1 : (axis == 1 ? nx : nx * ny);
    for (int o = threadIdx.x; o < n; o += blockDim.x) {
        const int x = o % nx, y = (o / nx) % ny, z = o / (nx * ny);
        const int k = axis == 0 ? x : (axis == 1 ? y : z);
        const int base = o - k * stride;
        double re = 0.0, im = 0.0;
        int m = 0;                                 // (j k) mod len
        for (int j = 0; j < len; ++j) {
            const double cs = tw[m].x, sn = sign * tw[m].y;
            const double2 v = in[base + j * stride];
            re += v.x * cs - v.y * sn;
            im += v.x * sn + v.y * cs;
            m += k;
            if (m >= len) m -= len;
        }
        out[o] = make_double2(re, im);
    }
}

__device__ inline double2 mg_to_c(double v) { return make_double2(v, 0.0); }
__device__ inline double2 mg_to_c(float v) { return make_double2(v, 0.0); }
__device__ inline double2 mg_to_c(double2 v) { return v; }
__device__ inline double2 mg_to_c(float2 v) { return make_double2(v.x, v.y); }
__device__ inline void mg_from_c(double2 v, double &o) { o = v.x; }
__device__ inline void mg_from_c(double2 v, float &o) { o = (float)v.x; }
__device__ inline void mg_from_c(double2 v, double2 &o) { o = v; }
__device__ inline void mg_from_c(double2 v, float2 &o) { o = make_float2((float)v.x, (float)v.y); }

template <typename TI, typename TO>
__global__ void __launch_bounds__(kMgThreads) mg_coarse_solve(MgDims d, MgArr<const TI> fa, MgArr<TO> ua,
                                                              MgShift sh) {
    const int q = blockIdx.x;                  // one workgroup per system
    if (!take_shift(sh, d, q)) return;
    const TI *__restrict__ f = fa.at(q);
    TO *__restrict__ u = ua.at(q);
    __shared__ double2 a[kMgCoarseMax * kMgCoarseMax * kMgCoarseMax];
    __shared__ double2 b[kMgCoarseMax * kMgCoarseMax * kMgCoarseMax];
    __shared__ double2 tw[3][kMgCoarseMax];
    const int n = (int)d.n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = mg_to_c(f[i]);
    for (int i = threadIdx.x; i < 3 * kMgCoarseMax; i += blockDim.x) {
        const int ax = i / kMgCoarseMax, m = i % kMgCoarseMax;
        const int len = ax == 0 ? d.nx : (ax == 1 ? d.ny : d.nz);
        double sn = 0.0, cs = 1.0;
        if (m < len) sincospi(2.0 * (double)m / (double)len, &sn, &cs);
        tw[ax][m] = make_double2(cs, sn);
    }
    __syncthreads();
    dft_axis(a, b, d.nx, d.ny, d.nz, 0, -1.0, tw[0]);
    __syncthreads();
    dft_axis(b, a, d.nx, d.ny, d.nz, 1, -1.0, tw[1]);
    __syncthreads();
    dft_axis(a, b, d.nx, d.ny, d.nz, 2, -1.0, tw[2]);
    __syncthreads();
    for (int o = threadIdx.x; o < n; o += blockDim.x) {
        const int x = o % d.nx, y = (o / d.nx) % d.ny, z = o / (d.nx * d.ny);
        const double lr = d.cx * (2.0 - 2.0 * tw[0][x].x) + d.cy * (2.0 - 2.0 * tw[1][y].x) +
                          d.cz * (2.0 - 2.0 * tw[2][z].x) + d.kre;
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
    dft_axis(b, a, d.nx, d.ny, d.nz, 0, 1.0, tw[0]);
    __syncthreads();
    dft_axis(a, b, d.nx, d.ny, d.nz, 1, 1.0, tw[1]);
    __syncthreads();
    dft_axis(b, a, d.nx, d.ny, d.nz, 2, 1.0, tw[2]);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) mg_from_c(a[i], u[i]);
}

// Level array of systems q0 .. q0 + count - 1 of a hierarchy.
template <typename S>
MgArr<S> lvl(void *base, const MgLevel &L, int q0) {
    return MgArr<S>{base ? (S *)base + (int64_t)q0 * L.n : nullptr, L.n, nullptr};
}

// V(2,2) cycle on level l >= 1 (arrays of S) of `count` systems from q0: f -> u.
template <typename S>
int vcycle_coarse(Multigrid &mg, int l, int q0, int count, double2 kappa, MgShift sh, hipStream_t s) {
    MgLevel &L = mg.lv[l];
    const MgDims d = dims_of(L, kappa);
    const MgArr<S> f = lvl<S>(L.f, L, q0), u = lvl<S>(L.u, L, q0), t = lvl<S>(L.t, L, q0), r = lvl<S>(L.r, L, q0);
    const MgArr<const S> fc{f.base, f.stride, nullptr}, uc_{u.base, u.stride, nullptr},
        tc{t.base, t.stride, nullptr}, rc{r.base, r.stride, nullptr};
    if (l + 1 == (int)mg.lv.size()) {
        hipLaunchKernelGGL((mg_coarse_solve<S, S>), dim3(count), dim3(kMgThreads), 0, s, d, fc, u, sh);
        OFDFT_CHECK_HIP(hipGetLastError());
        return OFDFT_OK;
    }
    const dim3 grid = mg_grid(L.nx, L.ny, L.nz, count), block(kMgBX, kMgBY);
    MgLevel &C = mg.lv[l + 1];
    const MgDims cd = dims_of(C, kappa);
    const MgArr<S> cf = lvl<S>(C.f, C, q0);
    const MgArr<const S> cu{(const S *)C.u + (int64_t)q0 * C.n, C.n, nullptr};
    const MgArr<S> none{nullptr, 0, nullptr};
    hipLaunchKernelGGL((mg_pre2<S, S>), grid, block, 0, s, d, mg.omega, fc, u, none, sh);
    hipLaunchKernelGGL((mg_residual<S, S>), grid, block, 0, s, d, fc, uc_, r, sh);
    hipLaunchKernelGGL(mg_restrict<S>, mg_grid(C.nx, C.ny, C.nz, count), block, 0, s, d, cd, rc, cf, sh);
    OFDFT_CHECK_HIP(hipGetLastError());
    OFDFT_TRY(vcycle_coarse<S>(mg, l + 1, q0, count, kappa, sh, s));
    hipLaunchKernelGGL((mg_prolong_smooth<S, S>), grid, block, 0, s, d, cd, mg.omega, fc, uc_, cu, t, sh);
    hipLaunchKernelGGL((mg_smooth<S, S, S>), grid, block, 0, s, d, mg.omega, fc, tc, u, sh);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

// The whole cycle z = M f for `count` systems from q0 of the hierarchy: level
// 0 reads f and writes z in FP64 (TIO), its work arrays are S.  V(2,2): both
// pre-sweeps in one pass into u, residual, coarse correction folded into the
// first post-sweep u -> t, second post-sweep t -> z.  With S narrower than
// TIO the pre-sweep pass also stores f in S (level 0's f array), which the
// residual and the post-sweeps read instead of the FP64 input.  f, z and sh
// address system q0 first.
template <typename TIO, typename S>
int vcycle(Multigrid &mg, int q0, int count, MgArr<const TIO> f, MgArr<TIO> z, double2 kappa, MgShift sh,
           hipStream_t s) {
    MgLevel &L = mg.lv[0];
    const MgDims d = dims_of(L, kappa);
    if (mg.lv.size() == 1) {
        hipLaunchKernelGGL((mg_coarse_solve<TIO, TIO>), dim3(count), dim3(kMgThreads), 0, s, d, f, z, sh);
        OFDFT_CHECK_HIP(hipGetLastError());
        return OFDFT_OK;
    }
    const dim3 grid = mg_grid(L.nx, L.ny, L.nz, count), block(kMgBX, kMgBY);
    const MgArr<S> u = lvl<S>(L.u, L, q0), t = lvl<S>(L.t, L, q0), r = lvl<S>(L.r, L, q0);
    const MgArr<const S> uc_{u.base, u.stride, nullptr}, tc{t.base, t.stride, nullptr},
        rc{r.base, r.stride, nullptr};
    MgLevel &C = mg.lv[1];
    const MgDims cd = dims_of(C, kappa);
    const MgArr<S> cf = lvl<S>(C.f, C, q0);
    const MgArr<const S> cu{(const S *)C.u + (int64_t)q0 * C.n, C.n, nullptr};
    if constexpr (sizeof(S) < sizeof(TIO)) {
        const MgArr<S> fl = lvl<S>(L.f, L, q0);
        const MgArr<const S> flc{fl.base, fl.stride, nullptr};
        hipLaunchKernelGGL((mg_pre2<TIO, S>), grid, block, 0, s, d, mg.omega, f, u, fl, sh);
        hipLaunchKernelGGL((mg_residual<S, S>), grid, block, 0, s, d, flc, uc_, r, sh);
    } else {
        const MgArr<S> none{nullptr, 0, nullptr};
        hipLaunchKernelGGL((mg_pre2<TIO, S>), grid, block, 0, s, d, mg.omega, f, u, none, sh);
        hipLaunchKernelGGL((mg_residual<TIO, S>), grid, block, 0, s, d, f, uc_, r, sh);
    }
    hipLaunchKernelGGL(mg_restrict<S>, mg_grid(C.nx, C.ny, C.nz, count), block, 0, s, d, cd, rc, cf, sh);
    OFDFT_CHECK_HIP(hipGetLastError());
    OFDFT_TRY(vcycle_coarse<S>(mg, 1, q0, count, kappa, sh, s));
    if constexpr (sizeof(S) < sizeof(TIO)) {
        const MgArr<const S> flc{(const S *)L.f + (int64_t)q0 * L.n, L.n, nullptr};
        hipLaunchKernelGGL((mg_prolong_smooth<S, S>), grid, block, 0, s, d, cd, mg.omega, flc, uc_, cu, t, sh);
        hipLaunchKernelGGL((mg_smooth<S, S, TIO>), grid, block, 0, s, d, mg.omega, flc, tc, z, sh);
    } else {
        hipLaunchKernelGGL((mg_prolong_smooth<TIO, S>), grid, block, 0, s, d, cd, mg.omega, f, uc_, cu, t, sh);
        hipLaunchKernelGGL((mg_smooth<TIO, S, TIO>), grid, block, 0, s, d, mg.omega, f, tc, z, sh);
    }
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

}  // namespace

int mg_create(Multigrid &mg, const ofdft_grid &g, int elem_bytes, bool fp32, int groups) {
    mg_free(mg);
    if ((elem_bytes != 8 && elem_bytes != 16) || groups < 1) return OFDFT_INVALID_ARG;
    if ((int64_t)mg_zch(g.nz) * groups > 65535) {     // grid z = systems x z chunks
        set_error("multigrid: %d systems of %d planes exceed one launch", groups, g.nz);
        return OFDFT_INVALID_ARG;
    }
    if (g.nz > 65535) {             // one z plane per grid row of the launches
        set_error("multigrid: nz = %d exceeds 65535", g.nz);
        return OFDFT_INVALID_ARG;
    }
    mg.elem = elem_bytes;
    mg.fp32 = fp32;
    mg.groups = groups;
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
    const size_t es = fp32 ? (size_t)elem_bytes / 2 : (size_t)elem_bytes;
    const int nlev = (int)mg.lv.size();
    for (int l = 0; l < nlev; ++l) {
        MgLevel &M = mg.lv[l];
        const size_t b = es * (size_t)M.n * (size_t)groups;
        void **own[4] = {&M.t, &M.r, &M.u, &M.f};
        // level 0 reads the caller's f (and keeps an FP32 copy of it when the
        // levels are FP32); a one-level hierarchy needs nothing
        const int count = nlev == 1 ? 0 : (l == 0 && !fp32 ? 3 : 4);
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
    ProfScope ps(K_MULTIGRID, mg_cycle_bytes(mg), s);
    const double2 k = make_double2(kappa, 0.0);
    const MgShift sh{nullptr, nullptr, 0, 0};
    const MgArr<const double> f{r, 0, nullptr};
    const MgArr<double> o{z, 0, nullptr};
    return mg.fp32 ? vcycle<double, float>(mg, 0, 1, f, o, k, sh, s)
                   : vcycle<double, double>(mg, 0, 1, f, o, k, sh, s);
}

int mg_apply_run(Multigrid &mg, const double *r, double *z, hipStream_t s, double kappa, const int *run) {
    if (mg.lv.empty() || mg.elem != 8) return OFDFT_INVALID_ARG;
    ProfScope ps(K_MULTIGRID, 0.0, s);      // bytes: the caller counts the cycles that ran
    const double2 k = make_double2(kappa, 0.0);
    const MgShift sh{nullptr, run, 0, 0};
    const MgArr<const double> f{r, 0, nullptr};
    const MgArr<double> o{z, 0, nullptr};
    return mg.fp32 ? vcycle<double, float>(mg, 0, 1, f, o, k, sh, s)
                   : vcycle<double, double>(mg, 0, 1, f, o, k, sh, s);
}

int mg_apply_shifted(Multigrid &mg, int q, const double2 *r, double2 *z, const double *kappa, const int *run,
                     hipStream_t s) {
    if (mg.lv.empty() || mg.elem != 16 || !kappa || q < 0 || q >= mg.groups) return OFDFT_INVALID_ARG;
    const double2 k = make_double2(0.0, 0.0);
    const MgShift sh{kappa, run, 0, 0};
    const MgArr<const double2> f{r, 0, nullptr};
    const MgArr<double2> o{z, 0, nullptr};
    return mg.fp32 ? vcycle<double2, float2>(mg, q, 1, f, o, k, sh, s)
                   : vcycle<double2, double2>(mg, q, 1, f, o, k, sh, s);
}

int mg_apply_shifted_group(Multigrid &mg, int count, const double2 *const *r, double2 *const *z,
                           const double *kappa, int kstride, const int *run, int rstride, hipStream_t s) {
    if (mg.lv.empty() || mg.elem != 16 || !kappa || !r || !z || count < 1 || count > mg.groups)
        return OFDFT_INVALID_ARG;
    const double2 k = make_double2(0.0, 0.0);
    const MgShift sh{kappa, run, kstride, rstride};
    const MgArr<const double2> f{nullptr, 0, r};
    const MgArr<double2> o{nullptr, 0, z};
    return mg.fp32 ? vcycle<double2, float2>(mg, 0, count, f, o, k, sh, s)
                   : vcycle<double2, double2>(mg, 0, count, f, o, k, sh, s);
}

// Algorithmic bytes of one cycle.  Fine level, FP64 levels: f is read by the
// pre-smoothing, the residual and both post-sweeps, z written once, and the
// work arrays move 7.25 elements per point (u written; residual reads u and
// writes r; restriction reads r and writes an eighth; the first post-sweep
// reads u and an eighth (the coarse correction) and writes t; the second
// reads t).  FP32 levels: f (FP64) is read once and stored as FP32, which the
// other three passes read (4 more FP32 moves).  Each coarser level moves
// 12.25 elements per point, and they hold 1/7 of the fine points in all.
double mg_cycle_bytes(const Multigrid &mg) {
    if (mg.lv.empty()) return 0.0;
    const double E = (double)mg.elem, e = mg.fp32 ? E / 2 : E;
    const double n = (double)mg.lv[0].n;
    if (mg.lv.size() == 1) return 2.0 * n * E;
    const double fine = mg.fp32 ? 2.0 * E + 11.25 * e : 5.0 * E + 7.25 * e;
    return n * fine + n / 7.0 * 12.25 * e;
}

// CG on the projected Poisson system preconditioned by the V-cycle (flexible
// CG form, which equals preconditioned CG for this fixed SPD operator).
// The start (residual, first cycle, rho = r^T z) runs with host reads; the
// iterations are driven from the device: alpha, the convergence test and
// beta are one-thread kernels on a device state (PDev), every pass returns
// at once when the solve is over, and blocks of kPcgBlock iterations are
// captured once in a HIP graph (x is read from the state, so one graph
// serves every solution array) and replayed with one host read per block.
// Profiled runs of the classes launch the same kernels one by one.
namespace {

constexpr int kPcgBlock = 4;
enum { P_RUN = 0, P_OK = 1, P_NONFINITE = 2, P_BREAKDOWN = 3, P_MAXIT = 4 };

struct PDev {
    double *x;
    double rz, pAp, r2, tol2, a, b;
    int iters, maxit, done;
    int n_ap, n_step, n_dots;
};

struct EpiApD {          // Ap = -L p, <p, Ap> into the state
    double *__restrict__ Ap;
    PDev *D;
    double *partials;
    unsigned int *counter;
    double acc;
    __device__ bool skip() const { return D->done != P_RUN; }
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
            D->pAp = t[0];
            D->n_ap += 1;
        }
    }
};

__global__ void pcg_alpha(PDev *D) {
    if (D->done != P_RUN) return;
    const double pAp = D->pAp, rz = D->rz;
    if (!isfinite(pAp) || !isfinite(rz)) D->done = P_NONFINITE;
    else if (!(pAp > 0.0) || !(rz > 0.0)) D->done = P_BREAKDOWN;
    else D->a = rz / pAp;
}

struct FcgStepOpD {      // x += a p; r_old = r; r -= a Ap; {<r,r>}
    static constexpr int kClass = K_CG_UPDATE;
    static constexpr int kBytes = 0;     // counted from the passes that did work
    double *r, *r_old;
    const double *p, *Ap;
    PDev *D;
    double *x;
    double a;
    __device__ bool skip() const { return D->done != P_RUN; }
    __device__ void prepare() {
        x = D->x;
        a = D->a;
    }
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        x[i] = ::fma(a, p[i], x[i]);
        const double ro = r[i];
        r_old[i] = ro;
        const double rn = ::fma(-a, Ap[i], ro);
        r[i] = rn;
        acc[0] = ::fma(rn, rn, acc[0]);
    }
};
struct FinStepP {
    PDev *D;
    __device__ void operator()(const double (&t)[1]) const {
        const double r2 = t[0];
        D->r2 = r2;
        D->iters += 1;
        D->n_step += 1;
        if (!isfinite(r2)) D->done = P_NONFINITE;
        else if (r2 <= D->tol2) D->done = P_OK;
        else if (D->iters >= D->maxit) D->done = P_MAXIT;
    }
};

struct FcgDotsOpD {      // {<z, r - r_old>, <r, z>}: beta and the next rho
    static constexpr int kClass = K_CG_UPDATE;
    static constexpr int kBytes = 0;
    const double *z, *r, *r_old;
    PDev *D;
    __device__ bool skip() const { return D->done != P_RUN; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const double zi = z[i], ri = r[i];
        acc[0] = ::fma(zi, ri - r_old[i], acc[0]);
        acc[1] = ::fma(ri, zi, acc[1]);
    }
};
struct FinDotsP {
    PDev *D;
    __device__ void operator()(const double (&t)[2]) const {
        const double b = t[0] / D->rz;
        D->b = isfinite(b) ? b : 0.0;
        D->rz = t[1];
        D->n_dots += 1;
    }
};

struct DirOpD {          // p = z + b p
    static constexpr int kClass = K_CG_UPDATE;
    static constexpr int kBytes = 0;
    double *p;
    const double *z;
    PDev *D;
    double b;
    __device__ bool skip() const { return D->done != P_RUN; }
    __device__ void prepare() { b = D->b; }
    __device__ void operator()(int64_t i, double (&)[1]) const { p[i] = ::fma(b, p[i], z[i]); }
};

int pcg_iteration(ofdft_poisson *s, hipStream_t st) {
    const ofdft_grid &g = s->g;
    const int64_t n = npoints(g);
    PDev *D = (PDev *)s->pdev;
    double *r = s->r, *p = s->pA, *r_old = s->pB, *Ap = s->Ap, *z = s->z;
    {
        ProfScope ps(K_CG_STENCIL, 0.0, st);
        OFDFT_TRY(launch_stencil<double>(g, s->coef, LoadPlain<double>{p},
                                         EpiApD{Ap, D, s->rb.partials, s->rb.counter, 0.0}, st));
    }
    hipLaunchKernelGGL(pcg_alpha, dim3(1), dim3(1), 0, st, D);
    OFDFT_CHECK_HIP(hipGetLastError());
    OFDFT_TRY((launch_reduce<1>(n, FcgStepOpD{r, r_old, p, Ap, D, nullptr, 0.0}, FinStepP{D}, s->rb, st)));
    OFDFT_TRY(mg_apply_run(*s->mg, r, z, st, 0.0, &D->done));
    OFDFT_TRY((launch_reduce<2>(n, FcgDotsOpD{z, r, r_old, D}, FinDotsP{D}, s->rb, st)));
    OFDFT_TRY((launch_reduce<1>(n, DirOpD{p, z, D, 0.0}, NoFin{}, s->rb, st)));
    return OFDFT_OK;
}

int pcg_graph(ofdft_poisson *s) {
    if (s->mggraph) return OFDFT_OK;
    if (!s->mgcap) OFDFT_CHECK_HIP(hipStreamCreateWithFlags(&s->mgcap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    OFDFT_CHECK_HIP(hipStreamBeginCapture(s->mgcap, hipStreamCaptureModeThreadLocal));
    prof_suspend(true);
    int rc = OFDFT_OK;
    for (int k = 0; k < kPcgBlock && rc == OFDFT_OK; ++k) rc = pcg_iteration(s, s->mgcap);
    prof_suspend(false);
    const hipError_t e = hipStreamEndCapture(s->mgcap, &graph);
    if (rc != OFDFT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    OFDFT_CHECK_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&s->mggraph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    OFDFT_CHECK_HIP(ei);
    return OFDFT_OK;
}

}  // namespace

int poisson_solve_mg(ofdft_poisson *s, double *x, double rel_tol, int max_iter, ofdft_solve_stats &stats,
                     hipStream_t st) {
    const ofdft_grid &g = s->g;
    const int64_t n = npoints(g);
    double *r = s->r, *p = s->pA, *z = s->z;
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
    const double r2 = th[1];
    stats.iters = 0;
    if (!std::isfinite(r2)) return OFDFT_NONFINITE;
    if (r2 <= tol2) return OFDFT_OK;
    if (max_iter <= 0) return OFDFT_NOT_CONVERGED;
    OFDFT_TRY(mg_apply(*s->mg, r, z, st));
    OFDFT_TRY((launch_reduce<2>(n, FcgDotsOp{z, r, r}, StoreTotals<2>{tot}, s->rb, st)));
    OFDFT_TRY(sync_tot(2));
    OFDFT_TRY((launch_reduce<1>(n, CopyOp2{p, z}, NoFin{}, s->rb, st)));
    if (!s->pdev) {
        OFDFT_CHECK_HIP(hipMalloc(&s->pdev, sizeof(PDev)));
        OFDFT_CHECK_HIP(hipHostMalloc(&s->pdev_h, sizeof(PDev), hipHostMallocDefault));
    }
    PDev *Dh = (PDev *)s->pdev_h;
    *Dh = PDev{};
    Dh->x = x;
    Dh->rz = th[1];
    Dh->tol2 = tol2;
    Dh->maxit = max_iter;
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->pdev, Dh, sizeof(PDev), hipMemcpyHostToDevice, st));
    auto read_state = [&]() -> int {
        OFDFT_CHECK_HIP(hipMemcpyAsync(Dh, s->pdev, sizeof(PDev), hipMemcpyDeviceToHost, st));
        OFDFT_CHECK_HIP(hipStreamSynchronize(st));
        return OFDFT_OK;
    };
    const bool eager = !s->use_graphs || prof_timed(K_CG_STENCIL) || prof_timed(K_CG_UPDATE) ||
                       prof_timed(K_MULTIGRID);
    if (eager) {
        for (int k = 0; k <= max_iter; ++k) {
            OFDFT_TRY(pcg_iteration(s, st));
            OFDFT_TRY(read_state());
            if (Dh->done != P_RUN) break;
        }
    } else {
        OFDFT_TRY(pcg_graph(s));
        for (int k = 0; k <= max_iter; k += kPcgBlock) {
            OFDFT_CHECK_HIP(hipGraphLaunch(s->mggraph, st));
            OFDFT_TRY(read_state());
            if (Dh->done != P_RUN) break;
        }
    }
    const double nd = (double)n;
    prof_add(K_CG_STENCIL, nd * 16.0 * Dh->n_ap, eager ? 0 : Dh->n_ap);
    prof_add(K_CG_UPDATE, nd * (56.0 * Dh->n_step + 48.0 * Dh->n_dots), eager ? 0 : Dh->n_step + 2 * Dh->n_dots);
    prof_add(K_MULTIGRID, mg_cycle_bytes(*s->mg) * Dh->n_dots, eager ? 0 : Dh->n_dots);
    stats.iters = Dh->iters;
    switch (Dh->done) {
        case P_OK: return OFDFT_OK;
        case P_NONFINITE: return OFDFT_NONFINITE;
        case P_BREAKDOWN: return OFDFT_BREAKDOWN;
        default: return OFDFT_NOT_CONVERGED;
    }
}

}  // namespace ofdft

using namespace ofdft;

// z = M r for a multigrid solver (for inspection and for callers that build
// their own Krylov loop around the preconditioner).
extern "C" int ofdft_poisson_apply_preconditioner(ofdft_poisson *s, const double *r, double *z,
                                                  void *stream) {
    if (!s || !r || !z || r == z || !s->mg) {
        set_error("ofdft_poisson_apply_preconditioner: multigrid solver and distinct r, z required");
        return OFDFT_INVALID_ARG;
    }
    return mg_apply(*s->mg, r, z, (hipStream_t)stream);
}
