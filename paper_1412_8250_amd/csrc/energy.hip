// Ground-state energy terms and forces on the nuclei (Section 3.3, the
// energy expression after the fixed point and the forces; Section 3.2, the
// local electrostatics; Appendix B, the overlap correction), evaluated from
// the SCF context's current u, phi and kernel solutions:
//   E = C_F h^3 sum rho^(5/3) - (lambda/2) h^3 <u, L_h u> + mu T_LR
//       + h^3 sum eps_xc(rho) rho + 1/2 h^3 sum (rho + b) phi
//       - 1/2 sum_J h^3 sum b_J V_J + E_c
// (the discrete von Weizsacker term is the one whose gradient is the
// density update's H u).  Pseudocharges: Gaussians of charge q and width
// sigma (the stand-in for the paper's pseudopotentials), V_J = q erf(r /
// (sqrt 2 sigma)) / r; the self term and the forces
//   f_J = sum_images h^3 sum grad b_J (phi - V_J) + f^c_J
// are sums over each atom's grid points within the cutoff (one workgroup per
// atom, unwrapped offsets so every image counts once).  With Gaussians the
// overlap correction has the closed form
//   E_c = 1/2 sum_{I != J, images} q^2 erfc(d_IJ / (2 sigma)) / d_IJ
// (point-charge repulsion minus the Gaussians' mutual repulsion; the
// reference charges of Appendix B are then point-like), evaluated on the
// host with a cell list, and f^c_J = -dE_c / dR_J.
//
// Paper forms (ofdft_scf_energy_paper_form / ofdft_scf_forces_paper_form):
// the von Weizsacker term (lambda/2) h^3 sum |grad_h u|^2 with the FD
// gradient of Section 4, and the overlap correction by the grid form of
// Appendix B: reference charges b~_J (Gaussians of width sigma_ref) gathered
// onto the grid with a cell list, V_c the zero-mean solution of
// -L_h V_c = 4 pi (b~ - b) (the context's Poisson solver) plus the constant
// that gives it the mean of sum_J (V~_J - V_J), -2 pi q M (sigma_ref^2 -
// sigma^2) / |Omega| (minus 2 pi / 3 times the second moment of b~_J - b_J
// per atom, the k = 0 limit of its potential),
//   E_c = 1/2 h^3 sum (b~ + b) V_c + 1/2 sum_J h^3 sum b_J V_J
//         - 1/2 sum_J h^3 sum b~_J V~_J,
//   f^c_J = 1/2 sum_images h^3 sum [grad b~_J (V_c - V~_J) + grad b_J (V_c + V_J)
//           + (grad V~_J - grad V_J)(b~ + b) + b_J grad V_J - b~_J grad V~_J].
#include <algorithm>
#include <cmath>
#include <vector>

#include "gradient.hpp"
#include "physics.hpp"
#include "scf.hpp"

namespace ofdft {

namespace {

// LDA exchange-correlation energy per particle (Perdew-Zunger correlation).
__device__ inline double eps_xc(double rho) {
    const double c = cbrt(rho);
    const double ex = -0.75 * kCx * c;
    const double rs = kRsC / c;
    double ec;
    if (rs >= 1.0) {
        ec = kG1 / (1.0 + kB1 * sqrt(rs) + kB2 * rs);
    } else {
        const double lr = log(rs);
        ec = kA1 * lr + kBB1 + kC1 * rs * lr + kD1 * rs;
    }
    return ex + ec;
}

// totals: {sum rho^(5/3), sum eps_xc rho, sum (rho + b) phi, sum u L u, kernel energy density}
struct EnergyOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 32;
    const double *u, *b, *phi, *Lu;
    int kind;                                   // 0: no kernel term; 1: K_00; 2: order 2
    const double2 *V0, *V2, *V4, *V6;           // K_00: beta r = 1, 3; alpha r = 1, 3
    double alpha, beta;
    const double *W[kLrMaxConv];
    double coef[kLrMaxTerms], pw[kLrMaxTerms];
    int conv[kLrMaxTerms];
    int nterms;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[5]) const {
        const double ui = u[i], rho = ui * ui;
        const double c = cbrt(rho);
        acc[0] += rho * c * c;
        acc[1] += rho > 0.0 ? eps_xc(rho) * rho : 0.0;
        acc[2] = ::fma(rho + b[i], phi[i], acc[2]);
        acc[3] = ::fma(ui, Lu[i], acc[3]);
        if (kind == 1 && rho > 0.0) {
            const double wb = 2.0 * (V0[i].x + V2[i].x), wa = 2.0 * (V4[i].x + V6[i].x);
            const double lr = log(rho);
            acc[4] += 0.5 * (exp(alpha * lr) * wb + exp(beta * lr) * wa);
        } else if (kind == 2 && rho > 0.0) {
            const double lr = log(rho);
            double t = 0.0;
            for (int k = 0; k < nterms; ++k) t = ::fma(coef[k] * exp(pw[k] * lr), W[conv[k]][i], t);
            acc[4] += t;
        }
    }
};

struct AtomArgs {
    const double *pos;          // 3 per atom
    int count;
    int nx, ny, nz;
    double hx, hy, hz;
    double q, sigma, cut;
    int bx, by, bz;             // box half-widths in points
};

__device__ inline double gauss_b(double r, double q, double s) {
    return q * pow(2.0 * kPi * s * s, -1.5) * exp(-r * r / (2.0 * s * s));
}
__device__ inline double gauss_v(double r, double q, double s) {
    return r < 1e-12 ? q * sqrt(2.0 / kPi) / s : q * erf(r / (sqrt(2.0) * s)) / r;
}
// dV/dr (0 at r = 0)
__device__ inline double gauss_dv(double r, double q, double s) {
    if (r < 1e-12) return 0.0;
    return q * (sqrt(2.0 / kPi) * exp(-r * r / (2.0 * s * s)) / (s * r) - erf(r / (sqrt(2.0) * s)) / (r * r));
}

// One workgroup per atom: out[4 J + {0, 1, 2, 3}] = {h^3 sum b V, f_x, f_y, f_z}
// (forces without the overlap correction).
constexpr int kAtomThreads = 256;

__global__ void __launch_bounds__(kAtomThreads) atom_sums(AtomArgs a, const double *__restrict__ phi,
                                                          double *__restrict__ out) {
    __shared__ double scratch[4 * (kAtomThreads / 64)];
    const int J = blockIdx.x;
    if (J >= a.count) return;
    const double X = a.pos[3 * J], Y = a.pos[3 * J + 1], Z = a.pos[3 * J + 2];
    const int ix0 = (int)floor(X / a.hx) - a.bx, iy0 = (int)floor(Y / a.hy) - a.by, iz0 = (int)floor(Z / a.hz) - a.bz;
    const int sx = 2 * a.bx + 2, sy = 2 * a.by + 2, sz = 2 * a.bz + 2;
    const int64_t total = (int64_t)sx * sy * sz;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t t = threadIdx.x; t < total; t += kAtomThreads) {
        const int ox = (int)(t % sx), oy = (int)((t / sx) % sy), oz = (int)(t / ((int64_t)sx * sy));
        const int ix = ix0 + ox, iy = iy0 + oy, iz = iz0 + oz;
        const double dx = ix * a.hx - X, dy = iy * a.hy - Y, dz = iz * a.hz - Z;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r > a.cut) continue;
        const int wx = ((ix % a.nx) + a.nx) % a.nx, wy = ((iy % a.ny) + a.ny) % a.ny, wz = ((iz % a.nz) + a.nz) % a.nz;
        const double p = phi[((int64_t)wz * a.ny + wy) * a.nx + wx];
        const double bv = gauss_b(r, a.q, a.sigma), vv = gauss_v(r, a.q, a.sigma);
        const double g = -bv / (a.sigma * a.sigma) * (p - vv);        // grad b = -b (x - R) / s^2
        acc[0] = ::fma(bv, vv, acc[0]);
        acc[1] = ::fma(g, dx, acc[1]);
        acc[2] = ::fma(g, dy, acc[2]);
        acc[3] = ::fma(g, dz, acc[3]);
    }
    block_sum<4>(acc, scratch);
    if (threadIdx.x == 0) {
        const double dv = a.hx * a.hy * a.hz;
        for (int k = 0; k < 4; ++k) out[4 * J + k] = dv * acc[k];
    }
}

// Appendix B forces: one workgroup per atom, out[3 J + k] = f^c_J (see the
// file header).  vc holds the zero-mean V_c; vc_shift is its constant.
__global__ void __launch_bounds__(kAtomThreads) appb_force_sums(AtomArgs a, double s_ref, const double *__restrict__ vc,
                                                                double vc_shift, const double *__restrict__ bt,
                                                                const double *__restrict__ b, double *__restrict__ out) {
    __shared__ double scratch[3 * (kAtomThreads / 64)];
    const int J = blockIdx.x;
    if (J >= a.count) return;
    const double X = a.pos[3 * J], Y = a.pos[3 * J + 1], Z = a.pos[3 * J + 2];
    const int ix0 = (int)floor(X / a.hx) - a.bx, iy0 = (int)floor(Y / a.hy) - a.by, iz0 = (int)floor(Z / a.hz) - a.bz;
    const int sx = 2 * a.bx + 2, sy = 2 * a.by + 2, sz = 2 * a.bz + 2;
    const int64_t total = (int64_t)sx * sy * sz;
    const double s = a.sigma, q = a.q;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t t = threadIdx.x; t < total; t += kAtomThreads) {
        const int ox = (int)(t % sx), oy = (int)((t / sx) % sy), oz = (int)(t / ((int64_t)sx * sy));
        const int ix = ix0 + ox, iy = iy0 + oy, iz = iz0 + oz;
        const double dx = ix * a.hx - X, dy = iy * a.hy - Y, dz = iz * a.hz - Z;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r > a.cut) continue;
        const int wx = ((ix % a.nx) + a.nx) % a.nx, wy = ((iy % a.ny) + a.ny) % a.ny, wz = ((iz % a.nz) + a.nz) % a.nz;
        const int64_t i = ((int64_t)wz * a.ny + wy) * a.nx + wx;
        const double v = vc[i] + vc_shift, tot = bt[i] + b[i];
        const double bj = gauss_b(r, q, s), vj = gauss_v(r, q, s);
        const double btj = gauss_b(r, q, s_ref), vtj = gauss_v(r, q, s_ref);
        // radial factors: grad b = -b d / s^2, grad V = V'(r) d / r
        const double inv_r = r < 1e-12 ? 0.0 : 1.0 / r;
        const double gv = gauss_dv(r, q, s) * inv_r, gvt = gauss_dv(r, q, s_ref) * inv_r;
        const double k = -btj / (s_ref * s_ref) * (v - vtj) - bj / (s * s) * (v + vj) + (gvt - gv) * tot +
                         bj * gv - btj * gvt;
        acc[0] = ::fma(k, dx, acc[0]);
        acc[1] = ::fma(k, dy, acc[1]);
        acc[2] = ::fma(k, dz, acc[2]);
    }
    block_sum<3>(acc, scratch);
    if (threadIdx.x == 0) {
        const double dv = a.hx * a.hy * a.hz;
        for (int c = 0; c < 3; ++c) out[3 * J + c] = 0.5 * dv * acc[c];
    }
}

// Reference charge b~ on the grid: each point sums the Gaussians of the atom
// images within the cutoff, found through a cell list of bins at least the
// cutoff wide (27 neighbour bins, wrapped with their image shift), or over
// every atom and image shift when a box side holds fewer than 3 bins.  Atom
// positions are taken inside the box; the sum order is fixed.
struct CellArgs {
    int nx, ny, nz;
    double hx, hy, hz;
    double L[3];
    int nb[3];
    int brute, ni[3];
    int count;
    const double *pos;          // wrapped into [0, L)
    const int *start, *ids;     // bin b holds ids[start[b] .. start[b + 1])
    double q, s, cut;
};

__global__ void __launch_bounds__(kVecThreads) ref_charge_kernel(CellArgs a, double *__restrict__ bt) {
    const int64_t n = (int64_t)a.nx * a.ny * a.nz;
    const int64_t stride = (int64_t)gridDim.x * kVecThreads;
    const double norm = a.q * pow(2.0 * kPi * a.s * a.s, -1.5), e2 = -1.0 / (2.0 * a.s * a.s);
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        const int ix = (int)(i % a.nx), iy = (int)((i / a.nx) % a.ny), iz = (int)(i / ((int64_t)a.nx * a.ny));
        const double x[3] = {ix * a.hx, iy * a.hy, iz * a.hz};
        double sum = 0.0;
        auto add = [&](int J, const double sh[3]) {
            double r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double d = x[k] - (a.pos[3 * J + k] + sh[k]);
                r2 = ::fma(d, d, r2);
            }
            if (r2 <= a.cut * a.cut) sum = ::fma(norm, exp(e2 * r2), sum);
        };
        if (a.brute) {
            for (int J = 0; J < a.count; ++J)
                for (int tz = -a.ni[2]; tz <= a.ni[2]; ++tz)
                    for (int ty = -a.ni[1]; ty <= a.ni[1]; ++ty)
                        for (int tx = -a.ni[0]; tx <= a.ni[0]; ++tx) {
                            const double sh[3] = {tx * a.L[0], ty * a.L[1], tz * a.L[2]};
                            add(J, sh);
                        }
        } else {
            int c[3];
            for (int k = 0; k < 3; ++k) c[k] = min(a.nb[k] - 1, (int)(x[k] / a.L[k] * a.nb[k]));
            for (int oz = -1; oz <= 1; ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int ox = -1; ox <= 1; ++ox) {
                        const int o[3] = {ox, oy, oz};
                        int bb[3];
                        double sh[3];
                        for (int k = 0; k < 3; ++k) {
                            bb[k] = c[k] + o[k];
                            sh[k] = 0.0;
                            if (bb[k] < 0) { bb[k] += a.nb[k]; sh[k] = -a.L[k]; }
                            else if (bb[k] >= a.nb[k]) { bb[k] -= a.nb[k]; sh[k] = a.L[k]; }
                        }
                        const int bin = (bb[2] * a.nb[1] + bb[1]) * a.nb[0] + bb[0];
                        for (int t = a.start[bin]; t < a.start[bin + 1]; ++t) add(a.ids[t], sh);
                    }
        }
        bt[i] = sum;
    }
}

struct AppbRhsOp {       // g = 4 pi (b~ - b)
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24;
    const double *bt, *b;
    double *g;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { g[i] = 4.0 * kPi * (bt[i] - b[i]); }
};

struct AppbSumOp {       // {sum (b~ + b) V_c0, sum (b~ + b)}
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24;
    const double *bt, *b, *vc;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[2]) const {
        const double t = bt[i] + b[i];
        acc[0] = ::fma(t, vc[i], acc[0]);
        acc[1] += t;
    }
};

struct ZeroOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 8;
    double *x;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&)[1]) const { x[i] = 0.0; }
};

// Overlap correction (energy and forces) with a cell list of bins at least rc
// wide (brute force over image shifts when the box holds fewer than 3 bins).
void overlap(const ofdft_gauss_atoms &at, const double L[3], double &e, std::vector<double> &f) {
    const int M = at.count;
    const double q = at.charge, s = at.sigma, rc = 12.0 * s;
    e = 0.0;
    f.assign(3 * (size_t)M, 0.0);
    auto pair = [&](int I, const double dvec[3]) {
        const double d = std::sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
        if (d == 0.0 || d > rc) return;
        e += 0.5 * q * q * std::erfc(d / (2.0 * s)) / d;
        const double g = q * q * (std::erfc(d / (2.0 * s)) / (d * d) + std::exp(-d * d / (4.0 * s * s)) / (s * std::sqrt(kPi) * d));
        for (int k = 0; k < 3; ++k) f[3 * (size_t)I + k] -= g * dvec[k] / d;
    };
    int nb[3];
    for (int k = 0; k < 3; ++k) nb[k] = std::max(1, (int)std::floor(L[k] / rc));
    if (nb[0] >= 3 && nb[1] >= 3 && nb[2] >= 3) {
        std::vector<std::vector<int>> bins((size_t)nb[0] * nb[1] * nb[2]);
        auto bin_of = [&](int J, int c[3]) {
            for (int k = 0; k < 3; ++k) {
                double x = std::fmod(at.pos[3 * J + k], L[k]);
                if (x < 0) x += L[k];
                c[k] = std::min(nb[k] - 1, (int)(x / L[k] * nb[k]));
            }
        };
        for (int J = 0; J < M; ++J) {
            int c[3];
            bin_of(J, c);
            bins[((size_t)c[2] * nb[1] + c[1]) * nb[0] + c[0]].push_back(J);
        }
        for (int I = 0; I < M; ++I) {
            int c[3];
            bin_of(I, c);
            for (int oz = -1; oz <= 1; ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int ox = -1; ox <= 1; ++ox) {
                        int b[3] = {c[0] + ox, c[1] + oy, c[2] + oz};
                        double sh[3];
                        for (int k = 0; k < 3; ++k) {
                            sh[k] = 0.0;
                            if (b[k] < 0) { b[k] += nb[k]; sh[k] = -L[k]; }
                            else if (b[k] >= nb[k]) { b[k] -= nb[k]; sh[k] = L[k]; }
                        }
                        for (int J : bins[((size_t)b[2] * nb[1] + b[1]) * nb[0] + b[0]]) {
                            double dvec[3];
                            for (int k = 0; k < 3; ++k) {
                                // positions taken inside the box, plus the bin wrap's image shift
                                double xj = std::fmod(at.pos[3 * J + k], L[k]), xi = std::fmod(at.pos[3 * I + k], L[k]);
                                if (xj < 0) xj += L[k];
                                if (xi < 0) xi += L[k];
                                dvec[k] = xj + sh[k] - xi;
                            }
                            pair(I, dvec);
                        }
                    }
        }
    } else {
        int ni[3];
        for (int k = 0; k < 3; ++k) ni[k] = (int)std::ceil(rc / L[k]);
        for (int I = 0; I < M; ++I)
            for (int J = 0; J < M; ++J)
                for (int a = -ni[0]; a <= ni[0]; ++a)
                    for (int b = -ni[1]; b <= ni[1]; ++b)
                        for (int c = -ni[2]; c <= ni[2]; ++c) {
                            const double dvec[3] = {at.pos[3 * J] + a * L[0] - at.pos[3 * I],
                                                    at.pos[3 * J + 1] + b * L[1] - at.pos[3 * I + 1],
                                                    at.pos[3 * J + 2] + c * L[2] - at.pos[3 * I + 2]};
                            pair(I, dvec);
                        }
    }
}

int check_atoms(const ofdft_scf *s, const ofdft_gauss_atoms *at) {
    if (!s || !at || at->count < 1 || !at->pos || !(at->sigma > 0) || !(at->cutoff > 0)) {
        set_error("ofdft_scf_energy/forces: bad context or atoms");
        return OFDFT_INVALID_ARG;
    }
    return OFDFT_OK;
}

// Per-atom sums on the device: out has 4 doubles per atom (host).
int atom_pass(ofdft_scf *s, const ofdft_gauss_atoms &at, std::vector<double> &out, hipStream_t st) {
    const int M = at.count;
    double *d_pos = nullptr, *d_out = nullptr;
    if (hipMalloc(&d_pos, sizeof(double) * 3 * M) != hipSuccess ||
        hipMalloc(&d_out, sizeof(double) * 4 * M) != hipSuccess) {
        if (d_pos) (void)hipFree(d_pos);
        set_error("ofdft_scf_energy/forces: out of device memory");
        return OFDFT_NO_MEMORY;
    }
    AtomArgs a{};
    a.pos = d_pos;
    a.count = M;
    a.nx = s->g.nx;
    a.ny = s->g.ny;
    a.nz = s->g.nz;
    a.hx = s->g.hx;
    a.hy = s->g.hy;
    a.hz = s->g.hz;
    a.q = at.charge;
    a.sigma = at.sigma;
    a.cut = at.cutoff;
    a.bx = (int)std::ceil(at.cutoff / a.hx) + 1;
    a.by = (int)std::ceil(at.cutoff / a.hy) + 1;
    a.bz = (int)std::ceil(at.cutoff / a.hz) + 1;
    out.assign(4 * (size_t)M, 0.0);
    hipError_t e = hipMemcpyAsync(d_pos, at.pos, sizeof(double) * 3 * M, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        ProfScope ps(K_POINTWISE, (double)M * (8.0 * (2 * a.bx + 2) * (2 * a.by + 2) * (2 * a.bz + 2)), st);
        hipLaunchKernelGGL(atom_sums, dim3(M), dim3(kAtomThreads), 0, st, a, s->phi, d_out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out.data(), d_out, sizeof(double) * 4 * M, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_pos);
    (void)hipFree(d_out);
    if (e != hipSuccess) {
        set_error("ofdft_scf_energy/forces: %s", hipGetErrorString(e));
        return OFDFT_HIP_ERROR;
    }
    return OFDFT_OK;
}

// b~ on the grid (device array bt) for Gaussians of width s_ref (the
// atoms' charge and cutoff).
int ref_charge(ofdft_scf *s, const ofdft_gauss_atoms &at, double s_ref, double *bt, hipStream_t st) {
    const int M = at.count;
    CellArgs a{};
    a.nx = s->g.nx;
    a.ny = s->g.ny;
    a.nz = s->g.nz;
    a.hx = s->g.hx;
    a.hy = s->g.hy;
    a.hz = s->g.hz;
    a.L[0] = s->g.nx * s->g.hx;
    a.L[1] = s->g.ny * s->g.hy;
    a.L[2] = s->g.nz * s->g.hz;
    a.count = M;
    a.q = at.charge;
    a.s = s_ref;
    a.cut = at.cutoff;
    std::vector<double> pos(3 * (size_t)M);
    for (int J = 0; J < M; ++J)
        for (int k = 0; k < 3; ++k) {
            double x = std::fmod(at.pos[3 * J + k], a.L[k]);
            if (x < 0) x += a.L[k];
            if (x >= a.L[k]) x -= a.L[k];
            pos[3 * (size_t)J + k] = x;
        }
    for (int k = 0; k < 3; ++k) a.nb[k] = std::max(1, (int)std::floor(a.L[k] / a.cut));
    a.brute = a.nb[0] < 3 || a.nb[1] < 3 || a.nb[2] < 3;
    std::vector<int> start(1, 0), ids;
    if (a.brute) {
        for (int k = 0; k < 3; ++k) a.ni[k] = (int)std::ceil(a.cut / a.L[k]) + 1;
    } else {
        const int nbins = a.nb[0] * a.nb[1] * a.nb[2];
        std::vector<int> bin(M), cnt(nbins + 1, 0);
        for (int J = 0; J < M; ++J) {
            int c[3];
            for (int k = 0; k < 3; ++k) c[k] = std::min(a.nb[k] - 1, (int)(pos[3 * (size_t)J + k] / a.L[k] * a.nb[k]));
            bin[J] = (c[2] * a.nb[1] + c[1]) * a.nb[0] + c[0];
            ++cnt[bin[J] + 1];
        }
        for (int b = 0; b < nbins; ++b) cnt[b + 1] += cnt[b];
        start = cnt;
        ids.assign(M, 0);
        std::vector<int> fill(cnt.begin(), cnt.end() - 1);
        for (int J = 0; J < M; ++J) ids[fill[bin[J]]++] = J;   // atom order kept within a bin
    }
    double *d_pos = nullptr;
    int *d_start = nullptr, *d_ids = nullptr;
    hipError_t e = hipMalloc(&d_pos, sizeof(double) * pos.size());
    if (e == hipSuccess) e = hipMalloc(&d_start, sizeof(int) * start.size());
    if (e == hipSuccess) e = hipMalloc(&d_ids, sizeof(int) * std::max<size_t>(ids.size(), 1));
    if (e == hipSuccess) e = hipMemcpyAsync(d_pos, pos.data(), sizeof(double) * pos.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !ids.empty())
        e = hipMemcpyAsync(d_ids, ids.data(), sizeof(int) * ids.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        a.pos = d_pos;
        a.start = d_start;
        a.ids = d_ids;
        const int64_t n = s->n;
        ProfScope ps(K_POINTWISE, (double)n * 8.0, st);
        hipLaunchKernelGGL(ref_charge_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, st, a, bt);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (d_pos) (void)hipFree(d_pos);
    if (d_start) (void)hipFree(d_start);
    if (d_ids) (void)hipFree(d_ids);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("ofdft_scf_*_paper_form: reference charge: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? OFDFT_NO_MEMORY : OFDFT_HIP_ERROR;
    }
    return OFDFT_OK;
}

// Appendix B grid form: E_c, and f^c (3 per atom) when fc is given.  Uses
// the density-update workspace rA (b~), rB (right-hand side), dA (V_c).
// Returns the Poisson solve's status (NOT_CONVERGED if it missed its
// tolerance; the results are still written).
int appendix_b(ofdft_scf *s, const ofdft_gauss_atoms &at, double s_ref, double &ec, std::vector<double> *fc,
               hipStream_t st) {
    const int64_t n = s->n;
    double *bt = s->rA, *g = s->rB, *vc = s->dA;
    OFDFT_TRY(ref_charge(s, at, s_ref, bt, st));
    OFDFT_TRY((launch_reduce<1>(n, AppbRhsOp{bt, s->b, g}, NoFin{}, s->rb, st)));
    OFDFT_TRY((launch_reduce<1>(n, ZeroOp{vc}, NoFin{}, s->rb, st)));
    ofdft_solve_stats ps{};
    const int pst = poisson_solve(s->pois, g, vc, s->p.poisson_tol, s->p.max_iter, ps, st);
    if (pst < 0) return pst;
    const double volume = s->dv * (double)n;
    const double shift = -2.0 * kPi * at.charge * at.count * (s_ref * s_ref - at.sigma * at.sigma) / volume;
    OFDFT_TRY((launch_reduce<2>(n, AppbSumOp{bt, s->b, vc}, StoreTotals<2>{s->dsc + 56}, s->rb, st)));
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->hsc + 56, s->dsc + 56, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    ec = 0.5 * s->dv * (s->hsc[56] + shift * s->hsc[57]);
    std::vector<double> per, per_ref;
    OFDFT_TRY(atom_pass(s, at, per, st));
    ofdft_gauss_atoms ref = at;
    ref.sigma = s_ref;
    OFDFT_TRY(atom_pass(s, ref, per_ref, st));
    for (int J = 0; J < at.count; ++J) ec += 0.5 * (per[4 * (size_t)J] - per_ref[4 * (size_t)J]);
    if (fc) {
        const int M = at.count;
        double *d_pos = nullptr, *d_out = nullptr;
        hipError_t e = hipMalloc(&d_pos, sizeof(double) * 3 * M);
        if (e == hipSuccess) e = hipMalloc(&d_out, sizeof(double) * 3 * M);
        AtomArgs a{};
        a.pos = d_pos;
        a.count = M;
        a.nx = s->g.nx;
        a.ny = s->g.ny;
        a.nz = s->g.nz;
        a.hx = s->g.hx;
        a.hy = s->g.hy;
        a.hz = s->g.hz;
        a.q = at.charge;
        a.sigma = at.sigma;
        a.cut = at.cutoff;
        a.bx = (int)std::ceil(at.cutoff / a.hx) + 1;
        a.by = (int)std::ceil(at.cutoff / a.hy) + 1;
        a.bz = (int)std::ceil(at.cutoff / a.hz) + 1;
        fc->assign(3 * (size_t)M, 0.0);
        if (e == hipSuccess) e = hipMemcpyAsync(d_pos, at.pos, sizeof(double) * 3 * M, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(appb_force_sums, dim3(M), dim3(kAtomThreads), 0, st, a, s_ref, vc, shift, bt, s->b,
                               d_out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(fc->data(), d_out, sizeof(double) * 3 * M, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (d_pos) (void)hipFree(d_pos);
        if (d_out) (void)hipFree(d_out);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("ofdft_scf_forces_paper_form: %s", hipGetErrorString(e));
            return OFDFT_HIP_ERROR;
        }
    }
    return pst;
}

int check_ref(const ofdft_gauss_atoms *at, double s_ref) {
    if (!(s_ref > 0) || !std::isfinite(s_ref)) {
        set_error("ofdft_scf_*_paper_form: sigma_ref must be positive");
        return OFDFT_INVALID_ARG;
    }
    (void)at;
    return OFDFT_OK;
}

// The energy terms of ofdft_scf_energy (see the header for the order).
int energy_terms(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double *terms, hipStream_t st);

}  // namespace

}  // namespace ofdft

using namespace ofdft;

namespace ofdft {
namespace {

int energy_terms(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double *terms, hipStream_t st) {
    const int64_t n = s->n;
    // L u into the H u workspace (free outside the density update)
    OFDFT_TRY(fd_laplacian_apply(&s->g, s->p.radius, OFDFT_F64, s->u, s->Hu, 1.0, 0.0, st));
    EnergyOp op{};
    op.u = s->u;
    op.b = s->b;
    op.phi = s->phi;
    op.Lu = s->Hu;
    op.kind = !s->p.mu ? 0 : (s->p.lr_order == 2 ? 2 : 1);
    op.alpha = 5.0 / 6.0 + 0.37267799624996495;
    op.beta = 5.0 / 6.0 - 0.37267799624996495;
    if (op.kind == 1) {
        op.V0 = s->Vr[0];
        op.V2 = s->Vr[2];
        op.V4 = s->Vr[4];
        op.V6 = s->Vr[6];
    } else if (op.kind == 2) {
        for (size_t c = 0; c < s->lr_W.size(); ++c) op.W[c] = s->lr_W[c];
        op.nterms = (int)s->lr_eterms.size();
        for (int k = 0; k < op.nterms; ++k) {
            op.coef[k] = s->lr_eterms[k].coef;
            op.pw[k] = s->lr_eterms[k].e;
            op.conv[k] = s->lr_eterms[k].conv;
        }
    }
    OFDFT_TRY((launch_reduce<5>(n, op, StoreTotals<5>{s->dsc + 48}, s->rb, st)));
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->hsc + 48, s->dsc + 48, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    const double dv = s->dv, *t = s->hsc + 48;
    std::vector<double> per;
    OFDFT_TRY(atom_pass(s, *atoms, per, st));
    double self = 0.0;
    for (int J = 0; J < atoms->count; ++J) self -= 0.5 * per[4 * (size_t)J];
    const double L[3] = {s->g.nx * s->g.hx, s->g.ny * s->g.hy, s->g.nz * s->g.hz};
    double ec;
    std::vector<double> fc;
    overlap(*atoms, L, ec, fc);
    terms[0] = dv * kCF * t[0];
    terms[1] = -0.5 * s->p.lambda * dv * t[3];
    terms[2] = dv * t[1];
    terms[3] = 0.5 * dv * t[2];
    terms[4] = self;
    terms[5] = ec;
    terms[6] = s->p.mu ? dv * (op.kind == 1 ? kCF * t[4] : t[4]) : 0.0;
    terms[7] = terms[0] + terms[1] + terms[2] + terms[3] + terms[4] + terms[5] + terms[6];
    return OFDFT_OK;
}

}  // namespace
}  // namespace ofdft

extern "C" int ofdft_scf_energy(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double *terms, void *stream) {
    OFDFT_TRY(check_atoms(s, atoms));
    if (!terms) return OFDFT_INVALID_ARG;
    return energy_terms(s, atoms, terms, (hipStream_t)stream);
}

extern "C" int ofdft_scf_energy_paper_form(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double sigma_ref,
                                           double *terms, void *stream) {
    OFDFT_TRY(check_atoms(s, atoms));
    OFDFT_TRY(check_ref(atoms, sigma_ref));
    if (!terms) return OFDFT_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    OFDFT_TRY(energy_terms(s, atoms, terms, st));
    OFDFT_TRY(grad_sq_sum(s->g, s->p.radius, s->u, s->dsc + 58, s->rb, st));
    OFDFT_CHECK_HIP(hipMemcpyAsync(s->hsc + 58, s->dsc + 58, sizeof(double), hipMemcpyDeviceToHost, st));
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    terms[1] = 0.5 * s->p.lambda * s->dv * s->hsc[58];
    double ec = 0.0;
    const int pst = appendix_b(s, *atoms, sigma_ref, ec, nullptr, st);
    if (pst < 0) return pst;
    terms[5] = ec;
    terms[7] = terms[0] + terms[1] + terms[2] + terms[3] + terms[4] + terms[5] + terms[6];
    return pst;
}

extern "C" int ofdft_scf_forces_paper_form(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double sigma_ref,
                                           double *forces, void *stream) {
    OFDFT_TRY(check_atoms(s, atoms));
    OFDFT_TRY(check_ref(atoms, sigma_ref));
    if (!forces) return OFDFT_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> per, fc;
    OFDFT_TRY(atom_pass(s, *atoms, per, st));
    double ec = 0.0;
    const int pst = appendix_b(s, *atoms, sigma_ref, ec, &fc, st);
    if (pst < 0) return pst;
    for (int J = 0; J < atoms->count; ++J)
        for (int k = 0; k < 3; ++k) forces[3 * J + k] = per[4 * (size_t)J + 1 + k] + fc[3 * (size_t)J + k];
    return pst;
}

extern "C" int ofdft_scf_forces(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double *forces, void *stream) {
    OFDFT_TRY(check_atoms(s, atoms));
    if (!forces) return OFDFT_INVALID_ARG;
    std::vector<double> per;
    OFDFT_TRY(atom_pass(s, *atoms, per, (hipStream_t)stream));
    const double L[3] = {s->g.nx * s->g.hx, s->g.ny * s->g.hy, s->g.nz * s->g.hz};
    double ec;
    std::vector<double> fc;
    overlap(*atoms, L, ec, fc);
    for (int J = 0; J < atoms->count; ++J)
        for (int k = 0; k < 3; ++k) forces[3 * J + k] = per[4 * (size_t)J + 1 + k] + fc[3 * (size_t)J + k];
    return OFDFT_OK;
}
