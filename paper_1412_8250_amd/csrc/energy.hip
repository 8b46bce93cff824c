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
#include <algorithm>
#include <cmath>
#include <vector>

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

}  // namespace

}  // namespace ofdft

using namespace ofdft;

extern "C" int ofdft_scf_energy(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double *terms, void *stream) {
    OFDFT_TRY(check_atoms(s, atoms));
    if (!terms) return OFDFT_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
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
