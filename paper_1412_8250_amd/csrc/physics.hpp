// Pointwise functionals of the density (Sections 2 and 3.3):
//  Thomas-Fermi  V_TF = (5/3) C_F rho^{2/3},  C_F = (3/10)(3 pi^2)^{2/3}
//  LDA exchange  V_x = -(3/pi)^{1/3} rho^{1/3}
//  Perdew-Zunger correlation, r_s = (3/(4 pi rho))^{1/3}:
//    r_s >= 1: V_c = (g1 + 7/6 g1 b1 sqrt(r_s) + 4/3 g1 b2 r_s) / (1 + b1 sqrt(r_s) + b2 r_s)^2
//    r_s <  1: V_c = (A1 + 2/3 C1 r_s) ln r_s + (B1 - A1/3) + 1/3 (2 D1 - C1) r_s
//  constants g1 = -0.1423, b1 = 1.0529, b2 = 0.3334, A1 = 0.0311, B1 = -0.048,
//  C1 = 0.002, D1 = -0.0116.
#pragma once

#include <hip/hip_runtime.h>

namespace ofdft {

constexpr double kPi = 3.14159265358979323846;
constexpr double kCF = 2.8712340001881915;          // (3/10)(3 pi^2)^{2/3}
constexpr double kCx = 0.98474502184269641;         // (3/pi)^{1/3}
constexpr double kRsC = 0.62035049089940009;        // (3/(4 pi))^{1/3}
constexpr double kG1 = -0.1423, kB1 = 1.0529, kB2 = 0.3334;
constexpr double kA1 = 0.0311, kBB1 = -0.048, kC1 = 0.002, kD1 = -0.0116;

// V_TF + V_xc at density rho > 0.
__device__ inline double v_local(double rho) {
    const double c = cbrt(rho);                 // rho^{1/3}
    const double vtf = (5.0 / 3.0) * kCF * c * c;
    const double vx = -kCx * c;
    const double rs = kRsC / c;
    double vc;
    if (rs >= 1.0) {
        const double sq = sqrt(rs);
        const double den = 1.0 + kB1 * sq + kB2 * rs;
        vc = (kG1 + (7.0 / 6.0) * kG1 * kB1 * sq + (4.0 / 3.0) * kG1 * kB2 * rs) / (den * den);
    } else {
        const double lr = log(rs);
        vc = (kA1 + (2.0 / 3.0) * kC1 * rs) * lr + (kBB1 - kA1 / 3.0) + (2.0 * kD1 - kC1) * rs / 3.0;
    }
    return vtf + vx + vc;
}

}  // namespace ofdft
