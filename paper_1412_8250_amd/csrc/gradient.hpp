// The FD gradient of Section 4 (FD gradient equation): component a at
// (i,j,k) is sum_{p=1..N} w~_p / h_a (f(+p along a) - f(-p along a)) with
// w~_p = (-1)^{p+1} (N!)^2 / (p (N-p)! (N+p)!), indices wrapped periodically.
#pragma once

#include "vec.hpp"

namespace ofdft {

struct GradCoef {
    int nx, ny, nz, N;
    double wx[kMaxRadius + 1], wy[kMaxRadius + 1], wz[kMaxRadius + 1];
};

GradCoef make_grad_coef(const ofdft_grid &g, int radius);

// Periodic wrap of i + d for |d| <= N (repeated for grids shorter than N).
__device__ inline int grad_wrap(int i, int n) {
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

// The three components at flat index i of an [nz][ny][nx] array.
__device__ inline void grad_at(const double *__restrict__ x, int64_t i, const GradCoef &c, double &gx,
                               double &gy, double &gz) {
    const int64_t nxy = (int64_t)c.nx * c.ny;
    const int iz = (int)(i / nxy);
    const int rem = (int)(i - (int64_t)iz * nxy);
    const int iy = rem / c.nx, ix = rem - iy * c.nx;
    const double *row = x + (int64_t)iz * nxy + (int64_t)iy * c.nx;
    const double *col = x + (int64_t)iz * nxy + ix;
    const double *pil = x + (int64_t)iy * c.nx + ix;
    gx = gy = gz = 0.0;
#pragma unroll
    for (int p = 1; p <= kMaxRadius; ++p) {
        if (p > c.N) break;
        gx = ::fma(c.wx[p], row[grad_wrap(ix + p, c.nx)] - row[grad_wrap(ix - p, c.nx)], gx);
        gy = ::fma(c.wy[p], col[(int64_t)grad_wrap(iy + p, c.ny) * c.nx] - col[(int64_t)grad_wrap(iy - p, c.ny) * c.nx],
                   gy);
        gz = ::fma(c.wz[p], pil[(int64_t)grad_wrap(iz + p, c.nz) * nxy] - pil[(int64_t)grad_wrap(iz - p, c.nz) * nxy],
                   gz);
    }
}

// sum |grad_h u|^2 over the grid (deterministic reduction) into dst[0] (device).
int grad_sq_sum(const ofdft_grid &g, int radius, const double *u, double *dst, const RedBuf &rb, hipStream_t s);

}  // namespace ofdft
