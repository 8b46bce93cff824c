// fd_gradient_apply and the gradient-form sums of the energy (Section 4, FD
// gradient equation).  Not on the solvers' path: one thread per point reads
// its 6N neighbours, which the L2 serves for the x rows and neighbouring
// waves.
#include "gradient.hpp"

namespace ofdft {

GradCoef make_grad_coef(const ofdft_grid &g, int radius) {
    GradCoef c{};
    c.nx = g.nx;
    c.ny = g.ny;
    c.nz = g.nz;
    c.N = radius;
    for (int p = 1; p <= radius; ++p) {
        // (N!)^2 / ((N-p)! (N+p)!) = prod_{k<p} (N - k) / prod_{k=1..p} (N + k)
        double r = 1.0;
        for (int k = 0; k < p; ++k) r *= (double)(radius - k) / (double)(radius + k + 1);
        const double w = (p % 2 ? 1.0 : -1.0) * r / p;
        c.wx[p] = w / g.hx;
        c.wy[p] = w / g.hy;
        c.wz[p] = w / g.hz;
    }
    return c;
}

namespace {

__global__ void __launch_bounds__(kVecThreads)
grad_kernel(GradCoef c, const double *__restrict__ x, double *__restrict__ gx, double *__restrict__ gy,
            double *__restrict__ gz) {
    const int64_t n = (int64_t)c.nx * c.ny * c.nz;
    const int64_t stride = (int64_t)gridDim.x * kVecThreads;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        double a, b, d;
        grad_at(x, i, c, a, b, d);
        gx[i] = a;
        gy[i] = b;
        gz[i] = d;
    }
}

struct GradSqOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 8;
    GradCoef c;
    const double *u;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        double a, b, d;
        grad_at(u, i, c, a, b, d);
        acc[0] = ::fma(a, a, ::fma(b, b, ::fma(d, d, acc[0])));
    }
};

}  // namespace

int grad_sq_sum(const ofdft_grid &g, int radius, const double *u, double *dst, const RedBuf &rb, hipStream_t s) {
    return launch_reduce<1>(npoints(g), GradSqOp{make_grad_coef(g, radius), u}, StoreTotals<1>{dst}, rb, s);
}

}  // namespace ofdft

using namespace ofdft;

extern "C" int fd_gradient_apply(const ofdft_grid *grid, int radius, const double *x, double *gx, double *gy,
                                 double *gz, void *stream) {
    OFDFT_TRY(check_grid(grid, radius));
    if (!x || !gx || !gy || !gz) {
        set_error("fd_gradient_apply: NULL array pointer");
        return OFDFT_INVALID_ARG;
    }
    if (x == gx || x == gy || x == gz || gx == gy || gx == gz || gy == gz) {
        set_error("fd_gradient_apply: x, gx, gy and gz must be four distinct arrays");
        return OFDFT_INVALID_ARG;
    }
    const int64_t n = npoints(*grid);
    hipStream_t s = (hipStream_t)stream;
    ProfScope ps(K_POINTWISE, (double)n * 32.0, s);
    hipLaunchKernelGGL(grad_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, make_grad_coef(*grid, radius), x,
                       gx, gy, gz);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}
