// fd_laplacian_apply: y = alpha L_h x + beta y for f64 / f32 / c128 / c64 (the
// kernels of each type are built in stencil_<type>.hip).
#include "stencil_apply.hpp"

using namespace ofdft;

extern "C" int fd_laplacian_apply(const ofdft_grid *grid, int radius, ofdft_dtype dtype,
                                  const void *x, void *y, double alpha, double beta, void *stream) {
    OFDFT_TRY(check_grid(grid, radius));
    if (!x || !y) {
        set_error("fd_laplacian_apply: NULL array pointer");
        return OFDFT_INVALID_ARG;
    }
    if (x == y) {
        set_error("fd_laplacian_apply: x and y must not overlap");
        return OFDFT_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const Coef<double> c = make_coef(*grid, radius);
    switch (dtype) {
        case OFDFT_F64: return apply_t<double>(*grid, c, x, y, alpha, beta, s);
        case OFDFT_F32: return apply_t<float>(*grid, to_float(c), x, y, alpha, beta, s);
        case OFDFT_C128: return apply_t<double2>(*grid, c, x, y, alpha, beta, s);
        case OFDFT_C64: return apply_t<float2>(*grid, to_float(c), x, y, alpha, beta, s);
        default:
            set_error("fd_laplacian_apply: unknown dtype %d", (int)dtype);
            return OFDFT_INVALID_ARG;
    }
}
