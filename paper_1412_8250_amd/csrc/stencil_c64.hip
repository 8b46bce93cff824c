// fd_laplacian_apply kernels for float2 elements.
#include "stencil_apply.hpp"

namespace ofdft {
template int apply_t<float2>(const ofdft_grid &, const Coef<float> &, const void *, void *, double, double, hipStream_t);
}  // namespace ofdft
