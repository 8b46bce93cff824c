// fd_laplacian_apply kernels for float elements.
#include "stencil_apply.hpp"

namespace ofdft {
template int apply_t<float>(const ofdft_grid &, const Coef<float> &, const void *, void *, double, double, hipStream_t);
}  // namespace ofdft
