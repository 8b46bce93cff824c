// fd_laplacian_apply kernels for double2 elements.
#include "stencil_apply.hpp"

namespace ofdft {
template int apply_t<double2>(const ofdft_grid &, const Coef<double> &, const void *, void *, double, double, hipStream_t);
}  // namespace ofdft
