// Plain FD Laplacian application, y = alpha L_h x + beta y, for one element
// type.  Each type is instantiated in a translation unit of its own
// (stencil_<type>.hip), so that the unrolled stencil kernels compile in
// parallel.
#pragma once

#include "stencil_launch.hpp"

namespace ofdft {

template <typename T>
int apply_t(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, const void *x, void *y, double alpha,
            double beta, hipStream_t s) {
    using S = typename VT<T>::S;
    LoadPlain<T> ld{(const T *)x};
    ProfScope ps(K_APPLY, (double)npoints(g) * sizeof(T) * (beta != 0.0 ? 3 : 2), s);
    if (beta != 0.0)
        return launch_stencil<T>(g, c, ld, EpiAxpby<T, true>{(T *)y, (S)alpha, (S)beta, {}}, s);
    return launch_stencil<T>(g, c, ld, EpiAxpby<T, false>{(T *)y, (S)alpha, (S)beta, {}}, s);
}

extern template int apply_t<double>(const ofdft_grid &, const Coef<double> &, const void *, void *, double,
                                    double, hipStream_t);
extern template int apply_t<float>(const ofdft_grid &, const Coef<float> &, const void *, void *, double,
                                   double, hipStream_t);
extern template int apply_t<double2>(const ofdft_grid &, const Coef<double> &, const void *, void *, double,
                                     double, hipStream_t);
extern template int apply_t<float2>(const ofdft_grid &, const Coef<float> &, const void *, void *, double,
                                    double, hipStream_t);

}  // namespace ofdft
