// Plain FD Laplacian application, y = alpha L_h x + beta y, for one element
// type.  Each type is instantiated in a translation unit of its own
// (stencil_<type>.hip), so that the unrolled stencil kernels compile in
// parallel.
#pragma once

#include <type_traits>

#include "stencil_launch.hpp"

namespace ofdft {

template <typename T>
int apply_t(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, const void *x, void *y, double alpha,
            double beta, hipStream_t s) {
    using S = typename VT<T>::S;
    LoadPlain<T> ld{(const T *)x};
    ProfScope ps(K_APPLY, (double)npoints(g) * sizeof(T) * (beta != 0.0 ? 3 : 2), s);
    // 64 x 32 tiles for the real types; with beta != 0 the FP64 form would
    // need more than 256 registers (the four y values per thread), so it
    // takes the 64 x 16 tile of the generic dispatch instead of spilling
    auto go = [&](const auto &ep) {
        using E = std::decay_t<decltype(ep)>;
        constexpr bool wide = std::is_same_v<T, float> ||
                              (std::is_same_v<T, double> && std::is_same_v<E, EpiAxpby<T, false>>);
        if constexpr (wide) {
            const StencilCfg cfg = pick_stencil_cfg(g, sizeof(T), FAMILY_APPLY);
            if (cfg.shape == SHAPE_64x8x4) return launch_stencil_shape<T, 64, 8, 4>(g, cfg.zlen, c, ld, ep, s);
        }
        return launch_stencil<T>(g, c, ld, ep, s, FAMILY_APPLY);
    };
    if (beta != 0.0) return go(EpiAxpby<T, true>{(T *)y, (S)alpha, (S)beta, {}});
    return go(EpiAxpby<T, false>{(T *)y, (S)alpha, (S)beta, {}});
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
