// One launcher for every single-pass stencil kernel: picks the tile shape,
// sizes the z chunks from the kernel's measured residency, launches.
#pragma once

#include <atomic>

#include "stencil_core.hpp"
#include "tuning.hpp"

namespace ofdft {

// Workgroups of `kern` resident on the current device at once (cached per
// kernel instantiation and device by the caller's static slot).
template <class Kern>
inline int resident_blocks(Kern kern, int threads, std::atomic<int> (&cache)[kMaxDevices]) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        per_cu <= 0 || cus <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    v = per_cu * cus;
    cache[dev].store(v, std::memory_order_relaxed);
    return v;
}

template <typename T, int TX, int TYT, int RY, class Load, class Epi>
inline int launch_stencil_shape(const ofdft_grid &g, int zlen, const Coef<typename VT<T>::S> &c,
                                const Load &ld, const Epi &ep, hipStream_t s) {
    static std::atomic<int> cache[kMaxDevices];
    auto kern = stencil_kernel<T, TX, TYT, RY, Load, Epi>;
    if (zlen <= 0) zlen = zlen_auto(g, TX, TYT * RY, resident_blocks(kern, TX * TYT, cache));
    const TileGeom tg = make_tile_geom<TX, TYT, RY>(g, zlen);
    hipLaunchKernelGGL(kern, dim3(tg.nblocks), dim3(TX, TYT), 0, s, tg, c, ld, ep);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

template <typename T, class Load, class Epi>
inline int launch_stencil(const ofdft_grid &g, const Coef<typename VT<T>::S> &c, const Load &ld,
                          const Epi &ep, hipStream_t s, int family = FAMILY_PASS) {
    const StencilCfg cfg = pick_stencil_cfg(g, sizeof(T), family);
    return dispatch_shape(cfg.shape, [&](auto sh) {
        using S = decltype(sh);
        return launch_stencil_shape<T, S::TX, S::TYT, S::RY>(g, cfg.zlen, c, ld, ep, s);
    });
}

}  // namespace ofdft
