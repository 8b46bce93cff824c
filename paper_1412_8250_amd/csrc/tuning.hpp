// Launch-shape selection for the stencil kernels.  A table keyed by (grid
// size, element bytes, kernel family) is consulted first; its entries are
// written by the library's autotuner (ofdft_tune_stencil, which times every
// legal shape and z-chunk length of a family on the grid) or set by hand
// (ofdft_stencil_set_config, for every family at once); without an entry a
// fixed heuristic measured at 320^3 decides.
#pragma once

#include "common.hpp"

namespace ofdft {

// Tile shapes: TX x TYT threads, RY rows per thread, tile TX x (TYT * RY).
enum StencilShape {
    SHAPE_64x4x4 = 0,    // 64 x 16 tile, 256 threads
    SHAPE_64x4x2 = 1,    // 64 x 8 tile, 256 threads
    SHAPE_32x8x2 = 2,    // 32 x 16 tile, 256 threads
    SHAPE_64x8x2 = 3,    // 64 x 16 tile, 512 threads
    SHAPE_64x8x1 = 4,    // 64 x 8 tile, 512 threads
    SHAPE_64x8x4 = 5,    // 64 x 32 tile, 512 threads: the plain FP64 and FP32 applies only
                         // (fused kernels given this id run 64 x 8 x 2)
    SHAPE_COUNT = 6
};

template <int TX_, int TYT_, int RY_>
struct ShapeTag {
    static constexpr int TX = TX_, TYT = TYT_, RY = RY_;
};

// Calls f(ShapeTag<...>{}) for the shape id (unknown ids: 64x4x2).
template <class F>
inline int dispatch_shape(int shape, F &&f) {
    switch (shape) {
        case SHAPE_64x4x4: return f(ShapeTag<64, 4, 4>{});
        case SHAPE_32x8x2: return f(ShapeTag<32, 8, 2>{});
        case SHAPE_64x8x2:
        case SHAPE_64x8x4: return f(ShapeTag<64, 8, 2>{});
        case SHAPE_64x8x1: return f(ShapeTag<64, 8, 1>{});
        default: return f(ShapeTag<64, 4, 2>{});
    }
}

struct StencilCfg {
    int shape;
    int zlen;     // planes per z chunk (0 = chosen from the kernel's residency)
};

constexpr int kMaxDevices = 16;

// Tile extents of each shape (x, y).
inline void shape_extent(int shape, int &tx, int &ty) {
    switch (shape) {
        case SHAPE_64x4x4: tx = 64; ty = 16; break;
        case SHAPE_32x8x2: tx = 32; ty = 16; break;
        case SHAPE_64x8x2: tx = 64; ty = 16; break;
        case SHAPE_64x8x4: tx = 64; ty = 32; break;
        default: tx = 64; ty = 8; break;
    }
}

// Kernel families with entries of their own: the plain apply (which also has
// 64 x 32 tiles for FP64) and the fused single-pass stencil kernels (CG,
// residual, density-update passes).  FAMILY_ALL entries (set by hand) serve
// every family without an entry of its own.
enum TuneFamily { FAMILY_ALL = -1, FAMILY_APPLY = 0, FAMILY_PASS = 1, FAMILY_COUNT = 2 };

StencilCfg pick_stencil_cfg(const ofdft_grid &g, int elem_bytes, int family);
// The heuristic alone (no table).
StencilCfg default_stencil_cfg(const ofdft_grid &g, int elem_bytes, int family);
void record_stencil_cfg(const ofdft_grid &g, int elem_bytes, int family, StencilCfg c);
void erase_stencil_cfg(const ofdft_grid &g, int elem_bytes, int family);
int zlen_for_blocks(const ofdft_grid &g, int shape, int target_blocks);
// z-chunk length minimising (waves of workgroups) x (chunk planes + warm-up)
// for `resident` workgroups in flight; tiles of tx x ty points.
int zlen_auto(const ofdft_grid &g, int tx, int ty, int resident);

}  // namespace ofdft
