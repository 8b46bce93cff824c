// Stencil launch-shape table and heuristics.
#include <mutex>
#include <map>
#include <tuple>

#include "tuning.hpp"

namespace ofdft {

namespace {
std::mutex g_mu;
std::map<std::tuple<int, int, int, int>, StencilCfg> g_table;   // (nx, ny, nz, bytes)
}

int zlen_for_blocks(const ofdft_grid &g, int shape, int target_blocks) {
    int tx, ty;
    shape_extent(shape, tx, ty);
    const int64_t tiles = (int64_t)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
    int64_t chunks = (target_blocks + tiles - 1) / tiles;
    // keep chunks long enough that the 12-plane queue warm-up stays small
    const int64_t max_chunks = g.nz / 24 > 0 ? g.nz / 24 : 1;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    if (tiles * chunks > 8192) chunks = 8192 / tiles > 0 ? 8192 / tiles : 1;
    return (int)((g.nz + chunks - 1) / chunks);
}

int zlen_auto(const ofdft_grid &g, int tx, int ty, int resident) {
    if (resident < 1) resident = 1;
    const int64_t tiles = (int64_t)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
    const int max_chunks = g.nz / 8 > 0 ? g.nz / 8 : 1;     // chunks of at least 8 planes
    constexpr int kWarm = 8;                                 // warm-up cost in plane steps
    int best = g.nz;
    int64_t best_cost = -1;
    for (int c = 1; c <= max_chunks; ++c) {
        const int zl = (g.nz + c - 1) / c;
        const int64_t blocks = tiles * ((g.nz + zl - 1) / zl);
        if (blocks > kRedSlots) break;
        const int64_t waves = (blocks + resident - 1) / resident;
        const int64_t cost = waves * (zl + kWarm);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = zl;
        }
    }
    return best;
}

StencilCfg pick_stencil_cfg(const ofdft_grid &g, int elem_bytes, bool plain_f64) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(std::make_tuple(g.nx, g.ny, g.nz, elem_bytes));
        if (it != g_table.end()) return it->second;
    }
    StencilCfg c;
    // Measured at 320^3 on MI355X: real types run fastest with 64 x 16 tiles
    // of 512 threads (two rows each), complex128 with 64 x 8 tiles of 512
    // threads (one row each: two rows of complex128 need too many registers).
    if (g.nx <= 40 || (g.nx % 64 != 0 && g.nx % 64 <= 32 && g.nx < 256))
        c.shape = SHAPE_32x8x2;                          // avoid a mostly idle last x tile
    else c.shape = elem_bytes >= 16 ? SHAPE_64x8x1 : SHAPE_64x8x2;
    // the plain FP64 apply on wide grids: 64 x 32 tiles (four rows per
    // thread) halve the halo fetched per point and cut the LDS reads
    if (plain_f64 && g.nx % 64 == 0 && g.ny >= 128) c.shape = SHAPE_64x8x4;
    c.zlen = 0;
    return c;
}

}  // namespace ofdft

// Record a launch shape for one (grid, element size); shape < 0 removes it.
extern "C" int ofdft_stencil_set_config(int nx, int ny, int nz, int elem_bytes, int shape, int zlen) {
    using namespace ofdft;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(nx, ny, nz, elem_bytes);
    if (shape < 0) {
        g_table.erase(key);
        return OFDFT_OK;
    }
    if (shape >= SHAPE_COUNT || zlen < 0) {
        set_error("ofdft_stencil_set_config: bad shape %d / zlen %d", shape, zlen);
        return OFDFT_INVALID_ARG;
    }
    g_table[key] = StencilCfg{shape, zlen};
    return OFDFT_OK;
}
