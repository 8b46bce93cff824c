// Stencil launch-shape table and heuristics.
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "tuning.hpp"

namespace ofdft {

namespace {
std::mutex g_mu;
std::map<std::tuple<int, int, int, int, int>, StencilCfg> g_table;   // (nx, ny, nz, bytes, family)
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

StencilCfg default_stencil_cfg(const ofdft_grid &g, int elem_bytes, int family) {
    StencilCfg c;
    // Measured at 320^3 on MI355X: real types run fastest with 64 x 16 tiles
    // of 512 threads (two rows each), complex128 with 64 x 8 tiles of 512
    // threads (one row each: two rows of complex128 need too many registers).
    if (g.nx <= 40 || (g.nx % 64 != 0 && g.nx % 64 <= 32 && g.nx < 256))
        c.shape = SHAPE_32x8x2;                          // avoid a mostly idle last x tile
    else c.shape = elem_bytes >= 16 ? SHAPE_64x8x1 : SHAPE_64x8x2;
    // the plain FP64 apply on wide grids: 64 x 32 tiles (four rows per
    // thread) halve the halo fetched per point and cut the LDS reads
    if (family == FAMILY_APPLY && elem_bytes == 8 && g.nx % 64 == 0 && g.ny >= 128) c.shape = SHAPE_64x8x4;
    c.zlen = 0;
    return c;
}

StencilCfg pick_stencil_cfg(const ofdft_grid &g, int elem_bytes, int family) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(std::make_tuple(g.nx, g.ny, g.nz, elem_bytes, family));
        if (it != g_table.end()) return it->second;
        it = g_table.find(std::make_tuple(g.nx, g.ny, g.nz, elem_bytes, (int)FAMILY_ALL));
        if (it != g_table.end()) return it->second;
    }
    return default_stencil_cfg(g, elem_bytes, family);
}

void record_stencil_cfg(const ofdft_grid &g, int elem_bytes, int family, StencilCfg c) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[std::make_tuple(g.nx, g.ny, g.nz, elem_bytes, family)] = c;
}

void erase_stencil_cfg(const ofdft_grid &g, int elem_bytes, int family) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.erase(std::make_tuple(g.nx, g.ny, g.nz, elem_bytes, family));
}

// Text form of the table, one entry per line: family nx ny nz bytes shape zlen.
int table_save(const char *path) {
    std::lock_guard<std::mutex> lk(g_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) {
        set_error("ofdft_tune_save: cannot open %s", path);
        return OFDFT_INVALID_ARG;
    }
    std::fprintf(f, "# ofdft stencil launch table: family nx ny nz elem_bytes shape zlen\n");
    for (const auto &kv : g_table) {
        const auto &k = kv.first;
        std::fprintf(f, "%d %d %d %d %d %d %d\n", std::get<4>(k), std::get<0>(k), std::get<1>(k), std::get<2>(k),
                     std::get<3>(k), kv.second.shape, kv.second.zlen);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok) {
        set_error("ofdft_tune_save: writing %s failed", path);
        return OFDFT_INVALID_ARG;
    }
    return OFDFT_OK;
}

int table_load(const char *path, int *count) {
    FILE *f = std::fopen(path, "r");
    if (!f) {
        set_error("ofdft_tune_load: cannot open %s", path);
        return OFDFT_INVALID_ARG;
    }
    char line[256];
    int n = 0, lineno = 0;
    std::vector<std::pair<std::tuple<int, int, int, int, int>, StencilCfg>> entries;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        if (line[0] == '#' || line[0] == '\n') continue;
        int fam, nx, ny, nz, eb, shape, zlen;
        if (std::sscanf(line, "%d %d %d %d %d %d %d", &fam, &nx, &ny, &nz, &eb, &shape, &zlen) != 7 ||
            fam < FAMILY_ALL || fam >= FAMILY_COUNT || nx < 1 || ny < 1 || nz < 1 ||
            (eb != 4 && eb != 8 && eb != 16) || shape < 0 || shape >= SHAPE_COUNT || zlen < 0) {
            std::fclose(f);
            set_error("ofdft_tune_load: %s line %d is not a table entry", path, lineno);
            return OFDFT_INVALID_ARG;
        }
        entries.push_back({std::make_tuple(nx, ny, nz, eb, fam), StencilCfg{shape, zlen}});
        ++n;
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &e : entries) g_table[e.first] = e.second;
    if (count) *count = n;
    return OFDFT_OK;
}

}  // namespace ofdft

// Record a launch shape for one (grid, element size), every family; shape < 0
// removes that entry and the tuned entries of the grid.
extern "C" int ofdft_stencil_set_config(int nx, int ny, int nz, int elem_bytes, int shape, int zlen) {
    using namespace ofdft;
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(nx, ny, nz, elem_bytes, (int)FAMILY_ALL);
    if (shape < 0) {
        for (int f = FAMILY_ALL; f < FAMILY_COUNT; ++f) g_table.erase(std::make_tuple(nx, ny, nz, elem_bytes, f));
        return OFDFT_OK;
    }
    if (shape >= SHAPE_COUNT || zlen < 0) {
        set_error("ofdft_stencil_set_config: bad shape %d / zlen %d", shape, zlen);
        return OFDFT_INVALID_ARG;
    }
    // a hand-set shape overrides the tuned entries of the grid
    for (int f = 0; f < FAMILY_COUNT; ++f) g_table.erase(std::make_tuple(nx, ny, nz, elem_bytes, f));
    g_table[key] = StencilCfg{shape, zlen};
    return OFDFT_OK;
}

extern "C" int ofdft_tune_save(const char *path) {
    if (!path) {
        ofdft::set_error("ofdft_tune_save: NULL path");
        return OFDFT_INVALID_ARG;
    }
    return ofdft::table_save(path);
}

extern "C" int ofdft_tune_load(const char *path, int *entries) {
    if (!path) {
        ofdft::set_error("ofdft_tune_load: NULL path");
        return OFDFT_INVALID_ARG;
    }
    return ofdft::table_load(path, entries);
}
