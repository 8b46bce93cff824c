// Network context of the learned solver aid.
#pragma once

#include <vector>

#include "nn_kernels.hpp"
#include "vec.hpp"

namespace ofdft {
namespace nn {

constexpr int kLayers = 15;
struct LayerDef {
    const char *name;
    int cin, cout;
};
extern const LayerDef kDefs[kLayers];

struct Level {                   // tensors of one resolution level
    Geo g{};
    std::vector<u16 *> t;        // activation / gradient buffers (see nn_net.hip)
};

}  // namespace nn
}  // namespace ofdft

struct ofdft_nn {
    // parameters
    float *w[ofdft::nn::kLayers] = {}, *m[ofdft::nn::kLayers] = {}, *v[ofdft::nn::kLayers] = {},
          *gr[ofdft::nn::kLayers] = {};
    ofdft::nn::u16 *wf[ofdft::nn::kLayers] = {}, *wb[ofdft::nn::kLayers] = {};
    float *wf32[ofdft::nn::kLayers] = {}, *wb32[ofdft::nn::kLayers] = {};   // FP32-mode copies
    int adam_t = 0;
    // activation storage: 0 = BF16 (default), 1 = FP32 (the FP32 mode of the
    // same kernels, for element-wise checks against the FP64 reference)
    int fp32 = 0;
    // workspace for one grid (and one activation storage type)
    int nx = 0, ny = 0, nz = 0, ws_fp32 = -1;
    std::vector<void *> ws;
    void *buf[64] = {};
    float *out = nullptr;
    float *part = nullptr, *part2 = nullptr;   // weight-gradient chunk partials, slice sums
    size_t part_cap = 0;
    double *totals = nullptr;
    ofdft::RedBuf rb{};
    // training loss: 0 = relative L2 error of the solution, 1 = relative
    // energy-norm error; FP64 scratch of the energy loss (n each)
    int loss_kind = 0;
    double *e64 = nullptr, *ae64 = nullptr;
    size_t e_cap = 0;
    std::vector<void *> allocs;
};

namespace ofdft {
namespace nn {

int net_reserve(ofdft_nn *net, const ofdft_grid &g);
// out (FP64) = h^2 * rms(in) * N(in / rms(in)), optionally shifted to zero mean
// (scale = h^2).  Workspace must have been reserved for g.
int net_apply(ofdft_nn *net, const ofdft_grid &g, const double *in, double *out, double h2,
              bool zero_mean, hipStream_t s);

}  // namespace nn
}  // namespace ofdft
