// Network context: parameters, per-grid workspaces, forward / backward
// orchestration, Adam, and the C entry points of the learned solver aid.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>

#include "nn.hpp"
#include "nn_device.hpp"
#include "profile.hpp"

namespace ofdft {
namespace nn {

const LayerDef kDefs[kLayers] = {
    {"c0a", 1, 16}, {"c0b", 16, 16}, {"c1a", 16, 32}, {"c1b", 32, 32}, {"c2a", 32, 64},
    {"c2b", 64, 64}, {"c3a", 64, 64}, {"c3b", 64, 64}, {"d2a", 128, 64}, {"d2b", 64, 64},
    {"d1a", 96, 32}, {"d1b", 32, 32}, {"d0a", 48, 16}, {"d0b", 16, 16}, {"out", 16, 1},
};

namespace {

// workspace tensors: (level, channels)
enum Buf {
    X0, A0, S0, D0A, D0, P0, A1, S1, D1A, D1, P1, A2, S2, D2A, D2, P2, A3, B3,
    dOUT, dD0, dD0A, dCAT0, dS0, dA0, dD1, dD1A, dCAT1, dP0, dS1, dA1,
    dD2, dD2A, dCAT2, dP1, dS2, dA2, dB3, dA3, dP2, NBUF
};
const int kBufLevel[NBUF] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3,
                             0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3};
const int kBufCh[NBUF] = {1, 16, 16, 16, 16, 16, 32, 32, 32, 32, 32, 64, 64, 64, 64, 64, 64, 64,
                          1, 16, 16, 48, 16, 16, 32, 32, 96, 16, 32, 32, 64, 64, 128, 32, 64, 64,
                          64, 64, 64};

int ntile(int c) { return (c + 15) / 16; }
constexpr int kWgradSlices = 32;    // first-stage slices of the weight-gradient chunk sum

Geo geo_of(const ofdft_nn *net, int level) {
    Geo g;
    g.nx = net->nx >> level;
    g.ny = net->ny >> level;
    g.nz = net->nz >> level;
    g.npts = g.nx * g.ny * g.nz;
    return g;
}

template <typename P>
int nalloc(ofdft_nn *net, P **p, size_t bytes, std::vector<void *> &list) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(bytes, 256)) != hipSuccess) {
        set_error("network: out of device memory (%zu bytes)", bytes);
        return OFDFT_NO_MEMORY;
    }
    list.push_back(q);
    *p = (P *)q;
    return OFDFT_OK;
}

template <typename A>
InDescT<A> one(const void *s, int c, const void *mask = nullptr) {
    InDescT<A> d{};
    d.s1 = (const A *)s;
    d.mask1 = (const A *)mask;
    d.c1 = c;
    return d;
}
template <typename A>
InDescT<A> cat(const void *coarse, int c1, const void *skip, int c2) {
    InDescT<A> d{};
    d.s1 = (const A *)coarse;
    d.c1 = c1;
    d.up1 = 1;
    d.s2 = (const A *)skip;
    d.c2 = c2;
    return d;
}

// launch a convolution: cin == 1 uses the tap-packed path
template <typename A>
int conv(const InDescT<A> &in, const Geo &g, const A *w, int cin, int cout, void *out_act, float *out_f32,
         bool relu, hipStream_t s) {
    const int blocks = (g.npts + 63) / 64;
    // algorithmic bytes: read the input once, write the output once
    ProfScope ps(K_NN, (double)g.npts * sizeof(A) * (cin + cout), s);
    const int r = relu ? 1 : 0;
    A *oa = (A *)out_act;
    if (cin == 1) {
        switch (ntile(cout)) {
            case 1: hipLaunchKernelGGL((conv_c1<1, A>), dim3(blocks), dim3(256), 0, s, in, g, w, cout, oa, out_f32, r); break;
            case 2: hipLaunchKernelGGL((conv_c1<2, A>), dim3(blocks), dim3(256), 0, s, in, g, w, cout, oa, out_f32, r); break;
            default: hipLaunchKernelGGL((conv_c1<4, A>), dim3(blocks), dim3(256), 0, s, in, g, w, cout, oa, out_f32, r); break;
        }
    } else {
        // bricks of 16 x 4 x 4 points; at most 4 output tiles per block
        const int nbx = (g.nx + kWbX - 1) / kWbX, nby = (g.ny + kWbY - 1) / kWbY, nbz = (g.nz + kWbZ - 1) / kWbZ;
        const int nt = ntile(cout);
        const int ntb = nt <= 4 ? nt : (nt % 4 == 0 ? 4 : 3);
        if (nt % ntb) {
            set_error("network: unsupported channel count %d", cout);
            return OFDFT_INVALID_ARG;
        }
        const dim3 grid(nbx * nby * nbz, nt / ntb);
        switch (ntb) {
            case 1: hipLaunchKernelGGL((conv_brick<1, A>), grid, dim3(256), 0, s, in, g, w, cin, cout, oa, out_f32, r, nbx, nby); break;
            case 2: hipLaunchKernelGGL((conv_brick<2, A>), grid, dim3(256), 0, s, in, g, w, cin, cout, oa, out_f32, r, nbx, nby); break;
            case 3: hipLaunchKernelGGL((conv_brick<3, A>), grid, dim3(256), 0, s, in, g, w, cin, cout, oa, out_f32, r, nbx, nby); break;
            default: hipLaunchKernelGGL((conv_brick<4, A>), grid, dim3(256), 0, s, in, g, w, cin, cout, oa, out_f32, r, nbx, nby); break;
        }
    }
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

template <typename A>
int wgrad(ofdft_nn *net, int layer, const InDescT<A> &x, const Geo &g, const void *dy, const void *ymask,
          hipStream_t s) {
    const int cin = kDefs[layer].cin, cout = kDefs[layer].cout;
    int nbx, nby, ngz;
    const int chunks = wb_chunks(g, nbx, nby, ngz);
    const size_t count = (size_t)27 * cin * cout;
    if ((size_t)chunks * count > net->part_cap) {
        set_error("network: weight-gradient scratch too small");
        return OFDFT_INVALID_ARG;
    }
    ProfScope ps(K_NN, (double)g.npts * sizeof(A) * (cin + cout), s);
    hipLaunchKernelGGL(conv_wgrad_brick<A>, dim3(chunks, ntile(cin) * ntile(cout)), dim3(256), 0, s, x, g,
                       (const A *)dy, (const A *)ymask, cin, cout, nbx, nby, net->part);
    OFDFT_CHECK_HIP(hipGetLastError());
    // the chunk sum in two fixed-order stages (slices of chunks, then the slices)
    const int slices = std::min(kWgradSlices, chunks);
    hipLaunchKernelGGL(wgrad_reduce_slices, dim3((unsigned)((count + 255) / 256), slices), dim3(256), 0, s,
                       net->part, chunks, (int)count, slices, net->part2);
    OFDFT_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(wgrad_reduce, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, net->part2,
                       slices, (int)count, net->gr[layer]);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

int grid_blocks(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 8192); }

}  // namespace

int net_reserve(ofdft_nn *net, const ofdft_grid &g) {
    if (g.nx % 8 || g.ny % 8 || g.nz % 8) {
        set_error("network: grid sizes must be multiples of 8 (got %d x %d x %d)", g.nx, g.ny, g.nz);
        return OFDFT_INVALID_ARG;
    }
    if (net->nx == g.nx && net->ny == g.ny && net->nz == g.nz && net->ws_fp32 == net->fp32) return OFDFT_OK;
    for (void *p : net->ws) (void)hipFree(p);
    net->ws.clear();
    net->nx = g.nx;
    net->ny = g.ny;
    net->nz = g.nz;
    net->ws_fp32 = net->fp32;
    const size_t elem = net->fp32 ? sizeof(float) : sizeof(u16);
    for (int b = 0; b < NBUF; ++b) {
        const Geo gg = geo_of(net, kBufLevel[b]);
        OFDFT_TRY(nalloc(net, &net->buf[b], elem * (size_t)gg.npts * kBufCh[b], net->ws));
    }
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    OFDFT_TRY(nalloc(net, &net->out, sizeof(float) * n, net->ws));
    size_t cap = 0;
    for (int l = 0; l < kLayers; ++l) {
        // layer l runs on the level of its output
        static const int lvl[kLayers] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0};
        const Geo gg = geo_of(net, lvl[l]);
        int nbx, nby, ngz;
        const size_t chunks = (size_t)wb_chunks(gg, nbx, nby, ngz);
        cap = std::max(cap, chunks * 27 * kDefs[l].cin * kDefs[l].cout);
    }
    OFDFT_TRY(nalloc(net, &net->part, sizeof(float) * cap, net->ws));
    net->part_cap = cap;
    size_t cmax = 0;
    for (int l = 0; l < kLayers; ++l) cmax = std::max(cmax, (size_t)27 * kDefs[l].cin * kDefs[l].cout);
    OFDFT_TRY(nalloc(net, &net->part2, sizeof(float) * cmax * kWgradSlices, net->ws));
    return OFDFT_OK;
}

template <typename A> const A *wfwd(const ofdft_nn *net, int l);
template <> const u16 *wfwd<u16>(const ofdft_nn *net, int l) { return net->wf[l]; }
template <> const float *wfwd<float>(const ofdft_nn *net, int l) { return net->wf32[l]; }
template <typename A> const A *wbwd(const ofdft_nn *net, int l);
template <> const u16 *wbwd<u16>(const ofdft_nn *net, int l) { return net->wb[l]; }
template <> const float *wbwd<float>(const ofdft_nn *net, int l) { return net->wb32[l]; }

// forward pass from net->buf[X0]; output FP32 in net->out
template <typename A>
static int forward_t(ofdft_nn *net, hipStream_t s) {
    void **B = net->buf;
    const Geo g0 = geo_of(net, 0), g1 = geo_of(net, 1), g2 = geo_of(net, 2), g3 = geo_of(net, 3);
    auto W = [&](int l) { return wfwd<A>(net, l); };
    auto one = [](const void *p, int c, const void *mask = nullptr) { return ::ofdft::nn::one<A>(p, c, mask); };
    auto cat = [](const void *a, int c1, const void *b, int c2) { return ::ofdft::nn::cat<A>(a, c1, b, c2); };
    auto P = [&](int b) { return (A *)B[b]; };
    OFDFT_TRY(conv(one(B[X0], 1), g0, W(0), 1, 16, B[A0], nullptr, true, s));
    OFDFT_TRY(conv(one(B[A0], 16), g0, W(1), 16, 16, B[S0], nullptr, true, s));
    hipLaunchKernelGGL(pool2<A>, dim3(grid_blocks((int64_t)g1.npts * 16)), dim3(256), 0, s, P(S0), g0, 16, P(P0));
    OFDFT_TRY(conv(one(B[P0], 16), g1, W(2), 16, 32, B[A1], nullptr, true, s));
    OFDFT_TRY(conv(one(B[A1], 32), g1, W(3), 32, 32, B[S1], nullptr, true, s));
    hipLaunchKernelGGL(pool2<A>, dim3(grid_blocks((int64_t)g2.npts * 32)), dim3(256), 0, s, P(S1), g1, 32, P(P1));
    OFDFT_TRY(conv(one(B[P1], 32), g2, W(4), 32, 64, B[A2], nullptr, true, s));
    OFDFT_TRY(conv(one(B[A2], 64), g2, W(5), 64, 64, B[S2], nullptr, true, s));
    hipLaunchKernelGGL(pool2<A>, dim3(grid_blocks((int64_t)g3.npts * 64)), dim3(256), 0, s, P(S2), g2, 64, P(P2));
    OFDFT_TRY(conv(one(B[P2], 64), g3, W(6), 64, 64, B[A3], nullptr, true, s));
    OFDFT_TRY(conv(one(B[A3], 64), g3, W(7), 64, 64, B[B3], nullptr, true, s));
    OFDFT_TRY(conv(cat(B[B3], 64, B[S2], 64), g2, W(8), 128, 64, B[D2A], nullptr, true, s));
    OFDFT_TRY(conv(one(B[D2A], 64), g2, W(9), 64, 64, B[D2], nullptr, true, s));
    OFDFT_TRY(conv(cat(B[D2], 64, B[S1], 32), g1, W(10), 96, 32, B[D1A], nullptr, true, s));
    OFDFT_TRY(conv(one(B[D1A], 32), g1, W(11), 32, 32, B[D1], nullptr, true, s));
    OFDFT_TRY(conv(cat(B[D1], 32, B[S0], 16), g0, W(12), 48, 16, B[D0A], nullptr, true, s));
    OFDFT_TRY(conv(one(B[D0A], 16), g0, W(13), 16, 16, B[D0], nullptr, true, s));
    OFDFT_TRY(conv(one(B[D0], 16), g0, W(14), 16, 1, nullptr, net->out, false, s));
    return OFDFT_OK;
}

static int forward(ofdft_nn *net, hipStream_t s) {
    return net->fp32 ? forward_t<float>(net, s) : forward_t<u16>(net, s);
}

// backward pass from net->buf[dOUT]; weight gradients into net->gr
template <typename A>
static int backward_t(ofdft_nn *net, hipStream_t s) {
    void **B = net->buf;
    const Geo g0 = geo_of(net, 0), g1 = geo_of(net, 1), g2 = geo_of(net, 2), g3 = geo_of(net, 3);
    auto WB = [&](int l) { return wbwd<A>(net, l); };
    auto one = [](const void *p, int c, const void *mask = nullptr) { return ::ofdft::nn::one<A>(p, c, mask); };
    auto cat = [](const void *a, int c1, const void *b, int c2) { return ::ofdft::nn::cat<A>(a, c1, b, c2); };
    auto P = [&](int b) { return (A *)B[b]; };
    // out (no activation)
    OFDFT_TRY(wgrad(net, 14, one(B[D0], 16), g0, B[dOUT], nullptr, s));
    OFDFT_TRY(conv(one(B[dOUT], 1), g0, WB(14), 1, 16, B[dD0], nullptr, false, s));
    // level 0 decoder
    OFDFT_TRY(wgrad(net, 13, one(B[D0A], 16), g0, B[dD0], B[D0], s));
    OFDFT_TRY(conv(one(B[dD0], 16, B[D0]), g0, WB(13), 16, 16, B[dD0A], nullptr, false, s));
    OFDFT_TRY(wgrad(net, 12, cat(B[D1], 32, B[S0], 16), g0, B[dD0A], B[D0A], s));
    OFDFT_TRY(conv(one(B[dD0A], 16, B[D0A]), g0, WB(12), 16, 48, B[dCAT0], nullptr, false, s));
    hipLaunchKernelGGL(up_grad<A>, dim3(grid_blocks((int64_t)g1.npts * 32)), dim3(256), 0, s, P(dCAT0), g0, 48, 32, P(dD1));
    // level 1 decoder
    OFDFT_TRY(wgrad(net, 11, one(B[D1A], 32), g1, B[dD1], B[D1], s));
    OFDFT_TRY(conv(one(B[dD1], 32, B[D1]), g1, WB(11), 32, 32, B[dD1A], nullptr, false, s));
    OFDFT_TRY(wgrad(net, 10, cat(B[D2], 64, B[S1], 32), g1, B[dD1A], B[D1A], s));
    OFDFT_TRY(conv(one(B[dD1A], 32, B[D1A]), g1, WB(10), 32, 96, B[dCAT1], nullptr, false, s));
    hipLaunchKernelGGL(up_grad<A>, dim3(grid_blocks((int64_t)g2.npts * 64)), dim3(256), 0, s, P(dCAT1), g1, 96, 64, P(dD2));
    // level 2 decoder
    OFDFT_TRY(wgrad(net, 9, one(B[D2A], 64), g2, B[dD2], B[D2], s));
    OFDFT_TRY(conv(one(B[dD2], 64, B[D2]), g2, WB(9), 64, 64, B[dD2A], nullptr, false, s));
    OFDFT_TRY(wgrad(net, 8, cat(B[B3], 64, B[S2], 64), g2, B[dD2A], B[D2A], s));
    OFDFT_TRY(conv(one(B[dD2A], 64, B[D2A]), g2, WB(8), 64, 128, B[dCAT2], nullptr, false, s));
    hipLaunchKernelGGL(up_grad<A>, dim3(grid_blocks((int64_t)g3.npts * 64)), dim3(256), 0, s, P(dCAT2), g2, 128, 64, P(dB3));
    // bottleneck
    OFDFT_TRY(wgrad(net, 7, one(B[A3], 64), g3, B[dB3], B[B3], s));
    OFDFT_TRY(conv(one(B[dB3], 64, B[B3]), g3, WB(7), 64, 64, B[dA3], nullptr, false, s));
    OFDFT_TRY(wgrad(net, 6, one(B[P2], 64), g3, B[dA3], B[A3], s));
    OFDFT_TRY(conv(one(B[dA3], 64, B[A3]), g3, WB(6), 64, 64, B[dP2], nullptr, false, s));
    // level 2 encoder: skip gradient + pooled path
    hipLaunchKernelGGL(skip_grad<A>, dim3(grid_blocks((int64_t)g2.npts * 64)), dim3(256), 0, s, P(dCAT2), g2, 128, 64, 64, P(dP2), P(dS2));
    OFDFT_TRY(wgrad(net, 5, one(B[A2], 64), g2, B[dS2], B[S2], s));
    OFDFT_TRY(conv(one(B[dS2], 64, B[S2]), g2, WB(5), 64, 64, B[dA2], nullptr, false, s));
    OFDFT_TRY(wgrad(net, 4, one(B[P1], 32), g2, B[dA2], B[A2], s));
    OFDFT_TRY(conv(one(B[dA2], 64, B[A2]), g2, WB(4), 64, 32, B[dP1], nullptr, false, s));
    // level 1 encoder
    hipLaunchKernelGGL(skip_grad<A>, dim3(grid_blocks((int64_t)g1.npts * 32)), dim3(256), 0, s, P(dCAT1), g1, 96, 64, 32, P(dP1), P(dS1));
    OFDFT_TRY(wgrad(net, 3, one(B[A1], 32), g1, B[dS1], B[S1], s));
    OFDFT_TRY(conv(one(B[dS1], 32, B[S1]), g1, WB(3), 32, 32, B[dA1], nullptr, false, s));
    OFDFT_TRY(wgrad(net, 2, one(B[P0], 16), g1, B[dA1], B[A1], s));
    OFDFT_TRY(conv(one(B[dA1], 32, B[A1]), g1, WB(2), 32, 16, B[dP0], nullptr, false, s));
    // level 0 encoder
    hipLaunchKernelGGL(skip_grad<A>, dim3(grid_blocks((int64_t)g0.npts * 16)), dim3(256), 0, s, P(dCAT0), g0, 48, 32, 16, P(dP0), P(dS0));
    OFDFT_TRY(wgrad(net, 1, one(B[A0], 16), g0, B[dS0], B[S0], s));
    OFDFT_TRY(conv(one(B[dS0], 16, B[S0]), g0, WB(1), 16, 16, B[dA0], nullptr, false, s));
    OFDFT_TRY(wgrad(net, 0, one(B[X0], 1), g0, B[dA0], B[A0], s));
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

static int backward(ofdft_nn *net, hipStream_t s) {
    return net->fp32 ? backward_t<float>(net, s) : backward_t<u16>(net, s);
}

static int pack_all(ofdft_nn *net, hipStream_t s) {
    for (int l = 0; l < kLayers; ++l) {
        hipLaunchKernelGGL(pack_weights<u16>, dim3(64), dim3(256), 0, s, net->w[l], kDefs[l].cin, kDefs[l].cout,
                           ntile(kDefs[l].cout), ntile(kDefs[l].cin), net->wf[l], net->wb[l]);
        OFDFT_CHECK_HIP(hipGetLastError());
        hipLaunchKernelGGL(pack_weights<float>, dim3(64), dim3(256), 0, s, net->w[l], kDefs[l].cin, kDefs[l].cout,
                           ntile(kDefs[l].cout), ntile(kDefs[l].cin), net->wf32[l], net->wb32[l]);
        OFDFT_CHECK_HIP(hipGetLastError());
    }
    return OFDFT_OK;
}

// x = input / rms(input) in the activation type (totals[0] = sum input^2).
int cast_input(ofdft_nn *net, int64_t n, const double *in, hipStream_t s) {
    if (net->fp32)
        return launch_reduce<1>(n, CastInOp<float>{in, (float *)net->buf[X0], net->totals, 1.0 / n, 0.0}, NoFin{},
                                net->rb, s);
    return launch_reduce<1>(n, CastInOp<u16>{in, (u16 *)net->buf[X0], net->totals, 1.0 / n, 0.0}, NoFin{},
                            net->rb, s);
}

struct ToF64Op {          // out = h2 * rms * out32 (rms from totals {sum in^2})
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 12;
    const float *o;
    double *out;
    const double *totals;
    double inv_n, h2, scale;
    __device__ bool skip() const { return false; }
    __device__ void prepare() { scale = h2 * sqrt(totals[0] * inv_n); }
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        const double v = scale * (double)o[i];
        out[i] = v;
        acc[0] += v;
    }
};

struct SubMeanOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 16;
    double *a;
    const double *totals;
    double inv_n, mean;
    __device__ bool skip() const { return false; }
    __device__ void prepare() { mean = totals[0] * inv_n; }
    __device__ void operator()(int64_t i, double (&)[1]) const { a[i] -= mean; }
};

int net_apply(ofdft_nn *net, const ofdft_grid &g, const double *in, double *out, double h2,
              bool zero_mean, hipStream_t s) {
    if (g.nx != net->nx || g.ny != net->ny || g.nz != net->nz) {
        set_error("network: workspace not reserved for this grid");
        return OFDFT_INVALID_ARG;
    }
    const int64_t n = npoints(g);
    OFDFT_TRY((launch_reduce<1>(n, SqOp{in}, StoreTotals<1>{net->totals}, net->rb, s)));
    OFDFT_TRY(cast_input(net, n, in, s));
    OFDFT_TRY(forward(net, s));
    OFDFT_TRY((launch_reduce<1>(n, ToF64Op{net->out, out, net->totals, 1.0 / n, h2, 0.0},
                                StoreTotals<1>{net->totals + 4}, net->rb, s)));
    if (zero_mean)
        OFDFT_TRY((launch_reduce<1>(n, SubMeanOp{out, net->totals + 4, 1.0 / n, 0.0}, NoFin{}, net->rb, s)));
    return OFDFT_OK;
}

}  // namespace nn
}  // namespace ofdft

using namespace ofdft;
using namespace ofdft::nn;

static void net_free(ofdft_nn *net) {
    for (void *p : net->ws) (void)hipFree(p);
    for (void *p : net->allocs) (void)hipFree(p);
    net->ws.clear();
    net->allocs.clear();
    if (net->e64) (void)hipFree(net->e64);
    if (net->ae64) (void)hipFree(net->ae64);
    net->e64 = net->ae64 = nullptr;
    net->e_cap = 0;
    redbuf_free(net->rb);
}

extern "C" size_t ofdft_nn_param_count(void) {
    size_t c = 0;
    for (int l = 0; l < kLayers; ++l) c += (size_t)27 * kDefs[l].cin * kDefs[l].cout;
    return c;
}

extern "C" int ofdft_nn_create(uint64_t seed, ofdft_nn **out) {
    if (!out) return OFDFT_INVALID_ARG;
    ofdft_nn *net = new (std::nothrow) ofdft_nn();
    if (!net) return OFDFT_NO_MEMORY;
    auto fail = [&](int st) {
        net_free(net);
        delete net;
        return st;
    };
    std::mt19937_64 rng(seed);
    for (int l = 0; l < kLayers; ++l) {
        const int cin = kDefs[l].cin, cout = kDefs[l].cout;
        const size_t cnt = (size_t)27 * cin * cout;
        int st;
        if ((st = nalloc(net, &net->w[l], sizeof(float) * cnt, net->allocs)) ||
            (st = nalloc(net, &net->m[l], sizeof(float) * cnt, net->allocs)) ||
            (st = nalloc(net, &net->v[l], sizeof(float) * cnt, net->allocs)) ||
            (st = nalloc(net, &net->gr[l], sizeof(float) * cnt, net->allocs)) ||
            (st = nalloc(net, &net->wf[l], sizeof(u16) * (cin == 1 ? ntile(cout) * 16 * 32 : 27 * ntile(cout) * 16 * cin), net->allocs)) ||
            (st = nalloc(net, &net->wb[l], sizeof(u16) * (cout == 1 ? ntile(cin) * 16 * 32 : 27 * ntile(cin) * 16 * cout), net->allocs)) ||
            (st = nalloc(net, &net->wf32[l], sizeof(float) * (cin == 1 ? ntile(cout) * 16 * 32 : 27 * ntile(cout) * 16 * cin), net->allocs)) ||
            (st = nalloc(net, &net->wb32[l], sizeof(float) * (cout == 1 ? ntile(cin) * 16 * 32 : 27 * ntile(cin) * 16 * cout), net->allocs)))
            return fail(st);
        // He-normal initialisation, fan-in 27 cin
        std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (27.f * cin)));
        std::vector<float> h(cnt);
        for (auto &x : h) x = nd(rng);
        if (hipMemcpy(net->w[l], h.data(), sizeof(float) * cnt, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(net->m[l], 0, sizeof(float) * cnt) != hipSuccess ||
            hipMemset(net->v[l], 0, sizeof(float) * cnt) != hipSuccess)
            return fail(OFDFT_HIP_ERROR);
    }
    int st;
    if ((st = nalloc(net, &net->totals, sizeof(double) * 16, net->allocs)) || (st = redbuf_alloc(net->rb)))
        return fail(st);
    if ((st = pack_all(net, nullptr))) return fail(st);
    if (hipDeviceSynchronize() != hipSuccess) return fail(OFDFT_HIP_ERROR);
    *out = net;
    return OFDFT_OK;
}

extern "C" int ofdft_nn_destroy(ofdft_nn *net) {
    if (!net) return OFDFT_OK;
    net_free(net);
    delete net;
    return OFDFT_OK;
}

// weights: host FP32 array of ofdft_nn_param_count() values, layer after layer,
// each W[t][ci][co] with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)
extern "C" int ofdft_nn_set_weights(ofdft_nn *net, const float *w, size_t count) {
    if (!net || !w || count != ofdft_nn_param_count()) {
        set_error("ofdft_nn_set_weights: expected %zu values", ofdft_nn_param_count());
        return OFDFT_INVALID_ARG;
    }
    size_t off = 0;
    for (int l = 0; l < kLayers; ++l) {
        const size_t cnt = (size_t)27 * kDefs[l].cin * kDefs[l].cout;
        OFDFT_CHECK_HIP(hipMemcpy(net->w[l], w + off, sizeof(float) * cnt, hipMemcpyHostToDevice));
        off += cnt;
    }
    OFDFT_TRY(pack_all(net, nullptr));
    OFDFT_CHECK_HIP(hipDeviceSynchronize());
    net->adam_t = 0;
    return OFDFT_OK;
}

extern "C" int ofdft_nn_get_weights(ofdft_nn *net, float *w, size_t count, int gradients) {
    if (!net || !w || count != ofdft_nn_param_count()) {
        set_error("ofdft_nn_get_weights: expected %zu values", ofdft_nn_param_count());
        return OFDFT_INVALID_ARG;
    }
    OFDFT_CHECK_HIP(hipDeviceSynchronize());
    size_t off = 0;
    for (int l = 0; l < kLayers; ++l) {
        const size_t cnt = (size_t)27 * kDefs[l].cin * kDefs[l].cout;
        OFDFT_CHECK_HIP(hipMemcpy(w + off, gradients ? net->gr[l] : net->w[l], sizeof(float) * cnt,
                                  hipMemcpyDeviceToHost));
        off += cnt;
    }
    return OFDFT_OK;
}

// Network checkpoint: a header (magic, parameter count, Adam step, loss
// kind, activation storage), then every layer's FP32 weights and Adam
// moments; load repacks the BF16 / FP32 copies.
namespace {
constexpr char kNnMagic[8] = {'O', 'F', 'D', 'F', 'T', 'N', 'N', '1'};
struct NnHeader {
    char magic[8];
    int64_t params, adam_t, loss_kind, fp32;
};
}  // namespace

extern "C" int ofdft_nn_save(ofdft_nn *net, const char *path) {
    if (!net || !path) {
        set_error("ofdft_nn_save: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    OFDFT_CHECK_HIP(hipDeviceSynchronize());
    std::FILE *f = std::fopen(path, "wb");
    if (!f) {
        set_error("ofdft_nn_save: cannot open %s", path);
        return OFDFT_INVALID_ARG;
    }
    NnHeader h{};
    std::memcpy(h.magic, kNnMagic, 8);
    h.params = (int64_t)ofdft_nn_param_count();
    h.adam_t = net->adam_t;
    h.loss_kind = net->loss_kind;
    h.fp32 = net->fp32;
    int rc = ck_write(f, &h, sizeof h);
    for (int l = 0; rc == OFDFT_OK && l < kLayers; ++l) {
        const size_t b = sizeof(float) * 27 * kDefs[l].cin * kDefs[l].cout;
        if ((rc = ck_write_dev(f, net->w[l], b)) == OFDFT_OK && (rc = ck_write_dev(f, net->m[l], b)) == OFDFT_OK)
            rc = ck_write_dev(f, net->v[l], b);
    }
    if (std::fclose(f) != 0 && rc == OFDFT_OK) {
        set_error("ofdft_nn_save: closing %s failed", path);
        rc = OFDFT_INVALID_ARG;
    }
    return rc;
}

extern "C" int ofdft_nn_load(ofdft_nn *net, const char *path) {
    if (!net || !path) {
        set_error("ofdft_nn_load: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    std::FILE *f = std::fopen(path, "rb");
    if (!f) {
        set_error("ofdft_nn_load: cannot open %s", path);
        return OFDFT_INVALID_ARG;
    }
    NnHeader h{};
    int rc = ck_read(f, &h, sizeof h);
    if (rc == OFDFT_OK && (std::memcmp(h.magic, kNnMagic, 8) != 0 || h.params != (int64_t)ofdft_nn_param_count() ||
                           h.loss_kind < 0 || h.loss_kind > 2 || (h.fp32 != 0 && h.fp32 != 1) || h.adam_t < 0)) {
        set_error("ofdft_nn_load: %s is not a checkpoint of this network", path);
        rc = OFDFT_INVALID_ARG;
    }
    for (int l = 0; rc == OFDFT_OK && l < kLayers; ++l) {
        const size_t b = sizeof(float) * 27 * kDefs[l].cin * kDefs[l].cout;
        if ((rc = ck_read_dev(f, net->w[l], b)) == OFDFT_OK && (rc = ck_read_dev(f, net->m[l], b)) == OFDFT_OK)
            rc = ck_read_dev(f, net->v[l], b);
    }
    std::fclose(f);
    if (rc != OFDFT_OK) return rc;
    net->adam_t = (int)h.adam_t;
    net->loss_kind = (int)h.loss_kind;
    net->fp32 = (int)h.fp32;
    OFDFT_TRY(pack_all(net, nullptr));
    OFDFT_CHECK_HIP(hipDeviceSynchronize());
    return OFDFT_OK;
}

extern "C" int ofdft_nn_set_loss(ofdft_nn *net, int kind) {
    if (!net || kind < 0 || kind > 2) {
        set_error("ofdft_nn_set_loss: kind must be 0 (L2), 1 (energy norm) or 2 (residual norm)");
        return OFDFT_INVALID_ARG;
    }
    net->loss_kind = kind;
    return OFDFT_OK;
}

// Activation storage of the network's kernels: 0 = BF16 (default), 1 = FP32
// (same kernels, FP32 MFMA; the workspace is reallocated on the next use).
extern "C" int ofdft_nn_set_precision(ofdft_nn *net, int fp32) {
    if (!net || (fp32 != 0 && fp32 != 1)) {
        set_error("ofdft_nn_set_precision: fp32 must be 0 (BF16) or 1 (FP32)");
        return OFDFT_INVALID_ARG;
    }
    net->fp32 = fp32;
    return OFDFT_OK;
}

extern "C" int ofdft_nn_reserve(ofdft_nn *net, const ofdft_grid *grid) {
    if (!net) return OFDFT_INVALID_ARG;
    OFDFT_TRY(check_grid(grid, 1));
    return net_reserve(net, *grid);
}

// out = N(in) with the scaling used by the solver: in / rms(in) -> network ->
// times scale * rms(in) (scale = h^2 for a preconditioner / initial guess).
extern "C" int ofdft_nn_forward(ofdft_nn *net, const ofdft_grid *grid, const double *in, double *out,
                                double scale, void *stream) {
    if (!net || !in || !out) return OFDFT_INVALID_ARG;
    OFDFT_TRY(check_grid(grid, 1));
    OFDFT_TRY(net_reserve(net, *grid));
    return net_apply(net, *grid, in, out, scale, false, (hipStream_t)stream);
}

// Numerator a.b of an operator-weighted loss and dL/d(out) = 2 grad / den.
static int energy_loss(ofdft_nn *net, int64_t n, const double *a, const double *b, const double *grad, double h2,
                       hipStream_t s) {
    if (net->fp32)
        return launch_reduce<1>(n, EnergyLossOp<float>{a, b, grad, (float *)net->buf[dOUT], net->totals, 1.0 / n,
                                                       h2, 0},
                                StoreTotals<1>{net->totals + 2}, net->rb, s);
    return launch_reduce<1>(n, EnergyLossOp<u16>{a, b, grad, (u16 *)net->buf[dOUT], net->totals, 1.0 / n, h2, 0},
                            StoreTotals<1>{net->totals + 2}, net->rb, s);
}

// Loss of the current output against phi, and dL/d(out) into buf[dOUT].
// totals[0] = sum g^2 must be set; leaves totals[1] = the loss denominator
// before scaling and totals[2] = its numerator.
static int loss_pass(ofdft_nn *net, const ofdft_grid &g, const double *phi, double h2, hipStream_t s) {
    const int64_t n = npoints(g);
    if (net->loss_kind == 0) {
        OFDFT_TRY((launch_reduce<1>(n, SqOp{phi}, StoreTotals<1>{net->totals + 1}, net->rb, s)));
        OFDFT_TRY(forward(net, s));
        if (net->fp32)
            return launch_reduce<1>(n, LossOp<float>{net->out, phi, (float *)net->buf[dOUT], net->totals, 1.0 / n,
                                                     h2, 0, 0},
                                    StoreTotals<1>{net->totals + 2}, net->rb, s);
        return launch_reduce<1>(n, LossOp<u16>{net->out, phi, (u16 *)net->buf[dOUT], net->totals, 1.0 / n, h2, 0, 0},
                                StoreTotals<1>{net->totals + 2}, net->rb, s);
    }
    if (net->e_cap < (size_t)n) {
        if (net->e64) OFDFT_CHECK_HIP(hipFree(net->e64));
        if (net->ae64) OFDFT_CHECK_HIP(hipFree(net->ae64));
        net->e64 = net->ae64 = nullptr;
        net->e_cap = 0;
        OFDFT_CHECK_HIP(hipMalloc(&net->e64, sizeof(double) * n));
        OFDFT_CHECK_HIP(hipMalloc(&net->ae64, sizeof(double) * n));
        net->e_cap = (size_t)n;
    }
    // denominator up to the tscale^2 factor: kind 1 phi^T A phi, kind 2 |A phi|^2
    const bool res = net->loss_kind == 2;
    OFDFT_TRY(fd_laplacian_apply(&g, 6, OFDFT_F64, phi, net->ae64, -h2, 0.0, s));
    if (res) OFDFT_TRY((launch_reduce<1>(n, SqOp{net->ae64}, StoreTotals<1>{net->totals + 1}, net->rb, s)));
    else OFDFT_TRY((launch_reduce<1>(n, DotOp{phi, net->ae64}, StoreTotals<1>{net->totals + 1}, net->rb, s)));
    OFDFT_TRY(forward(net, s));
    OFDFT_TRY((launch_reduce<1>(n, EnergyErrOp{net->out, phi, net->e64, net->totals, 1.0 / n, h2, 0},
                                NoFin{}, net->rb, s)));
    OFDFT_TRY(fd_laplacian_apply(&g, 6, OFDFT_F64, net->e64, net->ae64, -h2, 0.0, s));
    if (res) {     // e <- A (A e): numerator |A e|^2, gradient 2 A A e / den
        OFDFT_TRY(fd_laplacian_apply(&g, 6, OFDFT_F64, net->ae64, net->e64, -h2, 0.0, s));
        return energy_loss(net, n, net->ae64, net->ae64, net->e64, h2, s);
    }
    return energy_loss(net, n, net->e64, net->ae64, net->ae64, h2, s);
}

// One training step on a pair (g, phi): loss (kind set by ofdft_nn_set_loss)
// of N(g / rms g) against t = phi / (h^2 rms g), backward pass, Adam update
// (lr; beta1 0.9, beta2 0.999, eps 1e-8).
// loss (host, optional) receives the loss before the update.
extern "C" int ofdft_nn_train_step(ofdft_nn *net, const ofdft_grid *grid, const double *g_rhs,
                                   const double *phi, double lr, double *loss, void *stream) {
    if (!net || !g_rhs || !phi) return OFDFT_INVALID_ARG;
    OFDFT_TRY(check_grid(grid, 1));
    OFDFT_TRY(net_reserve(net, *grid));
    hipStream_t s = (hipStream_t)stream;
    const ofdft_grid &g = *grid;
    const int64_t n = npoints(g);
    const double h2 = std::cbrt(g.hx * g.hy * g.hz) * std::cbrt(g.hx * g.hy * g.hz);
    OFDFT_TRY((launch_reduce<1>(n, SqOp{g_rhs}, StoreTotals<1>{net->totals}, net->rb, s)));
    OFDFT_TRY(cast_input(net, n, g_rhs, s));
    OFDFT_TRY(loss_pass(net, g, phi, h2, s));
    OFDFT_TRY(backward(net, s));
    net->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)net->adam_t), c2 = 1.f - std::pow(b2, (float)net->adam_t);
    for (int l = 0; l < kLayers; ++l) {
        LayerPtrs L{net->w[l], net->m[l], net->v[l], net->gr[l], net->wf[l], net->wb[l], kDefs[l].cin,
                    kDefs[l].cout, ntile(kDefs[l].cout), ntile(kDefs[l].cin)};
        hipLaunchKernelGGL(adam_kernel, dim3(64), dim3(256), 0, s, L, (float)lr, b1, b2, c1, c2, 1e-8f);
        OFDFT_CHECK_HIP(hipGetLastError());
    }
    OFDFT_TRY(pack_all(net, s));
    if (loss) {
        double t[4];
        OFDFT_CHECK_HIP(hipMemcpyAsync(t, net->totals, sizeof(double) * 4, hipMemcpyDeviceToHost, s));
        OFDFT_CHECK_HIP(hipStreamSynchronize(s));
        const double rms = std::sqrt(t[0] / n);
        const double ts = rms > 0 ? 1.0 / (h2 * rms) : 0.0;
        *loss = t[2] / (t[1] * ts * ts);
    }
    return OFDFT_OK;
}

// Gradients only (no update), for checking against the reference: loss as in
// ofdft_nn_train_step, gradients readable with ofdft_nn_get_weights(..., 1).
extern "C" int ofdft_nn_gradients(ofdft_nn *net, const ofdft_grid *grid, const double *g_rhs,
                                  const double *phi, double *loss, void *stream) {
    if (!net || !g_rhs || !phi) return OFDFT_INVALID_ARG;
    OFDFT_TRY(check_grid(grid, 1));
    OFDFT_TRY(net_reserve(net, *grid));
    hipStream_t s = (hipStream_t)stream;
    const ofdft_grid &g = *grid;
    const int64_t n = npoints(g);
    const double h2 = std::cbrt(g.hx * g.hy * g.hz) * std::cbrt(g.hx * g.hy * g.hz);
    OFDFT_TRY((launch_reduce<1>(n, SqOp{g_rhs}, StoreTotals<1>{net->totals}, net->rb, s)));
    OFDFT_TRY(cast_input(net, n, g_rhs, s));
    OFDFT_TRY(loss_pass(net, g, phi, h2, s));
    OFDFT_TRY(backward(net, s));
    double t[4];
    OFDFT_CHECK_HIP(hipMemcpyAsync(t, net->totals, sizeof(double) * 4, hipMemcpyDeviceToHost, s));
    OFDFT_CHECK_HIP(hipStreamSynchronize(s));
    if (loss) {
        const double rms = std::sqrt(t[0] / n);
        const double ts = rms > 0 ? 1.0 / (h2 * rms) : 0.0;
        *loss = t[2] / (t[1] * ts * ts);
    }
    return OFDFT_OK;
}
