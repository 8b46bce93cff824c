// The periodic order-12 star-stencil core used by every kernel that applies
// the FD Laplacian (Section 4, FD Laplacian equation, with periodic images).
//
// Design for gfx950 (memory-bound, no MFMA):
//  * A workgroup owns a TX x (TYT*RY) tile of an xy-plane and marches along z
//    over a chunk of planes.  Each thread owns one x column and RY
//    consecutive y rows.
//  * z-neighbours come from a per-thread register queue of 13 planes, filled
//    by one coalesced load per point per plane (the queue front, 7 planes
//    ahead of the output plane).
//  * x- and y-neighbours come from an LDS copy of the current plane with a
//    6-wide halo: the tile centre is written from the queue, only the halo
//    ring is fetched from global memory (mostly L2/MALL hits, since the
//    neighbouring tiles stream the same planes on the same XCD).
//  * y-register blocking: a thread reads RY+12 column values once and uses
//    them for its RY outputs.
//  * Periodic wrap: all wrapped x/y offsets are computed once per thread
//    before the z loop; the plane index wraps with one compare per plane.
//  * Loads and stores go through functors so that CG/COCG/H*u variants fuse
//    their vector updates and dot products into the stencil pass.
#pragma once

#include "common.hpp"
#include "profile.hpp"

namespace ofdft {

struct TileGeom {
    int nx, ny, nz;
    int tiles_x, tiles_y, zchunks, zlen;
    int nblocks;
};

template <int TX, int TYT, int RY>
struct TileShape {
    static constexpr int R = kMaxRadius;
    static constexpr int TY = TYT * RY;
    static constexpr int W = TX + 2 * R;
    static constexpr int H = TY + 2 * R;
    static constexpr int NT = TX * TYT;
    static constexpr int NRING = W * H - TX * TY;
    static constexpr int RING_PER_T = (NRING + NT - 1) / NT;
};

template <int TX, int TYT, int RY>
inline TileGeom make_tile_geom(const ofdft_grid &g, int zlen) {
    using TS = TileShape<TX, TYT, RY>;
    TileGeom t;
    t.nx = g.nx;
    t.ny = g.ny;
    t.nz = g.nz;
    t.tiles_x = (g.nx + TX - 1) / TX;
    t.tiles_y = (g.ny + TS::TY - 1) / TS::TY;
    if (zlen <= 0 || zlen > g.nz) zlen = g.nz;
    t.zlen = zlen;
    t.zchunks = (g.nz + zlen - 1) / zlen;
    t.nblocks = t.tiles_x * t.tiles_y * t.zchunks;
    return t;
}

__device__ inline int wrapi(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Loader: T operator()(int64_t idx) const -- value of the operand at idx.
// Epilogue: void point(int64_t idx, T centre, T lap) for every owned output
//   point (only valid points are passed), then finish(block, scratch) once.
template <typename T, int TX, int TYT, int RY, class Load, class Epi>
__device__ inline void stencil_tile(const TileGeom &g, const Coef<typename VT<T>::S> &w,
                                    const Load &ld, Epi &ep, int logical_block, T *lds) {
    using V = VT<T>;
    using TS = TileShape<TX, TYT, RY>;
    constexpr int R = TS::R, W = TS::W, H = TS::H, TY = TS::TY;

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;
    int b = logical_block;
    const int bxi = b % g.tiles_x;
    b /= g.tiles_x;
    const int byi = b % g.tiles_y;
    const int zc = b / g.tiles_y;
    const int x0 = bxi * TX, y0 = byi * TY;
    const int zb = zc * g.zlen;
    const int ze = min(zb + g.zlen, g.nz);
    const int64_t nxy = (int64_t)g.nx * g.ny;

    // Owned points: x = x0 + tx, rows y0 + ty*RY + r.
    const int xo = x0 + tx;
    const bool xvalid = xo < g.nx;
    const int gx = xo % g.nx;
    int own[RY];
    bool yvalid[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int yo = y0 + ty * RY + r;
        yvalid[r] = yo < g.ny;
        own[r] = (yo % g.ny) * g.nx + gx;
    }

    // Halo ring cells handled by this thread: LDS slot and wrapped xy offset.
    int ring_lds[TS::RING_PER_T], ring_glb[TS::RING_PER_T];
#pragma unroll
    for (int i = 0; i < TS::RING_PER_T; ++i) {
        const int c = tid + i * TS::NT;
        int lx = 0, ly = 0;
        if (c < TS::NRING) {
            if (c < R * W) {                      // top band
                ly = c / W;
                lx = c % W;
            } else if (c < 2 * R * W) {           // bottom band
                const int cc = c - R * W;
                ly = H - R + cc / W;
                lx = cc % W;
            } else {                              // left / right strips
                const int cc = c - 2 * R * W;
                ly = R + cc / (2 * R);
                const int s = cc % (2 * R);
                lx = s < R ? s : TX + s;
            }
            ring_lds[i] = ly * W + lx;
            ring_glb[i] = wrapi(y0 - R + ly, g.ny) * g.nx + wrapi(x0 - R + lx, g.nx);
        } else {
            ring_lds[i] = -1;
            ring_glb[i] = 0;
        }
    }

    // z queue: q[j][r] holds plane (k - R + j) for output plane k.
    T q[2 * R + 1][RY];
#pragma unroll
    for (int j = 0; j < 2 * R + 1; ++j) {
        const int64_t pb = (int64_t)wrapi(zb - R + j, g.nz) * nxy;
#pragma unroll
        for (int r = 0; r < RY; ++r) q[j][r] = ld(pb + own[r]);
    }

    int kf = wrapi(zb + R + 1, g.nz);   // plane index of the next queue front
    for (int k = zb; k < ze; ++k) {
        const int64_t pk = (int64_t)k * nxy;
        // prefetch the next queue front and this plane's halo ring
        T nxt[RY];
        const int64_t pf = (int64_t)kf * nxy;
#pragma unroll
        for (int r = 0; r < RY; ++r) nxt[r] = ld(pf + own[r]);
        T ring[TS::RING_PER_T];
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i)
            ring[i] = ring_lds[i] >= 0 ? ld(pk + ring_glb[i]) : V::zero();

#pragma unroll
        for (int r = 0; r < RY; ++r) lds[(ty * RY + r + R) * W + tx + R] = q[R][r];
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i)
            if (ring_lds[i] >= 0) lds[ring_lds[i]] = ring[i];
        __syncthreads();

        // y column values of this thread's x, rows ty*RY - R .. ty*RY + RY - 1 + R
        T col[RY + 2 * R];
#pragma unroll
        for (int j = 0; j < RY + 2 * R; ++j) col[j] = lds[(ty * RY + j) * W + tx + R];

#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const T c = q[R][r];
            T s = V::mul(w.c0, c);
            const T *row = lds + (ty * RY + r + R) * W + tx + R;
#pragma unroll
            for (int p = 1; p <= R; ++p) {
                s = V::fma(w.wx[p], V::add(row[p], row[-p]), s);
                s = V::fma(w.wy[p], V::add(col[r + R + p], col[r + R - p]), s);
                s = V::fma(w.wz[p], V::add(q[R + p][r], q[R - p][r]), s);
            }
            if (xvalid && yvalid[r]) ep.point(pk + own[r], c, s);
        }
        __syncthreads();

#pragma unroll
        for (int j = 0; j < 2 * R; ++j)
#pragma unroll
            for (int r = 0; r < RY; ++r) q[j][r] = q[j + 1][r];
#pragma unroll
        for (int r = 0; r < RY; ++r) q[2 * R][r] = nxt[r];
        kf = (kf + 1 == g.nz) ? 0 : kf + 1;
    }
}

// Plain kernel wrapper: one tile per workgroup, XCD-aware tile order, then the
// epilogue's block-level finish (reductions).
template <typename T, int TX, int TYT, int RY, class Load, class Epi>
__global__ void __launch_bounds__(TX * TYT)
stencil_kernel(TileGeom g, Coef<typename VT<T>::S> w, Load ld, Epi ep) {
    using TS = TileShape<TX, TYT, RY>;
    __shared__ T lds[TS::W * TS::H];
    __shared__ double red_scratch[64];
    if (ep.skip()) return;
    ld.prepare();
    const int lb = xcd_remap(blockIdx.x, g.nblocks);
    stencil_tile<T, TX, TYT, RY>(g, w, ld, ep, lb, lds);
    ep.finish(blockIdx.x, g.nblocks, red_scratch);
}

// ---- plain loaders / epilogues -------------------------------------------
template <typename T>
struct LoadPlain {
    const T *__restrict__ x;
    __device__ void prepare() {}
    __device__ T operator()(int64_t i) const { return x[i]; }
};

template <typename T>
struct EpiAxpby {        // y = alpha * L x + beta * y
    T *__restrict__ y;
    typename VT<T>::S alpha, beta;
    __device__ bool skip() const { return false; }
    __device__ void point(int64_t i, T, T s) {
        using V = VT<T>;
        T v = V::mul(alpha, s);
        if (beta != typename VT<T>::S(0)) v = V::fma(beta, y[i], v);
        y[i] = v;
    }
    __device__ void finish(int, int, double *) {}
};

}  // namespace ofdft
