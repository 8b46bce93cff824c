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

// Loader: T operator()(int64_t idx) const -- value of the operand at idx
//   (branch-free, so that the prefetched loads stay in flight).
// Epilogue: pre(r, idx) loads the per-point operands of owned row r of the
//   current plane (issued before the prefetches, so waiting for them does not
//   drain the pipeline); point(r, idx, centre, lap) for every valid owned
//   point; finish(block, nblocks, scratch) once per workgroup.

// Per-thread placement inside a tile: owned points and halo ring cells.
template <int TX, int TYT, int RY>
struct TileCtx {
    using TS = TileShape<TX, TYT, RY>;
    int zb, ze;
    bool xvalid;
    int own[RY];
    bool yvalid[RY];
    int ring_lds[TS::RING_PER_T], ring_glb[TS::RING_PER_T];

    __device__ TileCtx(const TileGeom &g, int logical_block) {
        constexpr int R = TS::R, W = TS::W, H = TS::H, TY = TS::TY;
        const int tx = threadIdx.x, ty = threadIdx.y;
        const int tid = ty * TX + tx;
        int b = logical_block;
        const int bxi = b % g.tiles_x;
        b /= g.tiles_x;
        const int byi = b % g.tiles_y;
        const int zc = b / g.tiles_y;
        const int x0 = bxi * TX, y0 = byi * TY;
        zb = zc * g.zlen;
        ze = min(zb + g.zlen, g.nz);
        // Owned points: x = x0 + tx, rows y0 + ty*RY + r.
        const int xo = x0 + tx;
        xvalid = xo < g.nx;
        const int gx = xo % g.nx;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int yo = y0 + ty * RY + r;
            yvalid[r] = yo < g.ny;
            own[r] = (yo % g.ny) * g.nx + gx;
        }
        // Halo ring cells handled by this thread: LDS cell and wrapped xy offset.
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
            } else {                                  // spare slot: harmless load, dummy LDS cell
                ring_lds[i] = W * H;
                ring_glb[i] = own[0];
            }
        }
    }
};

// Stencil arithmetic of one plane from an LDS plane buffer (centre + halo)
// and the register z queue; calls the epilogue for the valid owned points.
template <typename T, int TX, int TYT, int RY, class Epi>
__device__ inline void stencil_plane_compute(const Coef<typename VT<T>::S> &w, const T *buf,
                                             const T (&q)[2 * kMaxRadius + 1][RY],
                                             const TileCtx<TX, TYT, RY> &tc, bool active,
                                             int64_t pk, Epi &ep) {
    using V = VT<T>;
    using TS = TileShape<TX, TYT, RY>;
    constexpr int R = TS::R, W = TS::W;
    const int tx = threadIdx.x, ty = threadIdx.y;
    // y column values of this thread's x, rows ty*RY - R .. ty*RY + RY - 1 + R
    T col[RY + 2 * R];
#pragma unroll
    for (int j = 0; j < RY + 2 * R; ++j) col[j] = buf[(ty * RY + j) * W + tx + R];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const T c = q[R][r];
        T sacc = V::mul(w.c0, c);
        const T *row = buf + (ty * RY + r + R) * W + tx + R;
#pragma unroll
        for (int p = 1; p <= R; ++p) {
            sacc = V::fma(w.wx[p], V::add(row[p], row[-p]), sacc);
            sacc = V::fma(w.wy[p], V::add(col[r + R + p], col[r + R - p]), sacc);
            sacc = V::fma(w.wz[p], V::add(q[R + p][r], q[R - p][r]), sacc);
        }
        if (active && tc.xvalid && tc.yvalid[r]) ep.point(r, pk + tc.own[r], c, sacc);
    }
}

// Two-buffer form (used where LDS is scarce: complex128 tiles and the
// persistent COCG kernel).  `lds` holds 2 * (W*H + 1) elements.
template <typename T, int TX, int TYT, int RY, class Load, class Epi>
__device__ inline void stencil_tile(const TileGeom &g, const Coef<typename VT<T>::S> &w,
                                    const Load &ld, Epi &ep, int logical_block, T *lds) {
    using TS = TileShape<TX, TYT, RY>;
    constexpr int R = TS::R, W = TS::W, H = TS::H;
    const TileCtx<TX, TYT, RY> tc(g, logical_block);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int zb = tc.zb, ze = tc.ze;
    const int64_t nxy = (int64_t)g.nx * g.ny;

    // z queue: q[j][r] holds plane (k - R + j) for output plane k.
    T q[2 * R + 1][RY];
#pragma unroll
    for (int j = 0; j < 2 * R + 1; ++j) {
        const int64_t pb = (int64_t)wrapi(zb - R + j, g.nz) * nxy;
#pragma unroll
        for (int r = 0; r < RY; ++r) q[j][r] = ld(pb + tc.own[r]);
    }
    // Software pipeline: the halo ring is fetched two planes ahead and the
    // queue front (plane k + R + 1) two planes ahead of its use, so each
    // plane's global loads overlap two planes of compute.
    T ringA[TS::RING_PER_T], ringB[TS::RING_PER_T];
    {
        const int64_t p0 = (int64_t)zb * nxy, p1 = (int64_t)wrapi(zb + 1, g.nz) * nxy;
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i) {
            ringA[i] = ld(p0 + tc.ring_glb[i]);
            ringB[i] = ld(p1 + tc.ring_glb[i]);
        }
    }
    T qn1[RY], qn2[RY];
    {
        const int64_t f1 = (int64_t)wrapi(zb + R + 1, g.nz) * nxy;
        const int64_t f2 = (int64_t)wrapi(zb + R + 2, g.nz) * nxy;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            qn1[r] = ld(f1 + tc.own[r]);
            qn2[r] = ld(f2 + tc.own[r]);
        }
    }
    int kr = wrapi(zb + 2, g.nz);          // plane of the next ring prefetch
    int kf = wrapi(zb + R + 3, g.nz);      // plane of the next queue-front prefetch

    // One plane.  `ring`/`qn` hold loads issued two planes earlier; they are
    // consumed and then refilled in place (no register rotation of in-flight
    // loads, so the waits only cover old loads).  `active` is false for the
    // padding plane of an odd-length chunk: it still loads (in bounds) but
    // stores nothing.
    auto plane = [&](int k, T (&ring)[TS::RING_PER_T], T (&qn)[RY], bool active, int parity) {
        const int kk = active ? k : zb;
        const int64_t pk = (int64_t)kk * nxy;
        T *buf = lds + parity * (W * H + 1);
#pragma unroll
        for (int r = 0; r < RY; ++r) buf[(ty * RY + r + R) * W + tx + R] = q[R][r];
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i) buf[tc.ring_lds[i]] = ring[i];
        // epilogue operands of this plane first, then the prefetches
#pragma unroll
        for (int r = 0; r < RY; ++r) ep.pre(r, pk + tc.own[r]);
        T nxt[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) nxt[r] = qn[r];
        {
            const int64_t pr = (int64_t)kr * nxy, pf = (int64_t)kf * nxy;
#pragma unroll
            for (int i = 0; i < TS::RING_PER_T; ++i) ring[i] = ld(pr + tc.ring_glb[i]);
#pragma unroll
            for (int r = 0; r < RY; ++r) qn[r] = ld(pf + tc.own[r]);
        }
        __syncthreads();
        stencil_plane_compute<T, TX, TYT, RY>(w, buf, q, tc, active, pk, ep);
#pragma unroll
        for (int j = 0; j < 2 * R; ++j)
#pragma unroll
            for (int r = 0; r < RY; ++r) q[j][r] = q[j + 1][r];
#pragma unroll
        for (int r = 0; r < RY; ++r) q[2 * R][r] = nxt[r];
        kr = (kr + 1 == g.nz) ? 0 : kr + 1;
        kf = (kf + 1 == g.nz) ? 0 : kf + 1;
    };

    for (int k = zb; k < ze; k += 2) {
        plane(k, ringA, qn1, true, 0);
        plane(k + 1, ringB, qn2, k + 1 < ze, 1);
    }
    // the LDS buffers are reused by the next tile of a persistent caller
    __syncthreads();
}

// Slot form: the halo ring of plane P is fetched together with the queue
// front of plane P (R + 3 planes before P is computed), i.e. at the moment
// the tiles around it fetch P's centre, so that the halo reads hit L2 while
// the neighbours' lines are fresh.  The ring waits in one of kDeepSlots LDS
// plane buffers: plane P uses slot (P - zb) mod kDeepSlots; the ring is
// written R + 1 planes ahead and the centre at P, before P's barrier.  Nine
// slots keep the slot written at plane k clear of the slots still read at
// planes k - 1 and k.  Planes past the chunk end are never computed, so
// their ring fetches are clamped to the chunk's last plane (an L2 hit).
constexpr int kDeepSlots = kMaxRadius + 3;

template <typename T, int TX, int TYT, int RY, class Load, class Epi>
__device__ inline void stencil_tile_deep(const TileGeom &g, const Coef<typename VT<T>::S> &w,
                                         const Load &ld, Epi &ep, int logical_block, T *lds) {
    using TS = TileShape<TX, TYT, RY>;
    constexpr int R = TS::R, W = TS::W, H = TS::H;
    constexpr int SL = W * H + 1;
    const TileCtx<TX, TYT, RY> tc(g, logical_block);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int zb = tc.zb, ze = tc.ze;
    const int zlast = ze - 1;
    const int64_t nxy = (int64_t)g.nx * g.ny;

    T q[2 * R + 1][RY];
#pragma unroll
    for (int j = 0; j < 2 * R + 1; ++j) {
        const int64_t pb = (int64_t)wrapi(zb - R + j, g.nz) * nxy;
#pragma unroll
        for (int r = 0; r < RY; ++r) q[j][r] = ld(pb + tc.own[r]);
    }
    // rings of planes zb .. zb + R go straight to their slots
#pragma unroll
    for (int j = 0; j <= R; ++j) {
        const int64_t pb = (int64_t)min(zb + j, zlast) * nxy;
        T *slot = lds + j * SL;
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i) slot[tc.ring_lds[i]] = ld(pb + tc.ring_glb[i]);
    }
    // rings and queue fronts of planes zb + R + 1 and zb + R + 2 in flight
    T ringA[TS::RING_PER_T], ringB[TS::RING_PER_T];
    T qn1[RY], qn2[RY];
    {
        const int64_t r1 = (int64_t)min(zb + R + 1, zlast) * nxy;
        const int64_t r2 = (int64_t)min(zb + R + 2, zlast) * nxy;
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i) {
            ringA[i] = ld(r1 + tc.ring_glb[i]);
            ringB[i] = ld(r2 + tc.ring_glb[i]);
        }
        const int64_t f1 = (int64_t)wrapi(zb + R + 1, g.nz) * nxy;
        const int64_t f2 = (int64_t)wrapi(zb + R + 2, g.nz) * nxy;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            qn1[r] = ld(f1 + tc.own[r]);
            qn2[r] = ld(f2 + tc.own[r]);
        }
    }
    int kr = zb + R + 3;                   // plane of the next ring fetch (clamped at use)
    int kf = wrapi(zb + R + 3, g.nz);      // plane of the next queue-front fetch
    int sc = 0;                            // slot of the output plane

    auto plane = [&](int k, T (&ring)[TS::RING_PER_T], T (&qn)[RY], bool active) {
        const int kk = active ? k : zb;
        const int64_t pk = (int64_t)kk * nxy;
        T *buf = lds + sc * SL;
        const int sr = sc + R + 1 >= kDeepSlots ? sc + R + 1 - kDeepSlots : sc + R + 1;
        T *rbuf = lds + sr * SL;
#pragma unroll
        for (int r = 0; r < RY; ++r) buf[(ty * RY + r + R) * W + tx + R] = q[R][r];
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i) rbuf[tc.ring_lds[i]] = ring[i];
#pragma unroll
        for (int r = 0; r < RY; ++r) ep.pre(r, pk + tc.own[r]);
        T nxt[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) nxt[r] = qn[r];
        {
            const int64_t pr = (int64_t)min(kr, zlast) * nxy, pf = (int64_t)kf * nxy;
#pragma unroll
            for (int i = 0; i < TS::RING_PER_T; ++i) ring[i] = ld(pr + tc.ring_glb[i]);
#pragma unroll
            for (int r = 0; r < RY; ++r) qn[r] = ld(pf + tc.own[r]);
        }
        __syncthreads();
        stencil_plane_compute<T, TX, TYT, RY>(w, buf, q, tc, active, pk, ep);
#pragma unroll
        for (int j = 0; j < 2 * R; ++j)
#pragma unroll
            for (int r = 0; r < RY; ++r) q[j][r] = q[j + 1][r];
#pragma unroll
        for (int r = 0; r < RY; ++r) q[2 * R][r] = nxt[r];
        ++kr;
        kf = (kf + 1 == g.nz) ? 0 : kf + 1;
        sc = (sc + 1 == kDeepSlots) ? 0 : sc + 1;
    };

    for (int k = zb; k < ze; k += 2) {
        plane(k, ringA, qn1, true);
        plane(k + 1, ringB, qn2, k + 1 < ze);
    }
    __syncthreads();
}

// LDS plan of a tile shape and element type: the slot form where nine plane
// buffers fit in 150 KiB, otherwise the two-buffer form.
template <typename T, int TX, int TYT, int RY>
struct StencilLds {
    using TS = TileShape<TX, TYT, RY>;
    static constexpr int kPlane = TS::W * TS::H + 1;
    static constexpr bool kDeep = (size_t)kDeepSlots * kPlane * sizeof(T) <= 150 * 1024;
    static constexpr int kElems = (kDeep ? kDeepSlots : 2) * kPlane;
};

// Plain kernel wrapper: one tile per workgroup, XCD-aware tile order, then the
// epilogue's block-level finish (reductions).
template <typename T, int TX, int TYT, int RY, class Load, class Epi>
__global__ void __launch_bounds__(TX * TYT)
stencil_kernel(TileGeom g, Coef<typename VT<T>::S> w, Load ld, Epi ep) {
    using SL = StencilLds<T, TX, TYT, RY>;
    __shared__ T lds[SL::kElems];
    __shared__ double red_scratch[64];
    if (ep.skip()) return;
    ld.prepare();
    const int lb = xcd_remap(blockIdx.x, g.nblocks);
    if constexpr (SL::kDeep)
        stencil_tile_deep<T, TX, TYT, RY>(g, w, ld, ep, lb, lds);
    else
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

template <typename T, bool ReadY>
struct EpiAxpby {        // y = alpha * L x + beta * y  (ReadY: beta != 0)
    T *__restrict__ y;
    typename VT<T>::S alpha, beta;
    T yold[4];
    __device__ bool skip() const { return false; }
    __device__ void pre(int r, int64_t i) {
        if constexpr (ReadY) yold[r] = y[i];
    }
    __device__ void point(int r, int64_t i, T, T s) {
        using V = VT<T>;
        T v = V::mul(alpha, s);
        if constexpr (ReadY) v = V::fma(beta, yold[r], v);
        y[i] = v;
    }
    __device__ void finish(int, int, double *) {}
};

}  // namespace ofdft
