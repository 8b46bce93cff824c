// The periodic order-12 star-stencil core used by every kernel that applies
// the FD Laplacian (Section 4, FD Laplacian equation, with periodic images).
//
// Design for gfx950 (memory-bound, no MFMA):
//  * A workgroup owns a TX x (TYT*RY) tile of an xy-plane and marches along z
//    over a chunk of planes.  Each thread owns one x column and RY
//    consecutive y rows.
//  * z-neighbours come from a per-thread register ring of A + R + 1 planes,
//    filled by one coalesced load per point per plane (the queue front,
//    fetched A = R + 3 planes ahead of the output plane: 16 slots).  The z
//    loop is unrolled by the ring's period, so every ring index is a
//    constant: loads land in the register that holds the plane until it is
//    consumed, with no register copies, and the compiler waits only for the
//    plane being used, never for the younger prefetches (a shifting queue
//    makes it copy fresh loads at the loop latch, which drains every load in
//    flight).
//  * x- and y-neighbours come from an LDS copy of the current plane with a
//    6-wide halo: the tile centre is written from the queue, only the halo
//    ring is fetched from global memory.  The ring of a plane is fetched at
//    the same time as the neighbouring tiles (same XCD, launched together)
//    fetch that plane as their queue front, so it is served by L2, and
//    waits in an LDS slot until the plane is computed.
//  * y-register blocking: a thread reads RY+12 column values once and uses
//    them for its RY outputs.
//  * Periodic wrap: all wrapped x/y offsets are computed once per thread
//    before the z loop; the plane index wraps with one compare per plane.
//  * Loads and stores go through functors so that CG/COCG/H*u variants fuse
//    their vector updates and dot products into the stencil pass.
#pragma once

#include "common.hpp"
#include "profile.hpp"

#include <type_traits>

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
// and the register z ring; calls the epilogue for the valid owned points.
// Ring slot (J + R + d) mod NB holds plane k + d of output plane k.
template <typename T, int TX, int TYT, int RY, int NB, int J, class Epi>
__device__ __forceinline__ void stencil_plane_compute(const Coef<typename VT<T>::S> &w, const T *buf,
                                                      const T (&q)[NB][RY], const TileCtx<TX, TYT, RY> &tc,
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
        const T c = q[(J + R) % NB][r];
        T sacc = V::mul(w.c0, c);
        const T *row = buf + (ty * RY + r + R) * W + tx + R;
#pragma unroll
        for (int p = 1; p <= R; ++p) {
            sacc = V::fma(w.wx[p], V::add(row[p], row[-p]), sacc);
            sacc = V::fma(w.wy[p], V::add(col[r + R + p], col[r + R - p]), sacc);
            sacc = V::fma(w.wz[p], V::add(q[(J + R + p) % NB][r], q[(J + R - p + NB) % NB][r]), sacc);
        }
        if (tc.xvalid && tc.yvalid[r]) ep.point(r, pk + tc.own[r], c, sacc);
    }
}

// Compile-time loops: f(std::integral_constant<int, I>) for I = B .. E - 1;
// the _while form stops at the first call that returns false.
template <int I, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < E) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, E>(f);
    }
}
template <int I, int E, class F>
__device__ __forceinline__ void static_for_while(F &&f) {
    if constexpr (I < E) {
        if (f(std::integral_constant<int, I>{})) static_for_while<I + 1, E>(f);
    }
}

// LDS plan of a tile shape and element type.  The halo ring of plane P is
// fetched L planes before P is computed and parked in one of L plane buffers
// (slot (P - zb) mod L) until then; the centre is written from the z ring at
// P.  L = R + 3 fetches the ring together with the queue front of plane P,
// i.e. when the tiles around this one fetch P's centre, so that the halo
// reads hit in L2.  L is the largest value up to R + 3 whose buffers fit in
// 150 KiB (at least 2: a plain double buffer).
//
// Ring fetches wait in kRingDepth register buffers before going to LDS, so
// the ring of plane P is fetched L - 2 + kRingDepth planes ahead and the
// queue front R + 3 planes ahead: a depth of
// R + 5 - L (2..4) keeps the two fetches of a plane close together when
// fewer than R + 3 LDS slots fit.
template <typename T, int TX, int TYT, int RY>
struct StencilLds {
    using TS = TileShape<TX, TYT, RY>;
    static constexpr int kPlane = TS::W * TS::H + 1;
    static constexpr int kFit = (int)((150 * 1024) / ((size_t)kPlane * sizeof(T)));
    static_assert(kFit >= 2, "tile too large for a double-buffered LDS plane");
    static constexpr int kLead = kFit > kMaxRadius + 3 ? kMaxRadius + 3 : kFit;
    static constexpr int kElems = kLead * kPlane;
    static constexpr int kDepthWanted = kMaxRadius + 5 - kLead;
    static constexpr int kRingDepth = kDepthWanted <= 2 ? 2 : 4;
};

// One tile: march the z chunk, calling the epilogue for every owned point.
// `lds` holds L plane buffers of W*H + 1 elements (the last element of each
// is a dummy target for spare ring slots).
//
// Timeline of output plane k: write the ring slot of plane k into LDS slot(k)
// and the halo ring fetched PR planes ago (plane k + L - 2) into
// slot(k + L - 2); issue the epilogue's loads for plane k, then the fetches
// of halo ring k + L - 2 + PR and of queue front k + A (into the register
// slot that plane k - R - 1 has just left); barrier; compute plane k.  An LDS
// slot is rewritten two planes after its last reader, so one barrier per
// plane suffices.  The z ring has NB = A + R + 1 register slots and the loop
// is unrolled by lcm(NB, PR) planes, so that all register slots are
// constants; the last, partial step of a chunk stops at its end.  A queue
// front is first used A - R planes after its fetch, a halo ring PR planes
// after.  Halo fetches past the chunk end are clamped to its last plane
// (never used, an L2 hit).
//
// The geometry and the weights are taken by value, so they live in scalar
// registers for the whole march.  A reference into device memory (a field of
// a per-system descriptor) would be re-read after every store of the
// epilogue, since the stores may alias it; that re-read is a vector load, and
// waiting for it means waiting for every prefetch issued before it, which
// empties the z queue once per plane.
constexpr int gcd_i(int a, int b) { return b == 0 ? a : gcd_i(b, a % b); }

template <typename T, int TX, int TYT, int RY, class Load, class Epi,
          int L = StencilLds<T, TX, TYT, RY>::kLead, int PR = StencilLds<T, TX, TYT, RY>::kRingDepth,
          int A = kMaxRadius + 3>
__device__ inline void stencil_tile(const TileGeom g, const Coef<typename VT<T>::S> w,
                                    const Load &ld, Epi &ep, int logical_block, T *lds) {
    using TS = TileShape<TX, TYT, RY>;
    constexpr int R = TS::R, W = TS::W, H = TS::H;
    constexpr int SL = W * H + 1;
    // queue lead A: plane k + A is fetched at output plane k
    constexpr int NB = A + R + 1;           // register slots of the z ring
    constexpr int U = NB / gcd_i(NB, PR) * PR;   // unrolled planes: cycles ring and halo buffers
    static_assert(L >= 2 && L <= R + 3, "ring lead out of range");
    static_assert(PR >= 2 && PR <= 8, "halo register depth");
    static_assert(A > R, "the queue front must lead the stencil reach");
    const TileCtx<TX, TYT, RY> tc(g, logical_block);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int zb = tc.zb, ze = tc.ze;
    const int zlast = ze - 1;
    const int64_t nxy = (int64_t)g.nx * g.ny;

    // z ring: slot (P - zb + R) mod NB holds plane P; planes zb - R .. zb + A - 1 first
    T q[NB][RY];
#pragma unroll
    for (int j = 0; j < A + R; ++j) {
        const int64_t pb = (int64_t)wrapi(zb - R + j, g.nz) * nxy;
#pragma unroll
        for (int r = 0; r < RY; ++r) q[j][r] = ld(pb + tc.own[r]);
    }
    // halo rings of planes zb .. zb + L - 3 go straight to their slots
#pragma unroll
    for (int j = 0; j < L - 2; ++j) {
        const int64_t pb = (int64_t)min(zb + j, zlast) * nxy;
        T *slot = lds + j * SL;
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i) slot[tc.ring_lds[i]] = ld(pb + tc.ring_glb[i]);
    }
    // halo rings of planes zb + L - 2 .. zb + L - 3 + PR in flight
    T ring[PR][TS::RING_PER_T];
#pragma unroll
    for (int j = 0; j < PR; ++j) {
        const int64_t rp = (int64_t)min(zb + L - 2 + j, zlast) * nxy;
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i) ring[j][i] = ld(rp + tc.ring_glb[i]);
    }
    int kr = zb + L - 2 + PR;              // plane of the next halo fetch (clamped at use)
    int kf = wrapi(zb + A, g.nz);          // plane of the next queue-front fetch
    int sc = 0;                            // LDS slot of the output plane

    auto plane = [&](int k, auto jc) __attribute__((always_inline)) {
        constexpr int J = decltype(jc)::value;
        const int64_t pk = (int64_t)k * nxy;
        T *buf = lds + sc * SL;
        const int sr = sc + L - 2 >= L ? sc - 2 : sc + L - 2;
        T *rbuf = lds + sr * SL;
        T (&rb)[TS::RING_PER_T] = ring[J % PR];
#pragma unroll
        for (int r = 0; r < RY; ++r) buf[(ty * RY + r + R) * W + tx + R] = q[(J + R) % NB][r];
#pragma unroll
        for (int i = 0; i < TS::RING_PER_T; ++i) rbuf[tc.ring_lds[i]] = rb[i];
#pragma unroll
        for (int r = 0; r < RY; ++r) ep.pre(r, pk + tc.own[r]);
        {
            const int64_t pr = (int64_t)min(kr, zlast) * nxy, pf = (int64_t)kf * nxy;
#pragma unroll
            for (int i = 0; i < TS::RING_PER_T; ++i) rb[i] = ld(pr + tc.ring_glb[i]);
#pragma unroll
            for (int r = 0; r < RY; ++r) q[(J + NB - 1) % NB][r] = ld(pf + tc.own[r]);
        }
        __syncthreads();
        stencil_plane_compute<T, TX, TYT, RY, NB, J>(w, buf, q, tc, pk, ep);
        ++kr;
        kf = (kf + 1 == g.nz) ? 0 : kf + 1;
        sc = (sc + 1 == L) ? 0 : sc + 1;
    };

    int k0 = zb;
    for (; k0 + U <= ze; k0 += U)
        static_for<0, U>([&](auto jc) __attribute__((always_inline)) { plane(k0 + decltype(jc)::value, jc); });
    if (k0 < ze)
        static_for_while<0, U>([&](auto jc) __attribute__((always_inline)) {
            const int k = k0 + decltype(jc)::value;
            if (k >= ze) return false;
            plane(k, jc);
            return true;
        });
    // the LDS buffers are reused by the next tile of a persistent caller
    __syncthreads();
}

// Epilogues may read per-launch scalars from device memory in prepare().
template <class E>
__device__ inline auto epi_prepare(E &e, int) -> decltype(e.prepare(), void()) {
    e.prepare();
}
template <class E>
__device__ inline void epi_prepare(E &, long) {}

// Plain kernel wrapper: one tile per workgroup, XCD-aware tile order, then the
// epilogue's block-level finish (reductions).
template <typename T, int TX, int TYT, int RY, class Load, class Epi>
__global__ void __launch_bounds__(TX * TYT)
stencil_kernel(TileGeom g, Coef<typename VT<T>::S> w, Load ld, Epi ep) {
    __shared__ T lds[StencilLds<T, TX, TYT, RY>::kElems];
    __shared__ double red_scratch[64];
    if (ep.skip()) return;
    ld.prepare();
    epi_prepare(ep, 0);
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
