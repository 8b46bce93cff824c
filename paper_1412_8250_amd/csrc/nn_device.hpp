// Device kernels of the learned solver aid (included by nn_net.hip only).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "nn.hpp"
#include "profile.hpp"
#include "vec.hpp"

namespace ofdft {
namespace nn {

// Bricks of the convolution and weight-gradient kernels: 16 x 4 x 4 points,
// staged in LDS with a one-point halo.
constexpr int kWbX = 16, kWbY = 4, kWbZ = 4, kWbZg = 4;
constexpr int kWbTX = kWbX + 2, kWbTY = kWbY + 2, kWbTZ = kWbZ + 2;
constexpr int kWbHalo = kWbTX * kWbTY * kWbTZ;      // 648 points
constexpr int kWbPts = kWbX * kWbY * kWbZ;          // 256 points
constexpr int kWbStride = 20;                       // LDS elements per point (16 + pad: no bank conflicts)

__device__ inline int wrap_any(int i, int n) {
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------------------
// Convolution, C_in a multiple of 16.  Block = 4 waves, each 16 points.
// Weights Wt: [27][NTILE*16][Cin] (BF16, or FP32 in the FP32 mode; zero rows
// for co >= Cout).  Output: activation type A (with or without ReLU) or FP32
// (no ReLU), channels-last Cout.
//
// One 16-channel chunk of one tap is one v_mfma_f32_16x16x16 bf16 (lane
// (m, kq) supplies channels 4 kq .. 4 kq + 3 of point m and of output m) or,
// in the FP32 mode, four v_mfma_f32_16x16x4 f32 with the same loads: step j
// takes channel 4 kq + j from every lane, so its K = 4 values are channels
// j, 4 + j, 8 + j, 12 + j -- a permutation of the chunk's channels, applied
// to A and B alike.
template <int NTILE, typename A>
__global__ void __launch_bounds__(256)
conv_k16(InDescT<A> in, Geo g, const A *__restrict__ Wt, int cin, int cout, A *out_a,
         float *out_f32, int relu) {
    using V = typename Vec4<A>::type;
    using Raw = typename Vec4<A>::raw;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p0 = (blockIdx.x * 4 + wave) * 16;
    if (p0 >= g.npts) return;
    const int m = lane & 15, kq = lane >> 4;
    int p = p0 + m;
    if (p >= g.npts) p = p0;
    const int x = p % g.nx, y = (p / g.nx) % g.ny, z = p / (g.nx * g.ny);
    const int xs[3] = {wrapc(x - 1, g.nx), x, wrapc(x + 1, g.nx)};
    const int ys[3] = {wrapc(y - 1, g.ny), y, wrapc(y + 1, g.ny)};
    const int zs[3] = {wrapc(z - 1, g.nz), z, wrapc(z + 1, g.nz)};
    f32x4 acc[NTILE];
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    constexpr int CO = NTILE * 16;
    for (int t = 0; t < 27; ++t) {
        const int xx = xs[t % 3], yy = ys[(t / 3) % 3], zz = zs[t / 9];
        const A *wt = Wt + (size_t)t * CO * cin;
        for (int c0 = 0; c0 < cin; c0 += 16) {
            const V a = fetch4<A>(in, xx, yy, zz, c0 + 4 * kq, g);
#pragma unroll
            for (int nt = 0; nt < NTILE; ++nt) {
                const Raw raw = *reinterpret_cast<const Raw *>(wt + (size_t)(nt * 16 + m) * cin + c0 + 4 * kq);
                const V b = __builtin_bit_cast(V, raw);
                if constexpr (sizeof(A) == 2) {
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nt], 0, 0, 0);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], acc[nt], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt) {
        const int co = nt * 16 + m;
        if (co >= cout) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = p0 + 4 * kq + i;
            if (q >= g.npts) continue;
            float v = acc[nt][i];
            if (relu) v = fmaxf(v, 0.f);
            if (out_f32) out_f32[(size_t)q * cout + co] = v;
            else out_a[(size_t)q * cout + co] = Act<A>::from(v);
        }
    }
}

// Convolution on bricks, C_in a multiple of 16: one block (4 waves) owns a
// brick of 16 x 4 x 4 points and NTB output tiles of 16 channels (tile group
// blockIdx.y).  Per 16-channel input chunk the brick's input with its
// one-point halo (18 x 6 x 6 points) is staged in LDS once (periodic images,
// upsampled / concatenated / masked sources as in fetch4); then wave w runs
// the 27 taps over the 4 rows of brick plane z0 + w: per tap it loads the
// weights of its NTB tiles once (lane (m, kq): ci 4 kq .. 4 kq + 3 of output
// channel m) and, per row, the 16 points' shifted input (lane (m, kq): point
// m, channels 4 kq .. 4 kq + 3, one 8-byte LDS read) -- one MFMA K step per
// (tap, chunk, row, tile).  Each input value is read from memory once per
// brick and chunk instead of once per tap.  wgt layout as for conv_k16.
template <int NTB, typename A>
__global__ void __launch_bounds__(256)
conv_brick(InDescT<A> in, Geo g, const A *__restrict__ Wt, int cin, int cout, A *out_a, float *out_f32,
           int relu, int nbx, int nby) {
    using V = typename Vec4<A>::type;
    using Raw = typename Vec4<A>::raw;
    __shared__ __align__(16) A xs[kWbHalo * kWbStride];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, kq = lane >> 4;
    int b = blockIdx.x;
    const int bxi = b % nbx;
    b /= nbx;
    const int byi = b % nby;
    const int bzi = b / nby;
    const int x0 = bxi * kWbX, y0 = byi * kWbY, z0 = bzi * kWbZ;
    const int cop = ((cout + 15) / 16) * 16;          // padded rows of the weight layout
    const int cob = blockIdx.y * NTB * 16;            // first output channel of the block
    f32x4 acc[kWbY][NTB];
#pragma unroll
    for (int r = 0; r < kWbY; ++r)
#pragma unroll
        for (int nt = 0; nt < NTB; ++nt) acc[r][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < cin; c0 += 16) {
        __syncthreads();
        for (int e = tid; e < kWbHalo * 4; e += 256) {
            const int q = e >> 2, c4 = e & 3;
            const int lx = q % kWbTX, ly = (q / kWbTX) % kWbTY, lz = q / (kWbTX * kWbTY);
            const V v = fetch4<A>(in, wrap_any(x0 - 1 + lx, g.nx), wrap_any(y0 - 1 + ly, g.ny),
                                  wrap_any(z0 - 1 + lz, g.nz), c0 + 4 * c4, g);
            *reinterpret_cast<Raw *>(xs + q * kWbStride + 4 * c4) = __builtin_bit_cast(Raw, v);
        }
        __syncthreads();
        for (int t = 0; t < 27; ++t) {
            const int dx = t % 3, dyo = (t / 3) % 3, dz = t / 9;      // shift + 1
            const A *wt = Wt + ((size_t)t * cop + cob + m) * cin + c0 + 4 * kq;
            V bw[NTB];
#pragma unroll
            for (int nt = 0; nt < NTB; ++nt)
                bw[nt] = __builtin_bit_cast(V, *reinterpret_cast<const Raw *>(wt + (size_t)nt * 16 * cin));
#pragma unroll
            for (int r = 0; r < kWbY; ++r) {
                const A *xr = xs + (((wave + dz) * kWbTY + (r + dyo)) * kWbTX + m + dx) * kWbStride + 4 * kq;
                const V a = __builtin_bit_cast(V, *reinterpret_cast<const Raw *>(xr));
#pragma unroll
                for (int nt = 0; nt < NTB; ++nt) {
                    if constexpr (sizeof(A) == 2) {
                        acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[nt], acc[r][nt], 0, 0, 0);
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], bw[nt][j], acc[r][nt], 0, 0, 0);
                    }
                }
            }
        }
    }
    // lane holds D[point 4 kq + i][channel m] of each row and tile
    const int z = z0 + wave;
#pragma unroll
    for (int r = 0; r < kWbY; ++r) {
        const int y = y0 + r;
#pragma unroll
        for (int nt = 0; nt < NTB; ++nt) {
            const int co = cob + nt * 16 + m;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = x0 + 4 * kq + i;
                if (x >= g.nx || y >= g.ny || z >= g.nz || co >= cout) continue;
                const size_t q = (size_t)pidx(x, y, z, g);
                float v = acc[r][nt][i];
                if (relu) v = fmaxf(v, 0.f);
                if (out_f32) out_f32[q * cout + co] = v;
                else out_a[q * cout + co] = Act<A>::from(v);
            }
        }
    }
}

// Convolution with one input channel: the 27 taps (padded to 32) form K of a
// single 16x16x32 bf16 step (lane kq supplies taps 8 kq .. 8 kq + 7), or of
// eight 16x16x4 f32 steps in the FP32 mode (step j: tap 8 kq + j of every
// lane).  W1: [NTILE*16][32].
template <int NTILE, typename A>
__global__ void __launch_bounds__(256)
conv_c1(InDescT<A> in, Geo g, const A *__restrict__ W1, int cout, A *out_a, float *out_f32, int relu) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p0 = (blockIdx.x * 4 + wave) * 16;
    if (p0 >= g.npts) return;
    const int m = lane & 15, kq = lane >> 4;
    int p = p0 + m;
    if (p >= g.npts) p = p0;
    const int x = p % g.nx, y = (p / g.nx) % g.ny, z = p / (g.nx * g.ny);
    A a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int t = 8 * kq + j;
        A v = A(0);
        if (t < 27) {
            const int xx = wrapc(x + (t % 3) - 1, g.nx), yy = wrapc(y + (t / 3) % 3 - 1, g.ny),
                      zz = wrapc(z + t / 9 - 1, g.nz);
            v = fetch1<A>(in, xx, yy, zz, 0, g);
        }
        a[j] = v;
    }
#pragma unroll
    for (int nt = 0; nt < NTILE; ++nt) {
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        const A *wrow = W1 + (size_t)(nt * 16 + m) * 32 + 8 * kq;
        if constexpr (sizeof(A) == 2) {
            s16x8 av;
#pragma unroll
            for (int j = 0; j < 8; ++j) av[j] = (short)a[j];
            const uint4 raw = *reinterpret_cast<const uint4 *>(wrow);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                          __builtin_bit_cast(bf16x8, raw), acc, 0, 0, 0);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], wrow[j], acc, 0, 0, 0);
        }
        const int co = nt * 16 + m;
        if (co >= cout) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = p0 + 4 * kq + i;
            if (q >= g.npts) continue;
            float v = acc[i];
            if (relu) v = fmaxf(v, 0.f);
            if (out_f32) out_f32[(size_t)q * cout + co] = v;
            else out_a[(size_t)q * cout + co] = Act<A>::from(v);
        }
    }
}

// Weight gradient on bricks: one block (4 waves) owns a (16 ci x 16 co) tile
// pair and a column of kWbZg bricks of 16 x 4 x 4 points along z.  Per brick
// the input tile with its one-point halo (18 x 6 x 6 points, the ci tile)
// and the masked output gradient (256 points, the co tile) are staged in LDS
// once; every wave then runs its taps (t = wave + 4u) over the brick's 16
// rows of 16 points, one MFMA K step per row (bf16 16x16x16, or four f32
// 16x16x4 steps): lane (m, kq) supplies X[row point 4 kq + j + shift][ci m]
// and dY[row point 4 kq + j][co m] (zero outside the grid), so each input
// value is read from memory once per brick instead of once per tap.
// part[chunk][t][ci][co], chunk = block column; summed by wgrad_reduce.

inline int wb_chunks(const Geo &g, int &nbx, int &nby, int &ngz) {
    nbx = (g.nx + kWbX - 1) / kWbX;
    nby = (g.ny + kWbY - 1) / kWbY;
    const int nbz = (g.nz + kWbZ - 1) / kWbZ;
    ngz = (nbz + kWbZg - 1) / kWbZg;
    return nbx * nby * ngz;
}

template <typename A>
__global__ void __launch_bounds__(256)
conv_wgrad_brick(InDescT<A> x_in, Geo g, const A *__restrict__ dy, const A *__restrict__ ymask, int cin,
                 int cout, int nbx, int nby, float *__restrict__ part) {
    __shared__ A xs[kWbHalo * kWbStride];
    __shared__ A ys[kWbPts * kWbStride];
    const int cot = (cout + 15) / 16;
    const int cit = blockIdx.y / cot, co_t = blockIdx.y % cot;
    int b = blockIdx.x;
    const int bxi = b % nbx;
    b /= nbx;
    const int byi = b % nby;
    const int gz = b / nby;
    const int x0 = bxi * kWbX, y0 = byi * kWbY;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, kq = lane >> 4;
    const int ci0 = cit * 16, co0 = co_t * 16;
    const int nbz = (g.nz + kWbZ - 1) / kWbZ;
    f32x4 acc[7];
#pragma unroll
    for (int u = 0; u < 7; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int bz = gz * kWbZg; bz < min((gz + 1) * kWbZg, nbz); ++bz) {
        const int z0 = bz * kWbZ;
        __syncthreads();                      // the previous brick's readers are done
        // input tile with halo, channels [ci0, ci0 + 16), periodic images
        if (cin >= 16) {
            for (int e = tid; e < kWbHalo * 4; e += 256) {
                const int q = e >> 2, c4 = e & 3;
                const int lx = q % kWbTX, ly = (q / kWbTX) % kWbTY, lz = q / (kWbTX * kWbTY);
                const typename Vec4<A>::type v =
                    fetch4<A>(x_in, wrap_any(x0 - 1 + lx, g.nx), wrap_any(y0 - 1 + ly, g.ny),
                              wrap_any(z0 - 1 + lz, g.nz), ci0 + 4 * c4, g);
#pragma unroll
                for (int j = 0; j < 4; ++j) xs[q * kWbStride + 4 * c4 + j] = static_cast<A>(v[j]);   // same bits: short -> u16, float -> float
            }
        } else {                              // one input channel
            for (int q = tid; q < kWbHalo; q += 256) {
                const int lx = q % kWbTX, ly = (q / kWbTX) % kWbTY, lz = q / (kWbTX * kWbTY);
                xs[q * kWbStride] = fetch1<A>(x_in, wrap_any(x0 - 1 + lx, g.nx), wrap_any(y0 - 1 + ly, g.ny),
                                              wrap_any(z0 - 1 + lz, g.nz), 0, g);
#pragma unroll
                for (int c = 1; c < 16; ++c) xs[q * kWbStride + c] = A(0);
            }
        }
        // masked output gradient of the brick's points, channels [co0, co0 + 16)
        for (int e = tid; e < kWbPts * 16; e += 256) {
            const int q = e >> 4, c = e & 15;
            const int lx = q % kWbX, ly = (q / kWbX) % kWbY, lz = q / (kWbX * kWbY);
            const int x = x0 + lx, y = y0 + ly, z = z0 + lz, co = co0 + c;
            A d = A(0);
            if (x < g.nx && y < g.ny && z < g.nz && co < cout) {
                const size_t i = (size_t)pidx(x, y, z, g) * cout + co;
                d = dy[i];
                if (ymask && !Act<A>::pos(ymask[i])) d = A(0);
            }
            ys[q * kWbStride + c] = d;
        }
        __syncthreads();
        for (int r = 0; r < kWbY * kWbZ; ++r) {
            const int ly = r % kWbY, lz = r / kWbY;
            A bv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = ys[((lz * kWbY + ly) * kWbX + 4 * kq + j) * kWbStride + m];
#pragma unroll
            for (int u = 0; u < 7; ++u) {
                const int t = wave + 4 * u;
                if (t >= 27) break;
                const int dx = t % 3, dyo = (t / 3) % 3, dz = t / 9;      // shift + 1
                const A *xr = xs + (((lz + dz) * kWbTY + (ly + dyo)) * kWbTX + 4 * kq + dx) * kWbStride + m;
                A av[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) av[j] = xr[j * kWbStride];
                if constexpr (sizeof(A) == 2) {
                    s16x4 a, bb;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        a[j] = (short)av[j];
                        bb[j] = (short)bv[j];
                    }
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[u], 0, 0, 0);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], bv[j], acc[u], 0, 0, 0);
                }
            }
        }
    }
    // lane holds D[ci = ci0 + 4 kq + i][co = co0 + m] of each of its taps
    const int co = co0 + m;
#pragma unroll
    for (int u = 0; u < 7; ++u) {
        const int t = wave + 4 * u;
        if (t >= 27) break;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ci = ci0 + 4 * kq + i;
            if (ci < cin && co < cout)
                part[(((size_t)blockIdx.x * 27 + t) * cin + ci) * cout + co] = acc[u][i];
        }
    }
}

// First stage of the chunk sum: slice s of `slices` sums chunks
// [s * per, (s + 1) * per) in order into tmp[s][i] (per = ceil(chunks /
// slices)), so that many blocks share the work; wgrad_reduce then sums the
// slices in order.  The result does not depend on timing.
__global__ void wgrad_reduce_slices(const float *__restrict__ part, int chunks, int count, int slices,
                                    float *__restrict__ tmp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int sl = blockIdx.y;
    if (i >= count) return;
    const int per = (chunks + slices - 1) / slices;
    const int c0 = sl * per, c1 = min(c0 + per, chunks);
    float s = 0.f;
    for (int c = c0; c < c1; ++c) s += part[(size_t)c * count + i];
    tmp[(size_t)sl * count + i] = s;
}

// dW[i] = sum over chunks (fixed order) of part[chunk][i]
__global__ void wgrad_reduce(const float *__restrict__ part, int chunks, int count, float *__restrict__ dw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(size_t)c * count + i];
    dw[i] = s;
}

// 2x2x2 average pooling (fine grid g, C channels).
template <typename A>
__global__ void pool2(const A *__restrict__ in, Geo g, int C, A *__restrict__ out) {
    const int hx = g.nx / 2, hy = g.ny / 2, hz = g.nz / 2;
    const int64_t total = (int64_t)hx * hy * hz * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const int64_t q = i / C;
        const int x = (int)(q % hx), y = (int)((q / hx) % hy), z = (int)(q / ((int64_t)hx * hy));
        float s = 0.f;
        for (int d = 0; d < 8; ++d) {
            const int xx = 2 * x + (d & 1), yy = 2 * y + ((d >> 1) & 1), zz = 2 * z + (d >> 2);
            s += Act<A>::f(in[((size_t)(zz * g.ny + yy) * g.nx + xx) * C + c]);
        }
        out[i] = Act<A>::from(0.125f * s);
    }
}

// Gradient through [up(coarse), skip] concatenation at the fine level:
// dcoarse[q][c] = sum of dcat[child][c] over the 8 children (c < c1).
template <typename A>
__global__ void up_grad(const A *__restrict__ dcat, Geo g, int ccat, int c1, A *__restrict__ dcoarse) {
    const int hx = g.nx / 2, hy = g.ny / 2, hz = g.nz / 2;
    const int64_t total = (int64_t)hx * hy * hz * c1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % c1);
        const int64_t q = i / c1;
        const int x = (int)(q % hx), y = (int)((q / hx) % hy), z = (int)(q / ((int64_t)hx * hy));
        float s = 0.f;
        for (int d = 0; d < 8; ++d) {
            const int xx = 2 * x + (d & 1), yy = 2 * y + ((d >> 1) & 1), zz = 2 * z + (d >> 2);
            s += Act<A>::f(dcat[((size_t)(zz * g.ny + yy) * g.nx + xx) * ccat + c]);
        }
        dcoarse[i] = Act<A>::from(s);
    }
}

// dskip[p][c] = dcat[p][c1 + c] + pool_grad(dpool)[p][c]  (pool_grad = 1/8 of the parent)
template <typename A>
__global__ void skip_grad(const A *__restrict__ dcat, Geo g, int ccat, int c1, int cs,
                          const A *__restrict__ dpool, A *__restrict__ dskip) {
    const int64_t total = (int64_t)g.npts * cs;
    const int hx = g.nx / 2, hy = g.ny / 2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % cs);
        const int64_t p = i / cs;
        const int x = (int)(p % g.nx), y = (int)((p / g.nx) % g.ny), z = (int)(p / ((int64_t)g.nx * g.ny));
        const size_t parent = ((size_t)(z / 2) * hy + (y / 2)) * hx + (x / 2);
        dskip[i] = Act<A>::from(Act<A>::f(dcat[(size_t)p * ccat + c1 + c]) +
                                0.125f * Act<A>::f(dpool[parent * cs + c]));
    }
}

// Adam (FP32 masters) + BF16 copies in the forward and transposed layouts.
struct LayerPtrs {
    float *w, *m, *v, *g;
    u16 *wf, *wb;
    int cin, cout, ntf, ntb;   // padded tile counts of the forward / transposed layouts
};

__global__ void adam_kernel(LayerPtrs L, float lr, float b1, float b2, float c1, float c2, float eps) {
    const int count = 27 * L.cin * L.cout;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const float gr = L.g[i];
        const float m = b1 * L.m[i] + (1.f - b1) * gr;
        const float v = b2 * L.v[i] + (1.f - b2) * gr * gr;
        L.m[i] = m;
        L.v[i] = v;
        L.w[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    }
}

// BF16 (or, for the FP32 mode, FP32) copies of layer weights W[t][ci][co].
//   forward, cin >= 16: wf[t][co_pad][ci]; cin == 1: wf[co_pad][32 taps]
//   transposed (input gradient), flipped taps t' = 26 - t, roles swapped:
//   cout >= 16: wb[t'][ci_pad][co]; cout == 1: wb[ci_pad][32 taps]
template <typename A>
__global__ void pack_weights(const float *__restrict__ w, int cin, int cout, int ntf, int ntb,
                             A *__restrict__ wf, A *__restrict__ wb) {
    const int cof = ntf * 16, cib = ntb * 16;
    const int nf = cin == 1 ? cof * 32 : 27 * cof * cin;
    const int nb = cout == 1 ? cib * 32 : 27 * cib * cout;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nf + nb; i += gridDim.x * blockDim.x) {
        if (i < nf) {
            float v = 0.f;
            if (cin == 1) {
                const int co = i / 32, t = i % 32;
                if (co < cout && t < 27) v = w[(size_t)t * cout + co];
            } else {
                const int ci = i % cin, co = (i / cin) % cof, t = i / (cin * cof);
                if (co < cout) v = w[((size_t)t * cin + ci) * cout + co];
            }
            wf[i] = Act<A>::from(v);
        } else {
            const int j = i - nf;
            float v = 0.f;
            if (cout == 1) {
                const int ci = j / 32, t = j % 32;
                if (ci < cin && t < 27) v = w[(size_t)(26 - t) * cin + ci];
            } else {
                const int co = j % cout, ci = (j / cout) % cib, t = j / (cout * cib);
                if (ci < cin) v = w[((size_t)(26 - t) * cin + ci) * cout + co];
            }
            wb[j] = Act<A>::from(v);
        }
    }
}

// Network input: x = A(a * scale); totals of a^2 are computed beforehand.
template <typename A>
struct CastInOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 8 + sizeof(A);
    const double *a;
    A *x;
    const double *totals;       // {sum a^2}
    double inv_n, scale;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {
        const double ms = totals[0] * inv_n;
        scale = ms > 0 ? 1.0 / sqrt(ms) : 0.0;
    }
    __device__ void operator()(int64_t i, double (&)[1]) const { x[i] = Act<A>::from((float)(a[i] * scale)); }
};

struct SqOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 8;
    const double *a;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[1]) const { acc[0] = ::fma(a[i], a[i], acc[0]); }
};

// Loss ||out - t||^2 / ||t||^2 and dout = 2 (out - t) / ||t||^2 (BF16), with
// t = phi / (h^2 rms(g)).  totals: {sum g^2 (input), sum phi^2} precomputed.
template <typename A>
struct LossOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 12 + sizeof(A);
    const float *out;
    const double *phi;
    A *dout;
    const double *totals;
    double inv_n, h2, tscale, den;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {
        const double rms = sqrt(totals[0] * inv_n);
        tscale = rms > 0 ? 1.0 / (h2 * rms) : 0.0;
        den = totals[1] * tscale * tscale;
    }
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        const double t = phi[i] * tscale;
        const double d = (double)out[i] - t;
        acc[0] = ::fma(d, d, acc[0]);
        dout[i] = Act<A>::from((float)(2.0 * d / den));
    }
};

// Operator-weighted losses with A = -h^2 L_h, e = out - t, t = phi / (h^2 rms g):
// energy norm e^T A e / t^T A t (the norm CG minimises) and residual norm
// |A e|^2 / |A t|^2 (the residual a correction leaves).  EnergyErrOp forms e;
// the caller applies A, puts the unscaled denominator (phi^T A phi or
// |A phi|^2) in totals[1]; EnergyLossOp sums the numerator and writes the
// BF16 gradient.
struct EnergyErrOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 20;
    const float *out;
    const double *phi;
    double *e;
    const double *totals;
    double inv_n, h2, tscale;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {
        const double rms = sqrt(totals[0] * inv_n);
        tscale = rms > 0 ? 1.0 / (h2 * rms) : 0.0;
    }
    __device__ void operator()(int64_t i, double (&)[1]) const { e[i] = (double)out[i] - phi[i] * tscale; }
};

struct DotOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 16;
    const double *a, *b;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {}
    __device__ void operator()(int64_t i, double (&acc)[1]) const { acc[0] = ::fma(a[i], b[i], acc[0]); }
};

// Sums a.b and writes dout = 2 grad / den (BF16): energy norm (a = e, b =
// grad = A e) or residual norm (a = b = A e, grad = A A e).
template <typename A>
struct EnergyLossOp {
    static constexpr int kClass = K_POINTWISE;
    static constexpr int kBytes = 24 + sizeof(A);
    const double *a, *b, *grad;
    A *dout;
    const double *totals;
    double inv_n, h2, den;
    __device__ bool skip() const { return false; }
    __device__ void prepare() {
        const double rms = sqrt(totals[0] * inv_n);
        const double tscale = rms > 0 ? 1.0 / (h2 * rms) : 0.0;
        den = totals[1] * tscale * tscale;
    }
    __device__ void operator()(int64_t i, double (&acc)[1]) const {
        acc[0] = ::fma(a[i], b[i], acc[0]);
        dout[i] = Act<A>::from((float)(2.0 * grad[i] / den));
    }
};

}  // namespace nn
}  // namespace ofdft
