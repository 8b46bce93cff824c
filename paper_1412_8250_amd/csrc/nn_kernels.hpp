// Kernels of the learned solver aid: a 4-level periodic 3D convolutional
// U-Net (channels 16/32/64/64, 3x3x3 periodic convolutions, bias-free, ReLU,
// 2x average pooling, nearest upsampling, skip concatenation [up, skip]).
//
// Storage: activations and activation gradients are BF16, channels-last
// ([point][channel], point = (z*ny + y)*nx + x); weights are FP32 masters with
// BF16 copies in the layouts the kernels read; every product accumulates in
// FP32 on the matrix cores.
//
// Convolution as implicit GEMM on gfx950 MFMA:
//   out[p][co] = sum_{t<27} sum_ci in[p + off_t][ci] W[t][ci][co]
//   M = 16 points per wave, N = C_out (16-channel tiles), K = (tap, 16 channels)
//   per v_mfma_f32_16x16x16 bf16 step.  Lane layout of that instruction:
//   lane l supplies A[l%16][4*(l/16)+j] and B[4*(l/16)+j][l%16] (j<4) and
//   receives D[4*(l/16)+i][l%16] (i<4).  Layers with one input channel pack
//   the 27 taps into K of one v_mfma_f32_16x16x32 bf16 step (8 K values/lane).
#pragma once

#include "common.hpp"

namespace ofdft {
namespace nn {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

__device__ __host__ inline float bf2f(u16 v) {
    union { unsigned u; float f; } c;
    c.u = (unsigned)v << 16;
    return c.f;
}
// round to nearest even
__device__ __host__ inline u16 f2bf(float f) {
    union { unsigned u; float f; } c;
    c.f = f;
    if ((c.u & 0x7fffffffu) > 0x7f800000u) return (u16)((c.u >> 16) | 0x40);   // NaN stays NaN
    const unsigned r = c.u + 0x7fffu + ((c.u >> 16) & 1u);
    return (u16)(r >> 16);
}

// Input of a convolution: channels [0, c1) from s1 (optionally stored at half
// resolution = nearest upsampling, optionally multiplied by (mask1 > 0)) and
// channels [c1, c1 + c2) from s2 (full resolution).
struct InDesc {
    const u16 *s1;
    const u16 *mask1;
    const u16 *s2;
    int c1, c2;
    int up1;             // 1: s1 lives on the (nx/2, ny/2, nz/2) grid
};

struct Geo {
    int nx, ny, nz;
    int npts;
};

__device__ inline int pidx(int x, int y, int z, const Geo &g) { return (z * g.ny + y) * g.nx + x; }
__device__ inline int pidx_half(int x, int y, int z, const Geo &g) {
    return ((z >> 1) * (g.ny >> 1) + (y >> 1)) * (g.nx >> 1) + (x >> 1);
}

// 4 consecutive channels [c, c+4) of point (x,y,z) of the input (c % 4 == 0;
// a 4-channel group never straddles the two sources because c1 % 16 == 0).
__device__ inline s16x4 fetch4(const InDesc &in, int x, int y, int z, int c, const Geo &g) {
    s16x4 v;
    if (c < in.c1) {
        const int q = in.up1 ? pidx_half(x, y, z, g) : pidx(x, y, z, g);
        const uint2 raw = *reinterpret_cast<const uint2 *>(in.s1 + (size_t)q * in.c1 + c);
        v = __builtin_bit_cast(s16x4, raw);
        if (in.mask1) {
            const uint2 mr = *reinterpret_cast<const uint2 *>(in.mask1 + (size_t)q * in.c1 + c);
            const s16x4 m = __builtin_bit_cast(s16x4, mr);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (!(m[j] > 0)) v[j] = 0;     // post-ReLU value > 0 <=> bf16 bits > 0
        }
    } else {
        const int q = pidx(x, y, z, g);
        const uint2 raw = *reinterpret_cast<const uint2 *>(in.s2 + (size_t)q * in.c2 + (c - in.c1));
        v = __builtin_bit_cast(s16x4, raw);
    }
    return v;
}

// one channel (scalar) of the input, for the gather-style operand loads
__device__ inline u16 fetch1(const InDesc &in, int x, int y, int z, int c, const Geo &g) {
    if (c < in.c1) {
        const int q = in.up1 ? pidx_half(x, y, z, g) : pidx(x, y, z, g);
        u16 v = in.s1[(size_t)q * in.c1 + c];
        if (in.mask1 && !((short)in.mask1[(size_t)q * in.c1 + c] > 0)) v = 0;
        return v;
    }
    if (c - in.c1 < in.c2) return in.s2[(size_t)pidx(x, y, z, g) * in.c2 + (c - in.c1)];
    return 0;
}

__device__ inline int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

}  // namespace nn
}  // namespace ofdft
