// Kernels of the learned solver aid: a 4-level periodic 3D convolutional
// U-Net (channels 16/32/64/64, 3x3x3 periodic convolutions, bias-free, ReLU,
// 2x average pooling, nearest upsampling, skip concatenation [up, skip]).
//
// Storage: activations and activation gradients are BF16, channels-last
// ([point][channel], point = (z*ny + y)*nx + x); weights are FP32 masters with
// BF16 copies in the layouts the kernels read; every product accumulates in
// FP32 on the matrix cores.  An FP32 mode of the same kernels stores
// activations, gradients and weight copies in FP32 and multiplies with
// v_mfma_f32_16x16x4 f32 (four K = 4 steps per 16-channel chunk, the same
// lane-to-operand pattern); it exists to check the kernels' indexing against
// the FP64 reference element by element.
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

// Activation storage: BF16 (u16 bits; the default) or FP32 (the FP32 mode of
// the same kernels, which checks their indexing against the FP64 reference
// element by element).
template <typename A> struct Act;
template <> struct Act<u16> {
    __device__ __host__ static float f(u16 v) { return bf2f(v); }
    __device__ __host__ static u16 from(float v) { return f2bf(v); }
    // post-ReLU value > 0 <=> bf16 bits > 0 as a signed 16-bit integer
    __device__ static bool pos(u16 v) { return (short)v > 0; }
};
template <> struct Act<float> {
    __device__ __host__ static float f(float v) { return v; }
    __device__ __host__ static float from(float v) { return v; }
    __device__ static bool pos(float v) { return v > 0.f; }
};

// Input of a convolution: channels [0, c1) from s1 (optionally stored at half
// resolution = nearest upsampling, optionally multiplied by (mask1 > 0)) and
// channels [c1, c1 + c2) from s2 (full resolution).
template <typename A>
struct InDescT {
    const A *s1;
    const A *mask1;
    const A *s2;
    int c1, c2;
    int up1;             // 1: s1 lives on the (nx/2, ny/2, nz/2) grid
};
using InDesc = InDescT<u16>;

struct Geo {
    int nx, ny, nz;
    int npts;
};

__device__ inline int pidx(int x, int y, int z, const Geo &g) { return (z * g.ny + y) * g.nx + x; }
__device__ inline int pidx_half(int x, int y, int z, const Geo &g) {
    return ((z >> 1) * (g.ny >> 1) + (y >> 1)) * (g.nx >> 1) + (x >> 1);
}

// 4 consecutive channels [c, c+4) of point (x,y,z) of the input (c % 4 == 0;
// a 4-channel group never straddles the two sources because c1 % 16 == 0):
// BF16 bits as s16x4, FP32 values as f32x4.
template <typename A> struct Vec4;
template <> struct Vec4<u16> { using type = s16x4; using raw = uint2; };
template <> struct Vec4<float> { using type = f32x4; using raw = uint4; };

template <typename A>
__device__ inline typename Vec4<A>::type fetch4(const InDescT<A> &in, int x, int y, int z, int c, const Geo &g) {
    using V = typename Vec4<A>::type;
    using Raw = typename Vec4<A>::raw;
    V v;
    if (c < in.c1) {
        const int q = in.up1 ? pidx_half(x, y, z, g) : pidx(x, y, z, g);
        const Raw raw = *reinterpret_cast<const Raw *>(in.s1 + (size_t)q * in.c1 + c);
        v = __builtin_bit_cast(V, raw);
        if (in.mask1) {
            const Raw mr = *reinterpret_cast<const Raw *>(in.mask1 + (size_t)q * in.c1 + c);
            const V m = __builtin_bit_cast(V, mr);
            // post-ReLU value > 0: the element compared as is (signed 16-bit
            // bits for BF16, the value for FP32)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (!(m[j] > 0)) v[j] = 0;
        }
    } else {
        const int q = pidx(x, y, z, g);
        const Raw raw = *reinterpret_cast<const Raw *>(in.s2 + (size_t)q * in.c2 + (c - in.c1));
        v = __builtin_bit_cast(V, raw);
    }
    return v;
}

// one channel (scalar) of the input, for the gather-style operand loads
template <typename A>
__device__ inline A fetch1(const InDescT<A> &in, int x, int y, int z, int c, const Geo &g) {
    if (c < in.c1) {
        const int q = in.up1 ? pidx_half(x, y, z, g) : pidx(x, y, z, g);
        A v = in.s1[(size_t)q * in.c1 + c];
        if (in.mask1 && !Act<A>::pos(in.mask1[(size_t)q * in.c1 + c])) v = A(0);
        return v;
    }
    if (c - in.c1 < in.c2) return in.s2[(size_t)pidx(x, y, z, g) * in.c2 + (c - in.c1)];
    return A(0);
}

__device__ inline int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

}  // namespace nn
}  // namespace ofdft
