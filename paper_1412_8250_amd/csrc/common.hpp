// Shared host/device helpers of the gfx950 library: status handling, FD
// coefficients, value traits for real/complex element types, and
// deterministic block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "ofdft.h"

namespace ofdft {

void set_error(const char *fmt, ...);

#define OFDFT_CHECK_HIP(call)                                                                \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            ::ofdft::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),        \
                               __FILE__, __LINE__);                                          \
            return OFDFT_HIP_ERROR;                                                          \
        }                                                                                    \
    } while (0)

#define OFDFT_TRY(expr)                                                                      \
    do {                                                                                     \
        int st_ = (expr);                                                                    \
        if (st_ < 0) return st_;                                                             \
    } while (0)

constexpr int kMaxRadius = 6;
// Block-partial slots of the reduction buffers (upper bound on reducing grids).
constexpr int kRedSlots = 8192;

// Coefficients of the order-2N Laplacian in the form used by the kernels:
//   L x = c0 * x + sum_{p=1..6} (wx[p] (x_{i+p}+x_{i-p}) + wy[p] (...) + wz[p] (...))
// with c0 = 2 (w0x + w0y + w0z).  Entries beyond the radius are zero.
template <typename S>
struct Coef {
    S c0;
    S wx[kMaxRadius + 1], wy[kMaxRadius + 1], wz[kMaxRadius + 1];
};

// Section 4 weight formulas for one axis (h given), written with a running
// product for (N!)^2 / ((N-p)!(N+p)!).
void axis_weights(int N, double h, double *w /* [kMaxRadius+1] */);
Coef<double> make_coef(const ofdft_grid &g, int radius);
Coef<float> to_float(const Coef<double> &c);

int check_grid(const ofdft_grid *g, int radius);

// Checkpoint files: device arrays written and read through a host staging
// buffer (blocking copies).  Each returns OFDFT_OK, or an error with the
// message set (INVALID_ARG for a short or failed file operation).
int ck_write_dev(std::FILE *f, const void *dev, size_t bytes);
int ck_read_dev(std::FILE *f, void *dev, size_t bytes);
int ck_write(std::FILE *f, const void *host, size_t bytes);
int ck_read(std::FILE *f, void *host, size_t bytes);
inline int64_t npoints(const ofdft_grid &g) { return (int64_t)g.nx * g.ny * g.nz; }

// ---------------------------------------------------------------------------
// Value traits: arithmetic with real weights on real and complex elements.
// ---------------------------------------------------------------------------
template <typename T> struct VT;

template <> struct VT<double> {
    using S = double;
    static constexpr int ncomp = 1;
    __device__ static double zero() { return 0.0; }
    __device__ static double add(double a, double b) { return a + b; }
    __device__ static double sub(double a, double b) { return a - b; }
    __device__ static double fma(S w, double x, double acc) { return ::fma(w, x, acc); }
    __device__ static double mul(S w, double x) { return w * x; }
};
template <> struct VT<float> {
    using S = float;
    static constexpr int ncomp = 1;
    __device__ static float zero() { return 0.0f; }
    __device__ static float add(float a, float b) { return a + b; }
    __device__ static float sub(float a, float b) { return a - b; }
    __device__ static float fma(S w, float x, float acc) { return fmaf(w, x, acc); }
    __device__ static float mul(S w, float x) { return w * x; }
};
template <> struct VT<double2> {
    using S = double;
    static constexpr int ncomp = 2;
    __device__ static double2 zero() { return make_double2(0.0, 0.0); }
    __device__ static double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
    __device__ static double2 sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
    __device__ static double2 fma(S w, double2 x, double2 acc) {
        return make_double2(::fma(w, x.x, acc.x), ::fma(w, x.y, acc.y));
    }
    __device__ static double2 mul(S w, double2 x) { return make_double2(w * x.x, w * x.y); }
};
template <> struct VT<float2> {
    using S = float;
    static constexpr int ncomp = 2;
    __device__ static float2 zero() { return make_float2(0.0f, 0.0f); }
    __device__ static float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
    __device__ static float2 sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
    __device__ static float2 fma(S w, float2 x, float2 acc) {
        return make_float2(fmaf(w, x.x, acc.x), fmaf(w, x.y, acc.y));
    }
    __device__ static float2 mul(S w, float2 x) { return make_float2(w * x.x, w * x.y); }
};

// Complex helpers on double2 (re, im).
__device__ __host__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __host__ inline double2 cdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  A block reduces its threads' values with wave64
// shuffles and LDS in a fixed pattern; each block writes its partial to a
// slot; the last block to finish (counted with a vector-memory atomic) sums
// the slots with all its threads in a fixed assignment and a fixed tree.
// Results are bitwise repeatable.
// ---------------------------------------------------------------------------
template <int K>
struct DVec {
    double v[K];
};

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Reduce K doubles over the block; result valid in thread 0.  `scratch` must
// hold K * (blockDim/64) doubles.  Includes the barriers it needs.
template <int K>
__device__ inline void block_sum(double (&x)[K], double *scratch) {
    const int lane = threadIdx.x + threadIdx.y * blockDim.x;
    const int nwaves = (blockDim.x * blockDim.y + 63) / 64;
    const int w = lane >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] = wave_sum(x[k]);
    __syncthreads();
    if ((lane & 63) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) scratch[w * K + k] = x[k];
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int i = 0; i < nwaves; ++i) s += scratch[i * K + k];
            x[k] = s;
        }
    }
}

// Publish a block partial (thread 0 holds it) and return true in thread 0 of
// the last block to arrive.  `counter` must start at 0; the last block resets
// it.  `partials` has K * gridDim slots laid out [k][block].
//
// Visibility without a device-wide cache flush: the partials are written
// with agent-scope atomic stores, which the gfx9 cache policy makes coherent
// at the device level (they write through the XCD's L2), and the arrival is
// counted only after those stores have completed: `s_waitcnt vmcnt(0)`
// stalls the wave until every vector-memory operation it issued, stores
// included, has been acknowledged by the memory system, and the asm
// statement's memory clobber keeps the compiler from moving the stores past
// it.  The last block reads the partials with agent-scope atomic loads, which
// do not hit a stale L2 line, issued after its counter RMW has returned.  No
// other data crosses blocks inside the kernel, so no agent-scope release
// fence (which writes back the L2 of the XCD and costs in proportion to the
// dirty data the kernel has produced) is needed.
__device__ inline void wait_vector_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <int K>
__device__ inline bool publish_partial(const double (&x)[K], double *partials, int nblocks,
                                       int block, unsigned int *counter) {
    bool last = false;
    if (threadIdx.x == 0 && threadIdx.y == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            __hip_atomic_store(partials + (size_t)k * nblocks + block, x[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        wait_vector_memory();
        const unsigned int prev =
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == (unsigned int)nblocks - 1);
        if (last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return last;
}

// Sum K partial arrays with the whole last block: thread t sums partials t,
// t + nthreads, ... in order, then a fixed tree combines the threads.
// Deterministic (the assignment does not depend on timing).  All threads of the block must call it; the result
// is valid in thread 0.  `scratch` as for block_sum.
template <int K>
__device__ inline void sum_partials_block(const double *partials, int nblocks, double (&out)[K],
                                          double *scratch) {
    const int nt = blockDim.x * blockDim.y;
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double a = 0.0;
        for (int i = t; i < nblocks; i += nt)
            a += __hip_atomic_load(partials + (size_t)k * nblocks + i, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        out[k] = a;
    }
    block_sum<K>(out, scratch);
}

// publish + (in the last block) whole-block sum.  Returns true in thread 0 of
// the last block, whose tot[] then holds the totals.  Every thread of every
// block must call it (it contains barriers).
template <int K>
__device__ inline bool reduce_grid(const double (&x)[K], double *partials, int nblocks, int block,
                                   unsigned int *counter, double *scratch, double (&tot)[K]) {
    __shared__ int s_last;
    const bool last0 = publish_partial<K>(x, partials, nblocks, block, counter);
    if (threadIdx.x == 0 && threadIdx.y == 0) s_last = last0 ? 1 : 0;
    __syncthreads();
    const bool last = s_last != 0;
    if (!last) return false;
    sum_partials_block<K>(partials, nblocks, tot, scratch);
    return threadIdx.x == 0 && threadIdx.y == 0;
}

// Global-address-space array view.  A pointer loaded from a device table is
// generic to the compiler, which then emits flat loads; those share a wait
// counter with LDS traffic, so every LDS wait would also wait for the
// prefetched loads.  GPtr casts to the global space (global loads/stores);
// two-component types go through the compiler's native vector types.
template <typename T> struct GNative { using type = T; };
template <> struct GNative<double2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct GNative<float2> { typedef float type __attribute__((ext_vector_type(2))); };

template <typename T>
struct GPtr {
    using N = typename GNative<T>::type;
    __attribute__((address_space(1))) N *p;
    GPtr() = default;
    __device__ explicit GPtr(const void *q) : p((__attribute__((address_space(1))) N *)q) {}
    __device__ T operator[](int64_t i) const {
        if constexpr (VT<T>::ncomp == 2) {
            const N v = p[i];
            T o;
            o.x = v.x;
            o.y = v.y;
            return o;
        } else {
            return p[i];
        }
    }
    __device__ void st(int64_t i, T v) const {
        if constexpr (VT<T>::ncomp == 2) {
            N w;
            w.x = v.x;
            w.y = v.y;
            p[i] = w;
        } else {
            p[i] = v;
        }
    }
};

// Logical block index such that the hardware's round-robin placement of
// consecutive workgroups over the 8 XCDs gives each XCD a contiguous range of
// logical tiles (neighbouring tiles then share that XCD's L2).
__device__ inline int xcd_remap(int b, int nblocks) {
    constexpr int kXcd = 8;
    const int xcd = b % kXcd, local = b / kXcd;
    const int per = nblocks / kXcd, rem = nblocks % kXcd;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

}  // namespace ofdft
