// Grid-stride elementwise kernels with fused deterministic reductions.
#pragma once

#include <type_traits>

#include "common.hpp"
#include "profile.hpp"

namespace ofdft {

constexpr int kVecThreads = 256;

// Functor F: __device__ void operator()(int64_t i, double (&acc)[K]) -- handles
// element i (may write outputs) and adds its contributions to acc.
// Fin: __device__ void operator()(const double (&tot)[K]) -- run by one thread
// of the last block with the grid totals.  F::skip() lets a kernel exit early.
template <int K, class F, class Fin>
__global__ void __launch_bounds__(kVecThreads)
reduce_kernel(int64_t n, F f, Fin fin, double *partials, unsigned int *counter) {
    __shared__ double scratch[K * (kVecThreads / 64)];
    if (f.skip()) return;
    f.prepare();
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kVecThreads;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) f(i, acc);
    block_sum<K>(acc, scratch);
    double tot[K];
    if (reduce_grid<K>(acc, partials, gridDim.x, blockIdx.x, counter, scratch, tot)) fin(tot);
}

inline int vec_blocks(int64_t n) {
    int64_t b = (n + kVecThreads * 4 - 1) / (kVecThreads * 4);
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

// Shared scratch for reductions: partial slots and an arrival counter.
struct RedBuf {
    double *partials = nullptr;   // capacity kRedSlots * 8 doubles
    unsigned int *counter = nullptr;
};
constexpr int kRedMaxK = 8;

// Accounting class and algorithmic bytes per element of an elementwise op
// (ops without kBytes count as pointwise work with no bytes recorded).
template <class F, class = void>
struct OpInfo {
    static constexpr int cls = K_POINTWISE;
    static constexpr int bytes = 0;
};
template <class F>
struct OpInfo<F, std::void_t<decltype(F::kBytes)>> {
    static constexpr int cls = F::kClass;
    static constexpr int bytes = F::kBytes;
};

template <int K, class F, class Fin>
inline int launch_reduce(int64_t n, const F &f, const Fin &fin, const RedBuf &rb, hipStream_t s,
                         int blocks = 0) {
    static_assert(K <= kRedMaxK, "too many reduction values");
    if (blocks <= 0) blocks = vec_blocks(n);
    if (blocks > kRedSlots) blocks = kRedSlots;
    ProfScope ps(OpInfo<F>::cls, (double)OpInfo<F>::bytes * (double)n, s);
    hipLaunchKernelGGL((reduce_kernel<K, F, Fin>), dim3(blocks), dim3(kVecThreads), 0, s, n, f, fin,
                       rb.partials, rb.counter);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

int redbuf_alloc(RedBuf &rb);
void redbuf_free(RedBuf &rb);

struct NoFin {
    template <int K>
    __device__ void operator()(const double (&)[K]) const {}
};

// Store the totals to device memory.
template <int K>
struct StoreTotals {
    double *dst;
    __device__ void operator()(const double (&t)[K]) const {
#pragma unroll
        for (int k = 0; k < K; ++k) dst[k] = t[k];
    }
};

}  // namespace ofdft
