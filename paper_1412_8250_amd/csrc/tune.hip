// Launch-shape autotuner for the stencil kernels (not part of the method: it
// picks how the FD Laplacian of Section 4 is tiled on the chip).
//
// ofdft_tune_stencil times every legal (tile shape, z-chunk length) of one
// kernel family on one grid and element type, on scratch vectors of that
// grid, and records the fastest in the launch table (pick_stencil_cfg):
//   * FAMILY_APPLY: the plain apply y = L_h x (every element type);
//   * FAMILY_PASS: the fused single-pass stencil kernels, timed on the CG
//     stencil pass (p = r + beta p_old in the operand loads, A p, p^T A p);
//     the residual and density-update passes share its entry (FP64, FP32).
// The configuration the library would use untuned is always a candidate and
// keeps its place unless another one is more than 2% faster, so noise does
// not flip the choice.  All candidates compute the same operator (the tests
// check every shape against the oracle); only the reduction order of the
// fused passes changes with the tiling.
#include <algorithm>
#include <vector>

#include "poisson.hpp"
#include "stencil_apply.hpp"

namespace ofdft {
namespace {

template <typename E>
__global__ void tune_fill(E *a, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        a[i] = (E)(1.0 + (double)((uint64_t)(i * 2654435761ull) % 1024u) / 1024.0);
}

struct Candidate {
    int shape, zlen;
};

// Shapes whose launch differs for the element type and family (the 64 x 32
// tile exists only for the plain FP64 and FP32 applies; elsewhere it runs
// 64 x 16).
std::vector<int> legal_shapes(int elem_bytes, int family) {
    std::vector<int> s = {SHAPE_64x4x4, SHAPE_64x4x2, SHAPE_32x8x2, SHAPE_64x8x2, SHAPE_64x8x1};
    if (family == FAMILY_APPLY && elem_bytes <= 8) s.push_back(SHAPE_64x8x4);
    return s;
}

// z-chunk lengths: 0 (chosen from the kernel's residency) and the lengths of
// 1, 2, 3, 4, 6, 8, 12, 16 chunks (at least 8 planes, within the reduction
// slots).
std::vector<int> zlen_candidates(const ofdft_grid &g, int shape) {
    int tx, ty;
    shape_extent(shape, tx, ty);
    const int64_t tiles = (int64_t)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
    std::vector<int> z = {0};
    for (int c : {1, 2, 3, 4, 6, 8, 12, 16}) {
        const int zl = (g.nz + c - 1) / c;
        if (c > 1 && zl < 8) break;
        if (tiles * ((g.nz + zl - 1) / zl) > kRedSlots) break;
        if (std::find(z.begin(), z.end(), zl) == z.end()) z.push_back(zl);
    }
    return z;
}

struct TuneBuffers {
    std::vector<void *> mem;
    ~TuneBuffers() {
        for (void *p : mem) (void)hipFree(p);
    }
    int alloc(void **p, size_t bytes) {
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            set_error("ofdft_tune_stencil: device allocation of %zu bytes failed", bytes);
            return OFDFT_NO_MEMORY;
        }
        mem.push_back(*p);
        return OFDFT_OK;
    }
};

template <typename E>
int fill(void *p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(tune_fill<E>, dim3(1024), dim3(256), 0, s, (E *)p, n);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

}  // namespace
}  // namespace ofdft

using namespace ofdft;

extern "C" int ofdft_tune_stencil(const ofdft_grid *grid, int radius, ofdft_dtype dtype, int family, int reps,
                                  ofdft_tune_result *out, void *stream) {
    OFDFT_TRY(check_grid(grid, radius));
    const int eb = dtype == OFDFT_F64 ? 8 : dtype == OFDFT_F32 ? 4 : dtype == OFDFT_C128 ? 16 : dtype == OFDFT_C64 ? 8 : 0;
    if (!eb || (family != FAMILY_APPLY && family != FAMILY_PASS) ||
        (family == FAMILY_PASS && dtype != OFDFT_F64 && dtype != OFDFT_F32) || reps < 1 || reps > 1000) {
        set_error("ofdft_tune_stencil: bad dtype %d / family %d (PASS: F64 or F32) / reps %d", (int)dtype, family,
                  reps);
        return OFDFT_INVALID_ARG;
    }
    const ofdft_grid &g = *grid;
    const int64_t n = npoints(g);
    hipStream_t s = (hipStream_t)stream;
    TuneBuffers buf;
    void *x = nullptr, *y = nullptr, *pA = nullptr, *pB = nullptr, *st = nullptr;
    RedBuf rb{};
    const size_t bytes = (size_t)n * eb;
    OFDFT_TRY(buf.alloc(&x, bytes));
    OFDFT_TRY(buf.alloc(&y, bytes));
    const bool real64 = dtype == OFDFT_F64 || dtype == OFDFT_C128, wide = eb == 16 || dtype == OFDFT_C64;
    const int64_t ncomp = wide ? 2 * n : n;
    OFDFT_TRY(real64 ? fill<double>(x, ncomp, s) : fill<float>(x, ncomp, s));
    if (family == FAMILY_PASS) {
        OFDFT_TRY(buf.alloc(&pA, bytes));
        OFDFT_TRY(buf.alloc(&pB, bytes));
        OFDFT_TRY(buf.alloc(&st, sizeof(CgState)));
        OFDFT_TRY(buf.alloc((void **)&rb.partials, sizeof(double) * kRedSlots * kRedMaxK));
        OFDFT_TRY(buf.alloc((void **)&rb.counter, 256));
        OFDFT_CHECK_HIP(hipMemsetAsync(rb.counter, 0, 256, s));
        OFDFT_TRY(real64 ? fill<double>(pA, n, s) : fill<float>(pA, n, s));
        CgState hs{};
        hs.rr = 1.0;
        hs.beta = 0.5;
        hs.first = 0;
        hs.done = CG_RUNNING;
        hs.maxit = 1 << 30;
        OFDFT_CHECK_HIP(hipMemcpyAsync(st, &hs, sizeof hs, hipMemcpyHostToDevice, s));
    }
    const Coef<double> c = make_coef(g, radius);
    const Coef<float> c32 = to_float(c);
    auto launch = [&]() -> int {
        if (family == FAMILY_APPLY) return fd_laplacian_apply(grid, radius, dtype, x, y, 1.0, 0.0, stream);
        if (dtype == OFDFT_F64)
            return cg_k1<double>(g, c, (const double *)x, (const double *)pA, (double *)pB, (double *)y,
                                 (CgState *)st, rb, s);
        return cg_k1<float>(g, c32, (const float *)x, (const float *)pA, (float *)pB, (float *)y, (CgState *)st,
                            rb, s);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    OFDFT_CHECK_HIP(hipEventCreate(&e0));
    OFDFT_CHECK_HIP(hipEventCreate(&e1));
    const StencilCfg def = default_stencil_cfg(g, eb, family);
    std::vector<Candidate> cand;
    for (int sh : legal_shapes(eb, family))
        for (int zl : zlen_candidates(g, sh)) cand.push_back({sh, zl});
    if (std::none_of(cand.begin(), cand.end(), [&](const Candidate &k) { return k.shape == def.shape && k.zlen == def.zlen; }))
        cand.push_back({def.shape, def.zlen});
    double best = -1.0, def_ms = -1.0;
    Candidate pick{def.shape, def.zlen};
    int rc = OFDFT_OK;
    for (const Candidate &k : cand) {
        record_stencil_cfg(g, eb, family, StencilCfg{k.shape, k.zlen});
        if ((rc = launch()) != OFDFT_OK) break;                        // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) { rc = OFDFT_HIP_ERROR; break; }
        for (int r = 0; r < reps && rc == OFDFT_OK; ++r) rc = launch();
        if (rc != OFDFT_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = OFDFT_HIP_ERROR;
            break;
        }
        const double t = ms / reps;
        if (k.shape == def.shape && k.zlen == def.zlen) def_ms = t;
        if (best < 0.0 || t < best) {
            best = t;
            pick = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != OFDFT_OK) {
        erase_stencil_cfg(g, eb, family);
        return rc;
    }
    // the untuned configuration stays unless beaten by more than 2%
    if (def_ms > 0.0 && best > 0.98 * def_ms) {
        pick = Candidate{def.shape, def.zlen};
        best = def_ms;
    }
    record_stencil_cfg(g, eb, family, StencilCfg{pick.shape, pick.zlen});
    OFDFT_CHECK_HIP(hipStreamSynchronize(s));
    if (out) {
        *out = ofdft_tune_result{};
        out->shape = pick.shape;
        out->zlen = pick.zlen;
        out->group = 0;
        out->candidates = (int)cand.size();
        out->best_ms = best;
        out->default_ms = def_ms;
    }
    return OFDFT_OK;
}
