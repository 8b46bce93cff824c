// cg_poisson_solve_noalloc: the plain FP64 form of cg_poisson_solve (Section
// 3.3 Poisson equation; Section 4 zero-mean convention) for callers that
// cannot allocate device memory.  The solver's workspace -- the projected
// right-hand side, the CG vectors r, p (two buffers) and A p, the device
// scalars, the reduction partials and their arrival counter -- lives in one
// file-scope device array instead of a context, so the call makes no device
// allocation, no host pinned allocation, creates no event and no graph.
//
// Every call on a GPU shares that GPU's copy of the array and leaves its
// contents behind; calls that overlap on one GPU (different streams or
// threads) race on it.  The arrival counter is cleared by a kernel at the
// start of each call; everything else is written before it is read.
#include <chrono>
#include <mutex>

#include "poisson.hpp"

namespace ofdft {
namespace {

// Largest grid (points) the static workspace holds: 2^20 (96^3 = 884,736 and
// 128 x 128 x 64 fit).
constexpr int64_t kNoAllocMaxPoints = int64_t(1) << 20;

// Layout in doubles: five vectors, then the CG state, totals, partials and
// the arrival counter (each part 256-byte aligned).
constexpr size_t kNaVec = (size_t)kNoAllocMaxPoints;
constexpr size_t kNaState = 5 * kNaVec;
constexpr size_t kNaTotals = kNaState + 64;
constexpr size_t kNaPart = kNaTotals + 32;
constexpr size_t kNaCtr = kNaPart + (size_t)kRedSlots * kRedMaxK;
constexpr size_t kNaDoubles = kNaCtr + 32;
static_assert(sizeof(CgState) <= 64 * sizeof(double), "CG state slot too small");

static __device__ __align__(256) double scratch[kNaDoubles];

// Device address of `scratch` on each device, looked up once per device.
std::mutex g_na_mu;
double *g_na_ptr[kMaxDevices] = {};

int na_base(double **out) {
    int dev = 0;
    OFDFT_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("cg_poisson_solve_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
        return OFDFT_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("cg_poisson_solve_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            return OFDFT_HIP_ERROR;
        }
        g_na_ptr[dev] = (double *)p;
    }
    *out = g_na_ptr[dev];
    return OFDFT_OK;
}

__global__ void na_clear_counter(unsigned int *ctr) {
    if (threadIdx.x < 64) ctr[threadIdx.x] = 0u;
}

}  // namespace
}  // namespace ofdft

using namespace ofdft;

extern "C" int cg_poisson_solve_noalloc(const ofdft_grid *grid, int radius, const double *rhs, double *x,
                                        double rel_tol, int max_iter, ofdft_solve_stats *stats, void *stream) {
    OFDFT_TRY(check_grid(grid, radius));
    if (!rhs || !x || rhs == x) {
        set_error("cg_poisson_solve_noalloc: NULL or aliased rhs / x");
        return OFDFT_INVALID_ARG;
    }
    if (!(rel_tol > 0) || max_iter < 0) {
        set_error("cg_poisson_solve_noalloc: rel_tol must be > 0 and max_iter >= 0");
        return OFDFT_INVALID_ARG;
    }
    const int64_t n = npoints(*grid);
    if (n > kNoAllocMaxPoints) {
        set_error("cg_poisson_solve_noalloc: %lld grid points exceed the static workspace (%lld points)",
                  (long long)n, (long long)kNoAllocMaxPoints);
        return OFDFT_INVALID_ARG;
    }
    double *base = nullptr;
    OFDFT_TRY(na_base(&base));
    hipStream_t st = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    // A solver view on the static workspace; host scalars live on this stack.
    CgState st_host{};
    double totals_host[16] = {};
    ofdft_poisson s{};
    s.g = *grid;
    s.radius = radius;
    s.mode = OFDFT_PLAIN_F64;
    s.coef = make_coef(*grid, radius);
    s.gp = base;
    s.r = base + kNaVec;
    s.pA = base + 2 * kNaVec;
    s.pB = base + 3 * kNaVec;
    s.Ap = base + 4 * kNaVec;
    s.st = (CgState *)(base + kNaState);
    s.st_host = &st_host;
    s.totals = base + kNaTotals;
    s.totals_host = totals_host;
    s.rb.partials = base + kNaPart;
    s.rb.counter = (unsigned int *)(base + kNaCtr);
    s.use_graphs = false;
    hipLaunchKernelGGL(na_clear_counter, dim3(1), dim3(64), 0, st, s.rb.counter);
    OFDFT_CHECK_HIP(hipGetLastError());
    ofdft_solve_stats local{};
    const int status = poisson_solve(&s, rhs, x, rel_tol, max_iter, local, st);
    OFDFT_CHECK_HIP(hipStreamSynchronize(st));
    local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    local.status = status;
    if (stats) *stats = local;
    if (status < 0 && status != OFDFT_HIP_ERROR) set_error("cg_poisson_solve_noalloc: status %d", status);
    return status;
}
