// anderson_mix (Appendix D):
//   v_{k+1} = v_k + zeta f_k - (S_k + zeta Y_k) (Y_k^T Y_k)^{-1} Y_k^T f_k
// with S_k, Y_k the last m differences of iterates and residuals.
//
// Three launches per call, no host synchronisation:
//  1. push + Gram pass: writes the new columns s = v - v_prev, y = f - f_prev
//     into the ring, saves v, f as the next v_prev, f_prev, and accumulates
//     Y^T Y and Y^T f over all active columns in one read of Y (FP64,
//     deterministic block partials);
//  2. one small workgroup solves the m x m system: Jacobi eigen-decomposition
//     of the Gram matrix, oldest columns dropped while cond >= 1e12, then
//     gamma = V diag(1/lambda) V^T (Y^T f);
//  3. update pass: v_next = v + zeta f - sum_j gamma_j (s_j + zeta y_j).
// The ring bookkeeping (head, count) lives in device memory so the sequence
// can be captured in a graph.
#include <algorithm>
#include <cmath>
#include <new>

#include "common.hpp"
#include "vec.hpp"

namespace ofdft {

constexpr int kAndMaxM = 8;
constexpr int kAndMaxK = kAndMaxM * (kAndMaxM + 1) / 2 + kAndMaxM;
constexpr int kAndBlocks = 1024;

struct AndState {
    int head, count, have_prev, m;
    int ncols;                 // columns used by the last solve (after drops)
    int pad[3];
    double gamma[kAndMaxM];    // coefficients, index = age order (0 = oldest)
    double totals[kAndMaxK];
};

// Index of the j-th oldest column after the push of this step.
__device__ inline int and_col(const AndState &s, int j, int m) { return (s.head + j) % m; }

template <int M>
__global__ void __launch_bounds__(kVecThreads)
and_push_gram(int64_t n, const double *__restrict__ v, const double *__restrict__ f,
              double *__restrict__ v_prev, double *__restrict__ f_prev, double *__restrict__ S,
              double *__restrict__ Y, AndState *st, double *partials, unsigned int *counter) {
    constexpr int K = M * (M + 1) / 2 + M;
    __shared__ double scratch[K * (kVecThreads / 64)];
    // Ring after this step's push (every block derives the same values).
    const int m = st->m, have = st->have_prev;
    int head = st->head, count = st->count, newc = -1;
    if (have && m > 0) {
        if (count < m) {
            newc = (head + count) % m;
            count += 1;
        } else {
            newc = head;
            head = (head + 1) % m;
        }
    }
    int cols[M];
#pragma unroll
    for (int j = 0; j < M; ++j) cols[j] = j < count ? (head + j) % m : 0;

    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kVecThreads;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        const double vi = v[i], fi = f[i];
        if (newc >= 0) {
            S[(int64_t)newc * n + i] = vi - v_prev[i];
            Y[(int64_t)newc * n + i] = fi - f_prev[i];
        }
        v_prev[i] = vi;
        f_prev[i] = fi;
        double y[M];
#pragma unroll
        for (int j = 0; j < M; ++j) y[j] = j < count ? Y[(int64_t)cols[j] * n + i] : 0.0;
        int k = 0;
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int b = a; b < M; ++b) {
                acc[k] = ::fma(y[a], y[b], acc[k]);
                ++k;
            }
#pragma unroll
        for (int a = 0; a < M; ++a) {
            acc[k] = ::fma(y[a], fi, acc[k]);
            ++k;
        }
    }
    block_sum<K>(acc, scratch);
    double tot[K];
    if (reduce_grid<K>(acc, partials, gridDim.x, blockIdx.x, counter, scratch, tot)) {
        for (int k = 0; k < K; ++k) st->totals[k] = tot[k];
        st->head = head;
        st->count = count;
        st->have_prev = 1;
    }
}

// Jacobi eigen-decomposition of a small symmetric matrix (n <= kAndMaxM).
__device__ inline void jacobi_eig(int n, double (*a)[kAndMaxM], double (*vec)[kAndMaxM], double *ev) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) vec[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += a[i][i] * a[i][i];
            for (int j = i + 1; j < n; ++j) off += a[i][j] * a[i][j];
        }
        if (off <= 1e-34 * diag || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (a[p][q] == 0.0) continue;
                const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = vec[k][p], vkq = vec[k][q];
                    vec[k][p] = c * vkp - s * vkq;
                    vec[k][q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) ev[i] = a[i][i];
}

template <int M>
__global__ void and_solve(AndState *st, double cond_max) {
    if (threadIdx.x != 0) return;
    const int count = st->count;
    double G[kAndMaxM][kAndMaxM], bvec[kAndMaxM];
    {
        int k = 0;
        for (int a = 0; a < M; ++a)
            for (int b = a; b < M; ++b, ++k) {
                G[a][b] = st->totals[k];
                G[b][a] = st->totals[k];
            }
        for (int a = 0; a < M; ++a, ++k) bvec[a] = st->totals[k];
    }
    for (int j = 0; j < kAndMaxM; ++j) st->gamma[j] = 0.0;
    // drop oldest columns while the Gram matrix is ill-conditioned
    int first = 0;
    while (first < count) {
        const int n = count - first;
        double A[kAndMaxM][kAndMaxM], V[kAndMaxM][kAndMaxM], ev[kAndMaxM];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) A[i][j] = G[first + i][first + j];
        jacobi_eig(n, A, V, ev);
        double lo = ev[0], hi = ev[0];
        for (int i = 1; i < n; ++i) {
            lo = fmin(lo, ev[i]);
            hi = fmax(hi, ev[i]);
        }
        if (lo > 0.0 && hi / lo < cond_max && isfinite(hi)) {
            // gamma = V diag(1/ev) V^T b
            double c[kAndMaxM];
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += V[j][i] * bvec[first + j];
                c[i] = s / ev[i];
            }
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int i = 0; i < n; ++i) s += V[j][i] * c[i];
                st->gamma[first + j] = s;
            }
            break;
        }
        ++first;
    }
    // dropped columns leave the history for good
    const int m = st->m;
    if (first > 0 && m > 0) {
        st->head = (st->head + first) % m;
        st->count = count - first;
        for (int j = 0; j < st->count; ++j) st->gamma[j] = st->gamma[j + first];
        for (int j = st->count; j < kAndMaxM; ++j) st->gamma[j] = 0.0;
    }
    st->ncols = st->count;
}

template <int M>
__global__ void __launch_bounds__(kVecThreads)
and_update(int64_t n, const double *__restrict__ v, const double *__restrict__ f,
           const double *__restrict__ S, const double *__restrict__ Y, double *v_next,
           const AndState *st, double zeta) {
    const int count = st->count, head = st->head, m = st->m;
    double gam[M];
    int cols[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        gam[j] = j < count ? st->gamma[j] : 0.0;
        cols[j] = j < count ? (head + j) % m : 0;
    }
    const int64_t stride = (int64_t)gridDim.x * kVecThreads;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        const double fi = f[i];
        double out = ::fma(zeta, fi, v[i]);
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j < count) {
                const int64_t o = (int64_t)cols[j] * n + i;
                out -= gam[j] * ::fma(zeta, Y[o], S[o]);
            }
        v_next[i] = out;
    }
}

}  // namespace ofdft

using namespace ofdft;

struct ofdft_anderson {
    int64_t n = 0;
    int m = 0;
    double zeta = 0.3;
    double *S = nullptr, *Y = nullptr, *v_prev = nullptr, *f_prev = nullptr;
    AndState *st = nullptr;
    double *partials = nullptr;
    unsigned int *counter = nullptr;
    int calls = 0;          // host-side count of mixes since the last reset (accounting only)
};

namespace {

template <int M>
int and_run(ofdft_anderson *a, const double *v, const double *f, double *v_next, hipStream_t s) {
    const int blocks = std::min(kAndBlocks, vec_blocks(a->n));
    const int have = a->calls > 0 ? 1 : 0;
    const int cols = std::min(a->calls, a->m);
    a->calls += 1;
    ProfScope ps1(K_ANDERSON, (double)a->n * 8.0 * (4 + 2 * (have && a->m > 0) + 2 + cols), s);
    hipLaunchKernelGGL((and_push_gram<M>), dim3(blocks), dim3(kVecThreads), 0, s, a->n, v, f,
                       a->v_prev, a->f_prev, a->S, a->Y, a->st, a->partials, a->counter);
    OFDFT_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL((and_solve<M>), dim3(1), dim3(64), 0, s, a->st, 1e12);
    OFDFT_CHECK_HIP(hipGetLastError());
    ProfScope ps2(K_ANDERSON, (double)a->n * 8.0 * (3 + 2 * cols), s);
    hipLaunchKernelGGL((and_update<M>), dim3(vec_blocks(a->n)), dim3(kVecThreads), 0, s, a->n, v,
                       f, a->S, a->Y, v_next, a->st, a->zeta);
    OFDFT_CHECK_HIP(hipGetLastError());
    return OFDFT_OK;
}

void and_free(ofdft_anderson *a) {
    void *p[] = {a->S, a->Y, a->v_prev, a->f_prev, a->st, a->partials, a->counter};
    for (void *q : p)
        if (q) (void)hipFree(q);
}

}  // namespace

extern "C" int ofdft_anderson_create(int64_t n, int m, double zeta, ofdft_anderson **out) {
    if (!out || n < 1 || m < 0 || m > kAndMaxM || !std::isfinite(zeta)) {
        set_error("ofdft_anderson_create: need n >= 1, 0 <= m <= %d, finite zeta", kAndMaxM);
        return OFDFT_INVALID_ARG;
    }
    ofdft_anderson *a = new (std::nothrow) ofdft_anderson();
    if (!a) return OFDFT_NO_MEMORY;
    a->n = n;
    a->m = m;
    a->zeta = zeta;
    auto fail = [&](int st) {
        and_free(a);
        delete a;
        return st;
    };
    const size_t cols = (size_t)(m > 0 ? m : 1) * n * sizeof(double);
    if (hipMalloc(&a->S, cols) != hipSuccess || hipMalloc(&a->Y, cols) != hipSuccess ||
        hipMalloc(&a->v_prev, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&a->f_prev, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&a->st, sizeof(AndState)) != hipSuccess ||
        hipMalloc(&a->partials, sizeof(double) * kAndBlocks * kAndMaxK) != hipSuccess ||
        hipMalloc(&a->counter, 256) != hipSuccess) {
        set_error("ofdft_anderson_create: out of device memory");
        return fail(OFDFT_NO_MEMORY);
    }
    if (hipMemset(a->counter, 0, 256) != hipSuccess) return fail(OFDFT_HIP_ERROR);
    int st = ofdft_anderson_reset(a);
    if (st != OFDFT_OK) return fail(st);
    *out = a;
    return OFDFT_OK;
}

extern "C" int ofdft_anderson_reset(ofdft_anderson *a) {
    if (!a) return OFDFT_INVALID_ARG;
    AndState h{};
    h.m = a->m;
    a->calls = 0;
    OFDFT_CHECK_HIP(hipMemcpy(a->st, &h, sizeof(AndState), hipMemcpyHostToDevice));
    return OFDFT_OK;
}

namespace ofdft {

// History of an Anderson context in a checkpoint: the host call count, the
// device state (ring head, column count, ...), S and Y (m columns) and the
// previous v and f.
int anderson_write(ofdft_anderson *a, std::FILE *f) {
    OFDFT_CHECK_HIP(hipDeviceSynchronize());
    const int64_t hdr[3] = {a->n, a->m, a->calls};
    OFDFT_TRY(ck_write(f, hdr, sizeof hdr));
    AndState h{};
    OFDFT_CHECK_HIP(hipMemcpy(&h, a->st, sizeof h, hipMemcpyDeviceToHost));
    OFDFT_TRY(ck_write(f, &h, sizeof h));
    const size_t col = sizeof(double) * (size_t)a->n * (size_t)std::max(a->m, 1);
    OFDFT_TRY(ck_write_dev(f, a->S, col));
    OFDFT_TRY(ck_write_dev(f, a->Y, col));
    OFDFT_TRY(ck_write_dev(f, a->v_prev, sizeof(double) * a->n));
    return ck_write_dev(f, a->f_prev, sizeof(double) * a->n);
}

int anderson_read(ofdft_anderson *a, std::FILE *f) {
    int64_t hdr[3];
    OFDFT_TRY(ck_read(f, hdr, sizeof hdr));
    if (hdr[0] != a->n || hdr[1] != a->m || hdr[2] < 0) {
        set_error("checkpoint: Anderson history of %lld values x %lld columns, the context has %lld x %d",
                  (long long)hdr[0], (long long)hdr[1], (long long)a->n, a->m);
        return OFDFT_INVALID_ARG;
    }
    AndState h{};
    OFDFT_TRY(ck_read(f, &h, sizeof h));
    const size_t col = sizeof(double) * (size_t)a->n * (size_t)std::max(a->m, 1);
    OFDFT_TRY(ck_read_dev(f, a->S, col));
    OFDFT_TRY(ck_read_dev(f, a->Y, col));
    OFDFT_TRY(ck_read_dev(f, a->v_prev, sizeof(double) * a->n));
    OFDFT_TRY(ck_read_dev(f, a->f_prev, sizeof(double) * a->n));
    OFDFT_CHECK_HIP(hipMemcpy(a->st, &h, sizeof h, hipMemcpyHostToDevice));
    a->calls = (int)hdr[2];
    return OFDFT_OK;
}

}  // namespace ofdft

extern "C" int ofdft_anderson_destroy(ofdft_anderson *a) {
    if (!a) return OFDFT_OK;
    and_free(a);
    delete a;
    return OFDFT_OK;
}

extern "C" int anderson_mix(ofdft_anderson *a, const double *v, const double *f, double *v_next,
                            void *stream) {
    if (!a || !v || !f || !v_next) {
        set_error("anderson_mix: NULL argument");
        return OFDFT_INVALID_ARG;
    }
    if (v_next == f) {
        set_error("anderson_mix: v_next must not alias f");
        return OFDFT_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    switch (a->m) {
        case 0: return and_run<1>(a, v, f, v_next, s);
        case 1: return and_run<1>(a, v, f, v_next, s);
        case 2: return and_run<2>(a, v, f, v_next, s);
        case 3: return and_run<3>(a, v, f, v_next, s);
        case 4: return and_run<4>(a, v, f, v_next, s);
        case 5: return and_run<5>(a, v, f, v_next, s);
        case 6: return and_run<6>(a, v, f, v_next, s);
        case 7: return and_run<7>(a, v, f, v_next, s);
        default: return and_run<8>(a, v, f, v_next, s);
    }
}
