// Status strings, FD coefficients and argument checks.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "vec.hpp"

namespace ofdft {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

// Section 4: w_0 = -(1/h^2) sum_{q=1}^{N} q^-2 and
// w_p = 2 (-1)^{p+1} / (h^2 p^2) * (N!)^2 / ((N-p)! (N+p)!).
// The factorial ratio equals prod_{j=1}^{p} (N-j+1)/(N+j).
void axis_weights(int N, double h, double *w) {
    for (int p = 0; p <= kMaxRadius; ++p) w[p] = 0.0;
    double s = 0.0;
    for (int q = 1; q <= N; ++q) s += 1.0 / (double(q) * q);
    const double ih2 = 1.0 / (h * h);
    w[0] = -s * ih2;
    double ratio = 1.0;
    for (int p = 1; p <= N; ++p) {
        ratio *= double(N - p + 1) / double(N + p);
        const double sign = (p & 1) ? 1.0 : -1.0;
        w[p] = 2.0 * sign * ratio / (double(p) * p) * ih2;
    }
}

Coef<double> make_coef(const ofdft_grid &g, int radius) {
    Coef<double> c;
    axis_weights(radius, g.hx, c.wx);
    axis_weights(radius, g.hy, c.wy);
    axis_weights(radius, g.hz, c.wz);
    c.c0 = 2.0 * (c.wx[0] + c.wy[0] + c.wz[0]);
    return c;
}

Coef<float> to_float(const Coef<double> &c) {
    Coef<float> f;
    f.c0 = (float)c.c0;
    for (int p = 0; p <= kMaxRadius; ++p) {
        f.wx[p] = (float)c.wx[p];
        f.wy[p] = (float)c.wy[p];
        f.wz[p] = (float)c.wz[p];
    }
    return f;
}

int check_grid(const ofdft_grid *g, int radius) {
    if (!g) {
        set_error("grid descriptor is NULL");
        return OFDFT_INVALID_ARG;
    }
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) {
        set_error("grid sizes must be >= 1 (got %d x %d x %d)", g->nx, g->ny, g->nz);
        return OFDFT_INVALID_ARG;
    }
    if ((int64_t)g->nx * g->ny > (int64_t)1 << 31 || npoints(*g) > ((int64_t)1 << 40)) {
        set_error("grid too large");
        return OFDFT_INVALID_ARG;
    }
    if (!(g->hx > 0) || !(g->hy > 0) || !(g->hz > 0) || !std::isfinite(g->hx) ||
        !std::isfinite(g->hy) || !std::isfinite(g->hz)) {
        set_error("grid spacings must be finite and > 0");
        return OFDFT_INVALID_ARG;
    }
    if (radius < 1 || radius > kMaxRadius) {
        set_error("radius must be in 1..%d (got %d)", kMaxRadius, radius);
        return OFDFT_INVALID_ARG;
    }
    return OFDFT_OK;
}

int redbuf_alloc(RedBuf &rb) {
    OFDFT_CHECK_HIP(hipMalloc(&rb.partials, sizeof(double) * kRedSlots * kRedMaxK));
    OFDFT_CHECK_HIP(hipMalloc(&rb.counter, 256));
    OFDFT_CHECK_HIP(hipMemset(rb.counter, 0, 256));
    return OFDFT_OK;
}

void redbuf_free(RedBuf &rb) {
    if (rb.partials) (void)hipFree(rb.partials);
    if (rb.counter) (void)hipFree(rb.counter);
    rb.partials = nullptr;
    rb.counter = nullptr;
}

}  // namespace ofdft

extern "C" int ofdft_last_error(char *buf, size_t len) {
    const std::string &e = ofdft::g_last_error;
    if (buf && len) {
        size_t n = e.size() < len - 1 ? e.size() : len - 1;
        memcpy(buf, e.data(), n);
        buf[n] = 0;
    }
    return (int)e.size();
}

extern "C" const char *ofdft_version(void) { return "ofdft-gfx950 0.3"; }

namespace ofdft {

int ck_write(std::FILE *f, const void *host, size_t bytes) {
    if (std::fwrite(host, 1, bytes, f) != bytes) {
        set_error("checkpoint: writing %zu bytes failed", bytes);
        return OFDFT_INVALID_ARG;
    }
    return OFDFT_OK;
}

int ck_read(std::FILE *f, void *host, size_t bytes) {
    if (std::fread(host, 1, bytes, f) != bytes) {
        set_error("checkpoint: the file ends before %zu more bytes", bytes);
        return OFDFT_INVALID_ARG;
    }
    return OFDFT_OK;
}

namespace {
constexpr size_t kCkChunk = (size_t)64 << 20;
}

int ck_write_dev(std::FILE *f, const void *dev, size_t bytes) {
    std::vector<char> buf(std::min(bytes, kCkChunk));
    for (size_t off = 0; off < bytes; off += kCkChunk) {
        const size_t b = std::min(kCkChunk, bytes - off);
        OFDFT_CHECK_HIP(hipMemcpy(buf.data(), (const char *)dev + off, b, hipMemcpyDeviceToHost));
        OFDFT_TRY(ck_write(f, buf.data(), b));
    }
    return OFDFT_OK;
}

int ck_read_dev(std::FILE *f, void *dev, size_t bytes) {
    std::vector<char> buf(std::min(bytes, kCkChunk));
    for (size_t off = 0; off < bytes; off += kCkChunk) {
        const size_t b = std::min(kCkChunk, bytes - off);
        OFDFT_TRY(ck_read(f, buf.data(), b));
        OFDFT_CHECK_HIP(hipMemcpy((char *)dev + off, buf.data(), b, hipMemcpyHostToDevice));
    }
    return OFDFT_OK;
}

}  // namespace ofdft
