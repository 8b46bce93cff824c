// Launch accounting and event timing (see profile.hpp).
#include <mutex>
#include <vector>

#include "common.hpp"
#include "profile.hpp"

namespace ofdft {

namespace {
struct Rec {
    int cls;
    hipEvent_t a, b;
};
std::mutex g_mu;
double g_bytes[K_CLASSES] = {};
int64_t g_launches[K_CLASSES] = {};
double g_ms[K_CLASSES] = {};
int64_t g_timed[K_CLASSES] = {};
unsigned g_mask = 0;
std::vector<Rec> g_pending;
std::vector<hipEvent_t> g_pool;

void drain_locked() {
    for (Rec &r : g_pending) {
        if (hipEventSynchronize(r.b) == hipSuccess) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                g_ms[r.cls] += ms;
                g_timed[r.cls] += 1;
            }
        }
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_pending.clear();
}
}  // namespace

namespace {
thread_local int t_suspend = 0;
}

void prof_suspend(bool on) { t_suspend += on ? 1 : -1; }
bool prof_suspended() { return t_suspend > 0; }

void prof_add(int cls, double bytes, int64_t launches) {
    if (t_suspend > 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_bytes[cls] += bytes;
    g_launches[cls] += launches;
}

bool prof_timed(int cls) { return (g_mask >> cls) & 1u; }

hipEvent_t prof_event() {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_pending.size() > 8192) drain_locked();
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_record(int cls, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back(Rec{cls, a, b});
}

}  // namespace ofdft

using namespace ofdft;

// Clear all counters; `timed_mask` selects the classes whose launches are
// bracketed by HIP events from now on (bit k = class k).
extern "C" int ofdft_profile_reset(unsigned timed_mask) {
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    for (int k = 0; k < K_CLASSES; ++k) {
        g_bytes[k] = 0;
        g_launches[k] = 0;
        g_ms[k] = 0;
        g_timed[k] = 0;
    }
    g_mask = timed_mask;
    return OFDFT_OK;
}

// Counters of one class: launches, algorithmic bytes, and (if timed) the number
// of timed launches and their summed duration in milliseconds.
extern "C" int ofdft_profile_read(int cls, int64_t *launches, double *bytes, int64_t *timed,
                                  double *ms) {
    if (cls < 0 || cls >= K_CLASSES) return OFDFT_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    if (launches) *launches = g_launches[cls];
    if (bytes) *bytes = g_bytes[cls];
    if (timed) *timed = g_timed[cls];
    if (ms) *ms = g_ms[cls];
    return OFDFT_OK;
}
