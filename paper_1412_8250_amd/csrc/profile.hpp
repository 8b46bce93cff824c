// Launch accounting: every kernel launch adds its algorithmic HBM bytes (the
// bytes the method must move: each operand read once, each result written
// once) to a per-class counter; classes selected with ofdft_profile_reset()
// are also timed with HIP events recorded on the launch stream.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ofdft {

enum KClass {
    K_APPLY = 0,       // fd_laplacian_apply
    K_CG_STENCIL,      // CG: p update + stencil + p.Ap
    K_CG_UPDATE,       // CG: x, r update + r.r
    K_RESIDUAL,        // true-residual stencil passes
    K_COCG,            // batched COCG: stencil phases (the whole solve when persistent)
    K_U_STENCIL,       // density update: H u and L d passes
    K_U_VECTOR,        // density update: residual, line-search probes, step
    K_ANDERSON,
    K_POINTWISE,       // other vector passes (projections, casts, assembly)
    K_NN,              // network convolutions and their gradients
    K_COCG_UPDATE,     // batched COCG (stepped): x, r update + r.r
    K_MULTIGRID,       // multigrid cycles on FP64 vectors (Poisson, density update)
    K_MULTIGRID_C,     // multigrid cycles on complex128 vectors (shifted systems)
    K_MS_STENCIL,      // multi-shift COCG: seed direction + stencil + p.q
    K_MS_UPDATE,       // multi-shift COCG: every shift's p, x update; r update + r.r
    K_CLASSES
};

void prof_add(int cls, double bytes, int64_t launches = 1);
bool prof_timed(int cls);
// While suspended (this thread), launches are neither accounted nor timed:
// launches captured into a graph are accounted per replay by their caller.
void prof_suspend(bool on);
bool prof_suspended();
void prof_record(int cls, hipEvent_t a, hipEvent_t b);
hipEvent_t prof_event();

// RAII helper around one launch.
struct ProfScope {
    int cls;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    // active = false: nothing is accounted or recorded (launches captured
    // into a graph, accounted per replay by the caller)
    ProfScope(int c, double bytes, hipStream_t st, bool active = true) : cls(c), s(st) {
        if (!active || prof_suspended()) return;
        prof_add(c, bytes);
        if (prof_timed(c)) {
            a = prof_event();
            b = prof_event();
            if (a && b) (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope() {
        if (a && b) {
            (void)hipEventRecord(b, s);
            prof_record(cls, a, b);
        }
    }
};

}  // namespace ofdft
