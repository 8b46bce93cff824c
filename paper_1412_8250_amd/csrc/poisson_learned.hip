// Learned form of the Poisson solve (network initial guess + flexible CG).
#include "poisson.hpp"

namespace ofdft {

int poisson_solve_learned(ofdft_poisson *s, double *, double, int, ofdft_solve_stats &, hipStream_t) {
    if (!s->net) {
        set_error("cg_poisson_solve: learned mode needs a network (ofdft_poisson_set_network)");
        return OFDFT_INVALID_ARG;
    }
    set_error("cg_poisson_solve: learned mode not available");
    return OFDFT_INVALID_ARG;
}

}  // namespace ofdft
