// Stencil instantiations for half-widths M = 1..4 (space orders 2..8).
#include "stencil_impl.hpp"

namespace awe {

hipError_t launch_step_lo(const Layout& L, const StencilCoef& k, const StepArgs& a, int mode, int cfg, int zchunk,
                          hipStream_t s, const FusedSparse& fs) {
    switch (L.half) {
        case 1: return launch_m<1>(L, k, a, mode, cfg, zchunk, s, fs);
        case 2: return launch_m<2>(L, k, a, mode, cfg, zchunk, s, fs);
        case 3: return launch_m<3>(L, k, a, mode, cfg, zchunk, s, fs);
        case 4: return launch_m<4>(L, k, a, mode, cfg, zchunk, s, fs);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace awe
