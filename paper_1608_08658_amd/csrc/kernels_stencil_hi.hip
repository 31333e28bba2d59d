// Stencil instantiations for half-widths M = 5..8 (space orders 10..16).
#include "stencil_impl.hpp"

namespace awe {

hipError_t launch_step_hi(const Layout& L, const StencilCoef& k, const StepArgs& a, int mode, int cfg, int zchunk,
                          hipStream_t s, const FusedSparse& fs) {
    switch (L.half) {
        case 5: return launch_m<5>(L, k, a, mode, cfg, zchunk, s, fs);
        case 6: return launch_m<6>(L, k, a, mode, cfg, zchunk, s, fs);
        case 7: return launch_m<7>(L, k, a, mode, cfg, zchunk, s, fs);
        case 8: return launch_m<8>(L, k, a, mode, cfg, zchunk, s, fs);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace awe
