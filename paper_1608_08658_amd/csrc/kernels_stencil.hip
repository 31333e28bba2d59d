// Stencil step launcher: validates the launch, then dispatches on the
// half-width M to the instantiations in kernels_stencil_lo.hip (M = 1..4) and
// kernels_stencil_hi.hip (M = 5..8).  The kernels are in stencil_impl.hpp.
#include "awe_internal.hpp"

namespace awe {

hipError_t launch_step_lo(const Layout& L, const StencilCoef& k, const StepArgs& a, int mode, int cfg, int zchunk,
                          hipStream_t s, const FusedSparse& fs);
hipError_t launch_step_hi(const Layout& L, const StencilCoef& k, const StepArgs& a, int mode, int cfg, int zchunk,
                          hipStream_t s, const FusedSparse& fs);

int num_tile_cfgs(int ndim) { return ndim == 3 ? 6 : 2; }

// 3-D workgroup shapes: cfg 0..5 = 64x16, 64x8, 64x32, 64x16, 128x8, 128x16
// points (x by y) per tile; 2-D: cfg 0 = 4 waves, 1 = 1 wave per block.
int tile_rows(int ndim, int cfg) {
    if (ndim == 3) {
        static const int rows[6] = {16, 8, 32, 16, 8, 16};
        return rows[(cfg >= 0 && cfg < 6) ? cfg : 3];
    }
    return cfg == 0 ? 4 : 1;
}

int tile_cols(int ndim, int cfg) { return (ndim == 3 && (cfg == 4 || cfg == 5)) ? 128 : 64; }

hipError_t launch_step(const Layout& L, const StencilCoef& k, const StepArgs& a, int mode, int cfg, int zchunk,
                       hipStream_t s, const FusedSparse* fused) {
    if (zchunk < 1 || cfg < 0 || cfg >= num_tile_cfgs(L.ndim) || mode < 0 || mode > kStepSaveT)
        return hipErrorInvalidValue;
    const FusedSparse none{};
    const FusedSparse& fs = fused ? *fused : none;
    // fused point operators: sampling of the input (any mode); injection into
    // the output of a plain step, or of a save-t step together with t (its
    // second output), at most kFuseMaxNodes nodes
    if (fused) {
        const bool inj = fs.inj.nrows > 0;
        const bool ok_inj = !inj || (fs.inj_zyx && fs.inj.field == a.out && fs.inj.nrows <= kFuseMaxNodes &&
                                     !fs.inj.usnap &&
                                     ((mode == kStepPlain && !fs.inj.grad) || (mode == kStepSaveT && fs.inj.grad == a.grad)));
        const bool ok_smp = fs.smp.npts == 0 || (fs.smp.npts > 0 && fs.smp.field == a.uc);
        if (!ok_inj || !ok_smp || fs.inj.nrows < 0) return hipErrorInvalidValue;
    }
    // a workgroup's slab (zchunk + 2M planes) must be addressable with 31-bit
    // byte offsets; tiling never changes results, so shorten the chunk if not
    const int64_t max_planes = 0x7FFFFFF0ll / (4 * L.sz);
    if (max_planes < 2 * L.half + 2) return hipErrorInvalidValue;
    if (zchunk > max_planes - 2 * L.half - 1) zchunk = (int)(max_planes - 2 * L.half - 1);
    if (L.half >= 1 && L.half <= 4) return launch_step_lo(L, k, a, mode, cfg, zchunk, s, fs);
    if (L.half >= 5 && L.half <= 8) return launch_step_hi(L, k, a, mode, cfg, zchunk, s, fs);
    return hipErrorInvalidValue;
}

}  // namespace awe
