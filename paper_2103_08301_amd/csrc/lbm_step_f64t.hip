// lbm_step_f64t.hip -- step kernels of the tangent-linear storage (FP64 value
// and FP64 tangent per population): the tile schedule with 12-row, 8-wave tiles.
#include "lbm_device.hpp"

namespace lbm {
hipError_t launch_step_f64t(const StepArgs& a, int eos, bool emit, hipStream_t s) {
    if (a.schedule != kScheduleTile || a.ty != 12 || a.tile_waves != 8) return hipErrorInvalidValue;
    return eos == LBM_EOS_CS ? launch_tile<CodecF64T, LBM_EOS_CS, 12, 8>(a, emit, s)
                             : launch_tile<CodecF64T, LBM_EOS_PR, 12, 8>(a, emit, s);
}
}  // namespace lbm
