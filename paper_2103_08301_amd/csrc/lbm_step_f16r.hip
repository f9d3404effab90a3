// lbm_step_f16r.hip -- step kernels of FP16 storage with stochastic rounding
// (CodecF16R): the tile schedule and batches, one step per launch.
#include "lbm_device.hpp"

namespace lbm {
namespace {
template <int EOS>
hipError_t launch_tile_f16r(const StepArgs& a, bool emit, hipStream_t s) {
    if (a.schedule != kScheduleTile) return hipErrorInvalidValue;
    if (a.tile_waves == 8) {
        switch (a.ty) {
            case 12: return launch_tile<CodecF16R, EOS, 12, 8>(a, emit, s);
            case 20: return launch_tile<CodecF16R, EOS, 20, 8>(a, emit, s);
            case 28: return launch_tile<CodecF16R, EOS, 28, 8>(a, emit, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (a.ty) {
        case 8: return launch_tile<CodecF16R, EOS, 8, 4>(a, emit, s);
        case 12: return launch_tile<CodecF16R, EOS, 12, 4>(a, emit, s);
        case 20: return launch_tile<CodecF16R, EOS, 20, 4>(a, emit, s);
        case 28: return launch_tile<CodecF16R, EOS, 28, 4>(a, emit, s);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_step_f16r(const StepArgs& a, int eos, bool emit, hipStream_t s) {
    return eos == LBM_EOS_CS ? launch_tile_f16r<LBM_EOS_CS>(a, emit, s) : launch_tile_f16r<LBM_EOS_PR>(a, emit, s);
}

hipError_t launch_batch_f16r(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                             int slot, int eos, int ty, int waves, bool emit, hipStream_t s) {
    return launch_batch_c<CodecF16R>(cases, tile_start, ncases, total_tiles, parity, slot, eos, ty, waves, emit, s);
}
}  // namespace lbm
