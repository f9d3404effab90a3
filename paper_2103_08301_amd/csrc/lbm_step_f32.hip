// lbm_step_f32.hip -- step kernels (all schedules, both equations of state) for
// FP32 storage and arithmetic.
#include "lbm_device.hpp"

LBM_DEFINE_STORAGE_LAUNCHERS(f32, CodecF32)
