// lbm_step_f32s.hip -- step kernels (all schedules, both equations of state) for
// FP32 storage of f - w rho0, FP32 arithmetic.
#include "lbm_device.hpp"

LBM_DEFINE_STORAGE_LAUNCHERS(f32s, CodecF32S)
