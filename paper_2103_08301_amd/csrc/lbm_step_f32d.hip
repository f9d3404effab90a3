// lbm_step_f32d.hip -- step kernels (all schedules, both equations of state) for
// FP32 storage, FP64 arithmetic.
#include "lbm_device.hpp"

LBM_DEFINE_STORAGE_LAUNCHERS(f32d, CodecF32D)
