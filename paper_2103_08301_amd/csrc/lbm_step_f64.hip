// lbm_step_f64.hip -- step kernels (all schedules, both equations of state) for
// FP64 storage and arithmetic.
#include "lbm_device.hpp"

LBM_DEFINE_STORAGE_LAUNCHERS(f64, CodecF64)
