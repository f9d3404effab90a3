// lbm_step_f16s.hip -- step kernels (all schedules, both equations of state) for
// FP16 storage of f - w rho0, FP32 arithmetic.
#include "lbm_device.hpp"

LBM_DEFINE_STORAGE_LAUNCHERS(f16s, CodecF16S)
