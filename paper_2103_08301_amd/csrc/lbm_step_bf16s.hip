// lbm_step_bf16s.hip -- step kernels (all schedules, both equations of state) for
// BF16 storage of f - w rho0, FP32 arithmetic.
#include "lbm_device.hpp"

LBM_DEFINE_STORAGE_LAUNCHERS(bf16s, CodecBF16S)
