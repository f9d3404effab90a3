// lbm_adjoint.hip -- placeholder
#include "lbm_device.hpp"
