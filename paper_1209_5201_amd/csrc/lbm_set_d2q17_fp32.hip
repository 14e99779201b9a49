// Kernels of the D2Q17 velocity set with FP32 storage.
#define LBM_DEFINE_SET_OPS
#include "lbm_device.hpp"

template struct lbm::dev::SetOps<lbm::D2Q17, lbm::dev::CF32, false>;
