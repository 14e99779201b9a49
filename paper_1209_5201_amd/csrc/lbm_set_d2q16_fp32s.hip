// Kernels of the D2Q16 velocity set with FP32 storage and FP64 arithmetic.
#define LBM_DEFINE_SET_OPS
#include "lbm_device.hpp"

template struct lbm::dev::SetOps<lbm::D2Q16, lbm::dev::CF32S, false>;
