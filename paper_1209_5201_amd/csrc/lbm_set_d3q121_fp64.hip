// Kernels of the D3Q121 velocity set with FP64 storage.
#define LBM_DEFINE_SET_OPS
#include "lbm_device.hpp"

template struct lbm::dev::SetOps<lbm::D3Q121, lbm::dev::CF64, false>;
