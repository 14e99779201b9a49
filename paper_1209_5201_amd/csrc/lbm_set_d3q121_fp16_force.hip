// Kernels of the D3Q121 velocity set with FP16 deviation storage, body-force variant.
#define LBM_DEFINE_SET_OPS
#include "lbm_device.hpp"

template struct lbm::dev::SetOps<lbm::D3Q121, lbm::dev::CFP16, true>;
