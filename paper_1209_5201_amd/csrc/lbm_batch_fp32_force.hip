// Batched persistent small-case kernel, FP32 storage (all velocity sets), body-force variant.
#define LBM_DEFINE_BATCH
#include "lbm_device.hpp"

template hipError_t lbm::dev::batch_launch<lbm::dev::CF32, true, 7>(const lbm::CaseDesc*, int,
                                                              lbm::CaseOut*, hipStream_t);
