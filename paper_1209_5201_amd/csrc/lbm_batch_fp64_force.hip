// Batched persistent small-case kernel, FP64 storage (2-D velocity sets), body-force variant.
#define LBM_DEFINE_BATCH
#include "lbm_device.hpp"

template hipError_t lbm::dev::batch_launch<lbm::dev::CF64, true, 3>(const lbm::CaseDesc*, int,
                                                              lbm::CaseOut*, hipStream_t);
