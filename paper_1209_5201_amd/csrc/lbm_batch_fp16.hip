// Batched persistent small-case kernel, FP16 deviation storage (all velocity sets).
#define LBM_DEFINE_BATCH
#include "lbm_device.hpp"

template hipError_t lbm::dev::batch_launch<lbm::dev::CFP16, false, 7>(const lbm::CaseDesc*, int,
                                                              lbm::CaseOut*, hipStream_t);
