// Batched persistent small-case kernel, BF16 storage (all velocity sets), body-force variant.
#define LBM_DEFINE_BATCH
#include "lbm_device.hpp"

template hipError_t lbm::dev::batch_launch<lbm::dev::CBF16, true>(const lbm::CaseDesc*, int,
                                                       lbm::CaseOut*, hipStream_t);
