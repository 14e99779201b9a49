// Batched persistent small-case kernel, FP32 storage with FP64 arithmetic (D3Q121).
#define LBM_DEFINE_BATCH
#include "lbm_device.hpp"

template hipError_t lbm::dev::batch_launch<lbm::dev::CF32S, false, 4>(const lbm::CaseDesc*, int,
                                                              lbm::CaseOut*, hipStream_t);
