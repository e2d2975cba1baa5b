// FP64 continuation kernels of the FP32 linear-drift shapes (NPL 4, 8, 16).
#include "hj_kernels.hpp"

HJ_INSTANTIATE_CONT_DRIFT(4)
HJ_INSTANTIATE_CONT_DRIFT(8)
HJ_INSTANTIATE_CONT_DRIFT(16)
