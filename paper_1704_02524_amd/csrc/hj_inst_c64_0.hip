// FP64 continuation kernels of the FP32 lane shapes 2x1 4x1 2x2 8x1 2x4.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_CONT(2, 1)
HJ_INSTANTIATE_CONT(4, 1)
HJ_INSTANTIATE_CONT(2, 2)
HJ_INSTANTIATE_CONT(8, 1)
HJ_INSTANTIATE_CONT(2, 4)
