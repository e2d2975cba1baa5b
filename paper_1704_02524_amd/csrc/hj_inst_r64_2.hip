// Tail-continuation kernel instances (FP64), lane shapes: 3x4 4x4 8x2 8x4.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_RESUME(3, 4)
HJ_INSTANTIATE_RESUME(4, 4)
HJ_INSTANTIATE_RESUME(8, 2)
HJ_INSTANTIATE_RESUME(8, 4)
