// Tail-continuation kernel instances (FP64), lane shapes: 2x1 4x1 2x2 8x1 2x4.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_RESUME(2, 1)
HJ_INSTANTIATE_RESUME(4, 1)
HJ_INSTANTIATE_RESUME(2, 2)
HJ_INSTANTIATE_RESUME(8, 1)
HJ_INSTANTIATE_RESUME(2, 4)
