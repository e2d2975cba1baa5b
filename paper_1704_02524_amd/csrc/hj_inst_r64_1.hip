// Tail-continuation kernel instances (FP64), lane shapes: 4x2 5x2 10x1.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_RESUME(4, 2)
HJ_INSTANTIATE_RESUME(5, 2)
HJ_INSTANTIATE_RESUME(10, 1)
