// Kernel instances for float, lane shapes: 4x2 5x2 10x1.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_BOTH(float, 4, 2)
HJ_INSTANTIATE_BOTH(float, 5, 2)
HJ_INSTANTIATE_BOTH(float, 10, 1)
