// Kernel instances for double, lane shapes: 3x4 4x4 8x2 8x4.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_BOTH(double, 3, 4)
HJ_INSTANTIATE_BOTH(double, 4, 4)
HJ_INSTANTIATE_BOTH(double, 8, 2)
HJ_INSTANTIATE_BOTH(double, 8, 4)
