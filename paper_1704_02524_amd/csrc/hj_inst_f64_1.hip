// Kernel instances for double, lane shapes: 4x2 5x2 10x1.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_BOTH(double, 4, 2)
HJ_INSTANTIATE_BOTH(double, 5, 2)
HJ_INSTANTIATE_BOTH(double, 10, 1)
