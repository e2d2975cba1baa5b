// Kernel instances for double, lane shapes: 8x8 4x8 13x8 16x8 7x16.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_BOTH(double, 8, 8)
HJ_INSTANTIATE_BOTH(double, 4, 8)
HJ_INSTANTIATE_BOTH(double, 13, 8)
HJ_INSTANTIATE_BOTH(double, 16, 8)
HJ_INSTANTIATE_BOTH(double, 7, 16)
