// Kernel instances for float, lane shapes: 8x8 4x8 13x8 16x8 7x16.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_BOTH(float, 8, 8)
HJ_INSTANTIATE_BOTH(float, 4, 8)
HJ_INSTANTIATE_BOTH(float, 13, 8)
HJ_INSTANTIATE_BOTH(float, 16, 8)
HJ_INSTANTIATE_BOTH(float, 7, 16)
