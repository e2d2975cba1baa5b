// Kernel instances for float with linear drift (matrix-core layout), NPL 4, 8, 16.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_DRIFT(float, 4)
HJ_INSTANTIATE_DRIFT(float, 8)
HJ_INSTANTIATE_DRIFT(float, 16)
