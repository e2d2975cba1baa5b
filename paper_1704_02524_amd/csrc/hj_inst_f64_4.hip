// Kernel instances for double with linear drift (matrix-core layout), NPL 4, 8, 16.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_DRIFT(double, 4)
HJ_INSTANTIATE_DRIFT(double, 8)
HJ_INSTANTIATE_DRIFT(double, 16)
