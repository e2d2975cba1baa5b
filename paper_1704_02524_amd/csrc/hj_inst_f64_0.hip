// Kernel instances for double, lane shapes: 2x1 4x1 2x2 8x1 2x4.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_BOTH(double, 2, 1)
HJ_INSTANTIATE_BOTH(double, 4, 1)
HJ_INSTANTIATE_BOTH(double, 2, 2)
HJ_INSTANTIATE_BOTH(double, 8, 1)
HJ_INSTANTIATE_BOTH(double, 2, 4)

template hipError_t hj::launch_select<double>(int64_t, int, int, int, const double*, const int32_t*,
                                              const double*, double*, double*, int32_t*,
                                              hipStream_t);

template hipError_t hj::launch_select_batched<double>(const hj::InstDesc<double>*, int, int64_t, int, int,
                                                     const double*, const int32_t*, const double*,
                                                     hipStream_t);
template hipError_t hj::launch_scatter_diag<double>(const hj::InstDesc<double>*, int, int64_t, int,
                                                   hj::SlotOut<double>, hipStream_t);
