// Kernel instances for float, lane shapes: 2x1 4x1 2x2 8x1 2x4.
#include "hj_kernels.hpp"

HJ_INSTANTIATE_BOTH(float, 2, 1)
HJ_INSTANTIATE_BOTH(float, 4, 1)
HJ_INSTANTIATE_BOTH(float, 2, 2)
HJ_INSTANTIATE_BOTH(float, 8, 1)
HJ_INSTANTIATE_BOTH(float, 2, 4)

template hipError_t hj::launch_select<float>(int64_t, int, int, int, const double*, const int32_t*,
                                             const float*, double*, float*, int32_t*,
                                             hipStream_t);

template hipError_t hj::launch_select_batched<float>(const hj::InstDesc<float>*, int, int64_t, int, int,
                                                     const double*, const int32_t*, const float*,
                                                     hipStream_t);
template hipError_t hj::launch_scatter_diag<float>(const hj::InstDesc<float>*, int, int64_t, int,
                                                   hj::SlotOut<float>, hipStream_t);
