// Instantiation of the compile-time-width banded kernels (W = 1 .. 15) for float.
#include "banded_w.hpp"

namespace qrk {

template hipError_t launch_bgivens_w<float>(int, int64_t, int64_t, int, const int32_t*, const float*, const float*,
                                           const double*, const double*, float*, float*, double*, float*, int*, hipStream_t);
template hipError_t launch_bsweep_w<float>(int, int, int64_t, int, const float*, const double*, const float*,
                                          const double*, double*, int*, hipStream_t);

template hipError_t launch_bapply_w<float>(int, int64_t, int64_t, int, const int32_t*, const float*, const float*,
                                          const double*, double*, hipStream_t);

}  // namespace qrk
