// Instantiation of the compile-time-width banded kernels (W = 1 .. 15) for double.
#include "banded_w.hpp"

namespace qrk {

template hipError_t launch_bgivens_w<double>(int, int64_t, int64_t, int, const int32_t*, const double*, const double*,
                                           const double*, const double*, double*, double*, double*, double*, int*, hipStream_t);
template hipError_t launch_bsweep_w<double>(int, int, int64_t, int, const double*, const double*, const double*,
                                          const double*, double*, int*, hipStream_t);

template hipError_t launch_bapply_w<double>(int, int64_t, int64_t, int, const int32_t*, const double*, const double*,
                                          const double*, double*, hipStream_t);

}  // namespace qrk
