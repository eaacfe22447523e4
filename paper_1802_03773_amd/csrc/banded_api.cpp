// Banded and adjoint entry points (placeholders until their kernels land).
#include "qrkit.h"
#include "qrk_host.hpp"

extern "C" {
qrk_status qrk_create_banded(int64_t, int64_t, int32_t, qrk_dtype, qrk_handle* out) {
  if (out) *out = nullptr;
  return QRK_EINVAL;
}
qrk_status qrk_factor_banded(qrk_handle, const int32_t*, const void*, const void*, const double*,
                             double, void*) {
  return QRK_EINVAL;
}
qrk_status qrk_solve_adjoint(qrk_handle, const double*, const double*, void*, void*, void*, double*,
                             double*, void*) {
  return QRK_EINVAL;
}
qrk_status qrk_colnorms_blockangular(qrk_handle, const void*, const void*, double*, void*) {
  return QRK_EINVAL;
}
}
qrk_status banded_solve(qrk_handle, double*, int, hipStream_t) { return QRK_EINVAL; }
