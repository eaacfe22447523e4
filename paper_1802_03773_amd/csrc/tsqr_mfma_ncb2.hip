// Instantiation of the float32 matrix-core tall-skinny QR for 2 column block(s) of 16
// (tiles of 64 rows per leaf wave).
#include "tsqr_mfma.hpp"

namespace qrk {

template <int NCB>
hipError_t launch_tsqr_mfma_n(const float* X, int64_t ldx, int64_t nrows, int L, int64_t rows_per_leaf,
                              int nleaves, const double* dB, double sqrt_lam, float* slots,
                              int* counters, float* Rout, hipStream_t st);

template <>
hipError_t launch_tsqr_mfma_n<2>(const float* X, int64_t ldx, int64_t nrows, int L,
                                 int64_t rows_per_leaf, int nleaves, const double* dB,
                                 double sqrt_lam, float* slots, int* counters, float* Rout,
                                 hipStream_t st) {
  return launch_tsqr_mfma_ncb<2, 4>(X, ldx, nrows, L, rows_per_leaf, nleaves, dB, sqrt_lam, slots,
                                      counters, Rout, st);
}

}  // namespace qrk
