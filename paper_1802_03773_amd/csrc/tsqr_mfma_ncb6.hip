// Instantiation of the float32 matrix-core tall-skinny QR for 6 column block(s) of 16
// (tiles of 128 rows per leaf wave; fp32 or BF16x3 trailing updates).
#include "tsqr_mfma.hpp"

namespace qrk {

template <int NCB>
hipError_t launch_tsqr_mfma_n(bool bf16x3, int leaf_begin, int nleaves_cls, const int32_t* leaf_prob, const int32_t* leaf_idx,
                              const ProbDesc* probs, int n, const float* Red, const double* d, const double* lam,
                              float* slots, int* counters, float* RB, const QStore& qs, hipStream_t st);

template <>
hipError_t launch_tsqr_mfma_n<6>(bool bf16x3, int leaf_begin, int nleaves_cls, const int32_t* leaf_prob,
                                 const int32_t* leaf_idx, const ProbDesc* probs, int n, const float* Red,
                                 const double* d, const double* lam, float* slots, int* counters, float* RB,
                                 const QStore& qs, hipStream_t st) {
  return launch_tsqr_mfma_ncb<6, 8>(bf16x3, leaf_begin, nleaves_cls, leaf_prob, leaf_idx, probs, n, Red, d, lam, slots,
                                     counters, RB, qs, st);
}

}  // namespace qrk
