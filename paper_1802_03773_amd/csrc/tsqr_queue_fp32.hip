// Instantiations of the persistent float32 leaf launch (k_tsqr_queue, tsqr_mfma.hpp) with
// fp32 trailing updates, with and without the stored Q.
#include "tsqr_mfma.hpp"

namespace qrk {

template <bool BF>
hipError_t launch_tsqr_queue(int nitems, const int32_t* leaf_prob, const int32_t* leaf_idx, const ProbDesc* probs,
                             int n, const float* Red, const double* d, const double* lam, float* slots, int* counters,
                             int* qhead, float* RB, const QStore& qs, int grid, hipStream_t st);

template <>
hipError_t launch_tsqr_queue<false>(int nitems, const int32_t* leaf_prob, const int32_t* leaf_idx, const ProbDesc* probs,
                                 int n, const float* Red, const double* d, const double* lam, float* slots,
                                 int* counters, int* qhead, float* RB, const QStore& qs, int grid,
                                 hipStream_t st) {
  if (qs.qt != nullptr)
    hipLaunchKernelGGL((k_tsqr_queue_keep<false>), dim3((unsigned)grid), dim3(256), 0, st, nitems, leaf_prob, leaf_idx,
                       probs, n, Red, d, lam, slots, counters, qhead, RB, qs);
  else
    hipLaunchKernelGGL((k_tsqr_queue<false>), dim3((unsigned)grid), dim3(256), 0, st, nitems, leaf_prob, leaf_idx, probs,
                       n, Red, d, lam, slots, counters, qhead, RB);
  return hipGetLastError();
}

}  // namespace qrk
