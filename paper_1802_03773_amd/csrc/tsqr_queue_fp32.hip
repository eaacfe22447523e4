// Instantiations of the persistent float32 leaf launch (k_tsqr_queue, tsqr_mfma.hpp) with
// fp32 trailing updates, with and without the stored Q.
#include "tsqr_mfma.hpp"

namespace qrk {

template <bool BF>
hipError_t launch_tsqr_queue(int nitems, const int32_t* leaf_prob, const int32_t* leaf_idx, const ProbDesc* probs,
                             int n, const float* Red, const double* d, const double* lam, float* slots, int* counters,
                             int* qhead, float* RB, float* qt, float* qn, int grid, hipStream_t st);

template <>
hipError_t launch_tsqr_queue<false>(int nitems, const int32_t* leaf_prob, const int32_t* leaf_idx, const ProbDesc* probs,
                                 int n, const float* Red, const double* d, const double* lam, float* slots,
                                 int* counters, int* qhead, float* RB, float* qt, float* qn, int grid,
                                 hipStream_t st) {
  if (qt != nullptr)
    hipLaunchKernelGGL((k_tsqr_queue<false, true>), dim3((unsigned)grid), dim3(256), 0, st, nitems, leaf_prob, leaf_idx,
                       probs, n, Red, d, lam, slots, counters, qhead, RB, qt, qn);
  else
    hipLaunchKernelGGL((k_tsqr_queue<false, false>), dim3((unsigned)grid), dim3(256), 0, st, nitems, leaf_prob, leaf_idx,
                       probs, n, Red, d, lam, slots, counters, qhead, RB, qt, qn);
  return hipGetLastError();
}

}  // namespace qrk
