// Dispatch of the float32 tall-skinny QR on the matrix cores (see tsqr_mfma.hpp).  Dense parts
// wider than kQueueNCB column blocks: a launch per column-block count.  Up to kQueueNCB: one
// launch of that width's kernel when the batch has a single such width (a single problem, or a
// batch of equal widths), else one persistent queue launch over all of them
// (tsqr_queue_*.hip).  The queue calls each width's body as a function, which costs that body
// registers (the single-width headline: 0.448 -> 0.524 ms), but lets the narrow problems' leaves
// fill the SIMDs the wide ones leave idle (512-problem ragged batch: 14.0 -> 11.7 ms).
#include <algorithm>

#include "qrk_launch.hpp"
#include "tsqr_mfma.hpp"

namespace qrk {

// One instantiation per column-block count lives in tsqr_mfma_ncb<N>.hip.
template <int NCB>
hipError_t launch_tsqr_mfma_n(bool bf16x3, int leaf_begin, int nleaves_cls, const int32_t* leaf_prob, const int32_t* leaf_idx,
                              const ProbDesc* probs, int n, const float* Red, const double* d, const double* lam,
                              float* slots, int* counters, float* RB, const QStore& qs, hipStream_t st);

__global__ void k_zero_ints(int* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_zero_ints(int* p, int64_t n, hipStream_t st) {
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

int tsqr_mfma_slot_floats(int L) {
  const int ncb = (L + 15) / 16;
  return ncb * (ncb + 1) / 2 * 256;
}

template <bool BF>
hipError_t launch_tsqr_queue(int nitems, const int32_t* leaf_prob, const int32_t* leaf_idx, const ProbDesc* probs,
                             int n, const float* Red, const double* d, const double* lam, float* slots, int* counters,
                             int* qhead, float* RB, const QStore& qs, int grid, hipStream_t st);

hipError_t launch_tsqr_mfma(bool bf16x3, const int* cls_begin, const int* cls_count, int queue_begin, bool use_queue,
                            int cus,
                            const int32_t* leaf_prob, const int32_t* leaf_idx, const ProbDesc* probs, int n,
                            const float* Red, const double* d, const double* lam, float* slots, int* counters,
                            int64_t nctr, int* qhead, float* RB, const QStore& qs, hipStream_t st) {
  // the arrival counters and the queue head are cleared by the factor call's first per-block
  // QR launch
  if (nctr < 1) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  int widths = 0;
  for (int c = kQueueNCB; c >= 1; --c) widths += cls_count[c] > 0;
  const bool queue = use_queue && widths > 1;
  const int own_last = queue ? kQueueNCB + 1 : 1;  // classes >= own_last: a launch each
  for (int c = 8; c >= own_last && e == hipSuccess; --c) {  // widest (slowest) problems first
    const int b = cls_begin[c], k = cls_count[c];
    if (k == 0) continue;
#define QRK_TS(N)                                                                                            \
  case N:                                                                                                    \
    e = launch_tsqr_mfma_n<N>(bf16x3, b, k, leaf_prob, leaf_idx, probs, n, Red, d, lam, slots, counters, RB, qs,     \
                              st);                                                                          \
    break;
    switch (c) { QRK_TS(1) QRK_TS(2) QRK_TS(3) QRK_TS(4) QRK_TS(5) QRK_TS(6) QRK_TS(7) QRK_TS(8) }
#undef QRK_TS
  }
  int nq = 0;
  for (int c = kQueueNCB; c >= 1; --c) nq += cls_count[c];
  if (e == hipSuccess && queue) {
    // one workgroup of four waves per compute unit holds a wave on every SIMD (the leaf bodies
    // need the whole register file)
    const int grid = std::max(1, std::min((nq + 3) / 4, cus));
    e = bf16x3 ? launch_tsqr_queue<true>(nq, leaf_prob + queue_begin, leaf_idx + queue_begin, probs, n, Red, d, lam,
                                         slots, counters, qhead, RB, qs, grid, st)
               : launch_tsqr_queue<false>(nq, leaf_prob + queue_begin, leaf_idx + queue_begin, probs, n, Red, d, lam,
                                          slots, counters, qhead, RB, qs, grid, st);
  }
  return e;
}

}  // namespace qrk
