// Dispatch of the float32 tall-skinny QR on the matrix cores (see tsqr_mfma.hpp): one launch
// per column-block count present in the batch.
#include "qrk_launch.hpp"
#include "tsqr_mfma.hpp"

namespace qrk {

// One instantiation per column-block count lives in tsqr_mfma_ncb<N>.hip.
template <int NCB>
hipError_t launch_tsqr_mfma_n(bool bf16x3, int leaf_begin, int nleaves_cls, const int32_t* leaf_prob, const int32_t* leaf_idx,
                              const ProbDesc* probs, int n, const float* Red, const double* d, const double* lam,
                              float* slots, int* counters, float* RB, hipStream_t st);

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

hipError_t launch_tsqr_mfma(bool bf16x3, const int* cls_begin, const int* cls_count, const int32_t* leaf_prob,
                            const int32_t* leaf_idx, const ProbDesc* probs, int n, const float* Red,
                            const double* d, const double* lam, float* slots, int* counters, int64_t nctr,
                            float* RB, hipStream_t st) {
  // the arrival counters are cleared by the factor call's first per-block QR launch
  if (nctr < 1) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  for (int c = 8; c >= 1 && e == hipSuccess; --c) {  // widest (slowest) problems first
    const int b = cls_begin[c], k = cls_count[c];
    if (k == 0) continue;
#define QRK_TS(N)                                                                                            \
  case N:                                                                                                    \
    e = launch_tsqr_mfma_n<N>(bf16x3, b, k, leaf_prob, leaf_idx, probs, n, Red, d, lam, slots, counters, RB, st); \
    break;
    switch (c) { QRK_TS(1) QRK_TS(2) QRK_TS(3) QRK_TS(4) QRK_TS(5) QRK_TS(6) QRK_TS(7) QRK_TS(8) }
#undef QRK_TS
  }
  return e;
}

}  // namespace qrk
