// Dispatch of the float32 tall-skinny QR on the matrix cores (see tsqr_mfma.hpp).
#include "qrk_launch.hpp"
#include "tsqr_mfma.hpp"

namespace qrk {

// One instantiation per column-block count lives in tsqr_mfma_ncb<N>.hip.
template <int NCB>
hipError_t launch_tsqr_mfma_n(const float* X, int64_t ldx, int64_t nrows, int L, int64_t rows_per_leaf,
                              int nleaves, const double* dB, double sqrt_lam, float* slots,
                              int* counters, float* Rout, hipStream_t st);

__global__ void k_zero_ints(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

int tsqr_mfma_slot_floats(int L) {
  const int ncb = (L + 15) / 16;
  return ncb * (ncb + 1) / 2 * 256;
}

hipError_t launch_tsqr_mfma(const float* X, int64_t ldx, int64_t nrows, int L, int nleaves,
                            const double* dB, double sqrt_lam, float* slots, int* counters,
                            float* Rout, hipStream_t st) {
  if (L < 1 || L > 128 || nleaves < 1) return hipErrorInvalidValue;
  const int nctr = 2 * nleaves + 2;
  hipLaunchKernelGGL(k_zero_ints, dim3((nctr + 255) / 256), dim3(256), 0, st, counters, nctr);
  int64_t rows_per_leaf = (nrows + nleaves - 1) / nleaves;
  if (rows_per_leaf < 1) rows_per_leaf = 1;
  switch ((L + 15) / 16) {
    case 1: return launch_tsqr_mfma_n<1>(X, ldx, nrows, L, rows_per_leaf, nleaves, dB, sqrt_lam, slots, counters, Rout, st);
    case 2: return launch_tsqr_mfma_n<2>(X, ldx, nrows, L, rows_per_leaf, nleaves, dB, sqrt_lam, slots, counters, Rout, st);
    case 3: return launch_tsqr_mfma_n<3>(X, ldx, nrows, L, rows_per_leaf, nleaves, dB, sqrt_lam, slots, counters, Rout, st);
    case 4: return launch_tsqr_mfma_n<4>(X, ldx, nrows, L, rows_per_leaf, nleaves, dB, sqrt_lam, slots, counters, Rout, st);
    case 5: return launch_tsqr_mfma_n<5>(X, ldx, nrows, L, rows_per_leaf, nleaves, dB, sqrt_lam, slots, counters, Rout, st);
    case 6: return launch_tsqr_mfma_n<6>(X, ldx, nrows, L, rows_per_leaf, nleaves, dB, sqrt_lam, slots, counters, Rout, st);
    case 7: return launch_tsqr_mfma_n<7>(X, ldx, nrows, L, rows_per_leaf, nleaves, dB, sqrt_lam, slots, counters, Rout, st);
    case 8: return launch_tsqr_mfma_n<8>(X, ldx, nrows, L, rows_per_leaf, nleaves, dB, sqrt_lam, slots, counters, Rout, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace qrk
