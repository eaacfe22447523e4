// Blocks of their own widths (QRkit Section 4.1 allows every block its own n_i): the handle
// runs the blocks at n = max n_i columns, block i's columns past n_i being zero in J with unit
// damping, and these kernels move A, d and p between the caller's layout (block i's values
// and unknowns at their own offsets, n_i per row) and the handle's (n per block).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrk {

// A at n columns (zeros past n_i) and d at n per block (1 past n_i), then the dense part's d;
// one thread per block, threads K .. K + nB - 1 for the dense part's d.
template <typename T>
__global__ void __launch_bounds__(256)
k_ragged_in(int64_t K, int n, int nB, const int64_t* __restrict__ row_off, const int32_t* __restrict__ ncol,
            const int64_t* __restrict__ aoff, const int64_t* __restrict__ poff, const T* __restrict__ Au,
            const double* __restrict__ du, T* __restrict__ Ap, double* __restrict__ dp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < K) {
    const int ni = ncol[t];
    const int64_t r0 = row_off[t], r1 = row_off[t + 1];
    const T* a = Au + aoff[t];
    for (int64_t r = r0; r < r1; ++r)
      for (int c = 0; c < n; ++c) Ap[r * n + c] = c < ni ? a[(r - r0) * ni + c] : T(0);
    for (int c = 0; c < n; ++c) dp[t * n + c] = c < ni ? du[poff[t] + c] : 1.0;
  } else if (t < K + nB) {
    const int64_t j = t - K;
    dp[K * n + j] = du[poff[K] + j];
  }
}

// p in the caller's layout from the handle's
__global__ void __launch_bounds__(256)
k_ragged_out(int64_t K, int n, int nB, const int32_t* __restrict__ ncol, const int64_t* __restrict__ poff,
             const double* __restrict__ pp, double* __restrict__ pu) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < K) {
    const int ni = ncol[t];
    for (int c = 0; c < ni; ++c) pu[poff[t] + c] = pp[t * n + c];
  } else if (t < K + nB) {
    const int64_t j = t - K;
    pu[poff[K] + j] = pp[K * n + j];
  }
}

template <typename T>
hipError_t launch_ragged_in(int64_t K, int n, int nB, const int64_t* row_off, const int32_t* ncol,
                            const int64_t* aoff, const int64_t* poff, const T* Au, const double* du, T* Ap,
                            double* dp, hipStream_t st) {
  const int64_t threads = K + nB;
  hipLaunchKernelGGL((k_ragged_in<T>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, K, n, nB, row_off,
                     ncol, aoff, poff, Au, du, Ap, dp);
  return hipGetLastError();
}

hipError_t launch_ragged_out(int64_t K, int n, int nB, const int32_t* ncol, const int64_t* poff, const double* pp,
                             double* pu, hipStream_t st) {
  const int64_t threads = K + nB;
  hipLaunchKernelGGL(k_ragged_out, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, K, n, nB, ncol, poff,
                     pp, pu);
  return hipGetLastError();
}

template hipError_t launch_ragged_in<float>(int64_t, int, int, const int64_t*, const int32_t*, const int64_t*,
                                            const int64_t*, const float*, const double*, float*, double*,
                                            hipStream_t);
template hipError_t launch_ragged_in<double>(int64_t, int, int, const int64_t*, const int32_t*, const int64_t*,
                                             const int64_t*, const double*, const double*, double*, double*,
                                             hipStream_t);

}  // namespace qrk
