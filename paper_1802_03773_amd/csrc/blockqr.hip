// Per-block Householder QR of the block-diagonal part and the in-place application of
// Q_i^T to the coupled columns (QRkit Sections 4.1 and 4.2; damping rows placed below
// each block as in the Backtrack LM of Section 5.2).
//
// One wave64 per block.  Lane j < n owns column j of [A_i; sqrt(lam) D_i]; every lane
// owns coupled columns lane and lane+64 of [B_i | b_i; 0 | 0] (b is column nB).  All
// rows of a block live in registers (ROWS >= m_i + n), so Q_i^T is applied without any
// cross-lane reduction: each Householder vector is broadcast once through LDS and each
// lane updates its own columns.  B_i rows are read with consecutive lanes on consecutive
// columns (coalesced) and the reduced rows are written the same way.
#include "blockqr.hpp"
#include "qrk_launch.hpp"

namespace qrk {

template <typename T, int ROWS, int SLOTS>
__global__ void __launch_bounds__(256)
k_blockqr(int64_t K, int n, int nB, const int64_t* __restrict__ row_off,
          const T* __restrict__ A, const T* __restrict__ B, int64_t ldb,
          const T* __restrict__ bvec, const double* __restrict__ d, double sqrt_lam,
          T* __restrict__ Rblk, T* __restrict__ Sc, T* __restrict__ Red, int64_t ldr) {
  __shared__ T vbuf[4][ROWS];
  __shared__ T tbuf[4];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t blk = (int64_t)blockIdx.x * 4 + wv; blk < K; blk += nwaves) {
    const int64_t r0 = row_off[blk];
    block_qr_wave<T, ROWS, SLOTS>(blk, n, nB, row_off, A, B, ldb, bvec, d, sqrt_lam, Rblk, Sc, vbuf[wv],
                                  &tbuf[wv], lane,
                                  [&](int r, int col, T val) { Red[(r0 + r) * ldr + col] = val; });
  }
}

template <typename T>
hipError_t launch_blockqr(int64_t K, int n, int nB, int max_rows, const int64_t* row_off,
                          const T* A, const T* B, int64_t ldb, const T* b, const double* d,
                          double sqrt_lam, T* Rblk, T* Sc, T* Red, int64_t ldr, int grid,
                          hipStream_t st) {
  const int L = nB + 1;
  const int slots = L <= 64 ? 1 : 2;
  dim3 blk(256), grd(grid);
#define QRK_BQR(R, S)                                                                          \
  hipLaunchKernelGGL((k_blockqr<T, R, S>), grd, blk, 0, st, K, n, nB, row_off, A, B, ldb, b, d, \
                     sqrt_lam, Rblk, Sc, Red, ldr)
  if (max_rows <= 16) {
    if (slots == 1) QRK_BQR(16, 1); else QRK_BQR(16, 2);
  } else if (max_rows <= 32) {
    if (slots == 1) QRK_BQR(32, 1); else QRK_BQR(32, 2);
  } else if (max_rows <= 64) {
    if (slots == 1) QRK_BQR(64, 1); else QRK_BQR(64, 2);
  } else {
    return hipErrorInvalidValue;
  }
#undef QRK_BQR
  return hipGetLastError();
}

template hipError_t launch_blockqr<float>(int64_t, int, int, int, const int64_t*, const float*,
                                          const float*, int64_t, const float*, const double*, double,
                                          float*, float*, float*, int64_t, int, hipStream_t);
template hipError_t launch_blockqr<double>(int64_t, int, int, int, const int64_t*, const double*,
                                           const double*, int64_t, const double*, const double*,
                                           double, double*, double*, double*, int64_t, int,
                                           hipStream_t);

}  // namespace qrk
