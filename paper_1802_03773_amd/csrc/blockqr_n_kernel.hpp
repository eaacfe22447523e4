// Kernel and launcher of the per-block QR with compile-time block width N (one
// instantiation per N, compiled in its own translation unit).
#pragma once

#include "blockqr_n.hpp"
#include "qrk_batch.hpp"

namespace qrk {

// One wave per block of the class list blk_list[begin, begin + count) (or blocks begin ..
// begin + count - 1 when the list is null), four blocks per workgroup, no grid-stride loop
// (so the kernel arguments are dead once the block's pointers are formed, which keeps the
// scalar registers for the reflector broadcasts); blk_prob == nullptr: a single problem.
// CAM: B holds camera rows (row stride ldb = the camera width) and cam the camera of every row
// (indexed by row, like A).
template <typename T, int N, int ROWS, int SLOTS, bool CAM>
__global__ void __launch_bounds__(256)
k_blockqr_n(const int32_t* __restrict__ blk_list, int64_t begin, int64_t count,
            const ProbDesc* __restrict__ probs, const int32_t* __restrict__ blk_prob,
            const int64_t* __restrict__ row_off, const T* __restrict__ A, const T* __restrict__ B,
            const int32_t* __restrict__ cam, const T* __restrict__ bvec, const double* __restrict__ d, const double* __restrict__ lam,
            T* __restrict__ Rblk, T* __restrict__ Sc, T* __restrict__ Red, BqrPrologue pro, QKeep qk) {
  bqr_prologue<256>(pro);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t it = (int64_t)blockIdx.x * 4 + wv;
  if (it >= count) return;
  const int64_t blk = blk_list ? (int64_t)blk_list[begin + it] : begin + it;
  const int pi = blk_prob ? blk_prob[blk] : 0;
  const ProbDesc& P = probs[pi];
  const int64_t r0 = row_off[blk];
  const int m = (int)(row_off[blk + 1] - r0);
  const int64_t lb = blk - P.koff;
  const int64_t rl = r0 - P.moff;
  block_qr_wave_n<T, N, ROWS, SLOTS, CAM>(P.nB, m, (int)P.ldb, (int)P.ldr, A + r0 * N, B + P.boff + rl * P.ldb,
                                     bvec + r0, d + P.noff + lb * N, sqrt(pro.lam_out ? pro.lam_val : lam[pi]),
                                     Rblk + blk * (N * N),
                                     Sc + P.soff + lb * N * P.L, Red + P.redoff + rl * P.ldr, lane,
                                     qk.vd ? static_cast<T*>(qk.vd) + r0 * N : nullptr,
                                     qk.vd ? static_cast<T*>(qk.vp) + blk * (N * N) : nullptr,
                                     qk.vd ? static_cast<T*>(qk.g) + blk * N : nullptr, CAM ? cam + r0 : nullptr);
}

template <typename T, int N>
hipError_t launch_blockqr_n(const int32_t* blk_list, int64_t begin, int64_t count, int rows, int slots,
                            const ProbDesc* probs, const int32_t* blk_prob, const int64_t* row_off, const T* A,
                            const T* B, const int32_t* cam, const T* b, const double* d, const double* lam, T* Rblk, T* Sc, T* Red,
                            const BqrPrologue& pro, const QKeep& qk, hipStream_t st) {
  if ((count + 3) / 4 > 0x7fffffff) return hipErrorInvalidValue;
  dim3 blk(256), grd((unsigned)((count + 3) / 4));
#define QRK_BQRN(R, S)                                                                                      \
  if (cam)                                                                                                 \
    hipLaunchKernelGGL((k_blockqr_n<T, N, R, S, true>), grd, blk, 0, st, blk_list, begin, count, probs,   \
                       blk_prob, row_off, A, B, cam, b, d, lam, Rblk, Sc, Red, pro, qk);                   \
  else                                                                                                     \
    hipLaunchKernelGGL((k_blockqr_n<T, N, R, S, false>), grd, blk, 0, st, blk_list, begin, count, probs,  \
                       blk_prob, row_off, A, B, cam, b, d, lam, Rblk, Sc, Red, pro, qk)
  if (rows == 16) {
    if (slots == 1) { QRK_BQRN(16, 1); } else { QRK_BQRN(16, 2); }
  } else if (rows == 32) {
    if (slots == 1) { QRK_BQRN(32, 1); } else { QRK_BQRN(32, 2); }
  } else if (rows == 64) {
    if (slots == 1) { QRK_BQRN(64, 1); } else { QRK_BQRN(64, 2); }
  } else {
    return hipErrorInvalidValue;
  }
#undef QRK_BQRN
  return hipGetLastError();
}

#define QRK_BQRN_INST(T, N)                                                                             \
  template hipError_t launch_blockqr_n<T, N>(const int32_t*, int64_t, int64_t, int, int, const ProbDesc*, \
                                             const int32_t*, const int64_t*, const T*, const T*,           \
                                             const int32_t*, const T*,                                     \
                                             const double*, const double*, T*, T*, T*, const BqrPrologue&, \
                                             const QKeep&, hipStream_t);

}  // namespace qrk
