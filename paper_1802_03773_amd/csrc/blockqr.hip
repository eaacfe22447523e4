// Per-block Householder QR of the block-diagonal part and the in-place application of
// Q_i^T to the coupled columns (QRkit Sections 4.1 and 4.2; damping rows placed below
// each block as in the Backtrack LM of Section 5.2), for every block of a batch.
//
// One wave64 per block, blocks of all problems in one grid-stride launch.  Lane j < n owns
// column j of [A_i; sqrt(lam) D_i]; every lane owns coupled columns lane and lane+64 of
// [B_i | b_i; 0 | 0] (b is column nB).  All rows of a block live in registers (ROWS >= m_i +
// n), so Q_i^T is applied without any cross-lane reduction: each Householder vector is
// broadcast once through LDS and each lane updates its own columns.  B_i rows are read with
// consecutive lanes on consecutive columns (coalesced) and the reduced rows are written the
// same way, into the problem's slice of the reduced-row buffer.  blk_prob == nullptr: a
// single problem.  This kernel, with n known only at run time, factors the blocks with fewer
// rows than columns; blocks with m_i >= n go to the kernels with compile-time n.  One launch
// per block class: the blocks of a class are listed in blk_list[begin, begin + count) (or
// are begin .. begin + count - 1 when the list is null).
#include "blockqr.hpp"
#include "qrk_batch.hpp"
#include "qrk_launch.hpp"
#include "block_classes.hpp"

namespace qrk {

template <typename T, int ROWS, int SLOTS>
__global__ void __launch_bounds__(256)
k_blockqr(const int32_t* __restrict__ blk_list, int64_t begin, int64_t count, int n,
          const ProbDesc* __restrict__ probs, const int32_t* __restrict__ blk_prob,
          const int64_t* __restrict__ row_off, const T* __restrict__ A, const T* __restrict__ B,
          const int32_t* __restrict__ cam, const T* __restrict__ bvec, const double* __restrict__ d,
          const double* __restrict__ lam, T* __restrict__ Rblk, T* __restrict__ Sc, T* __restrict__ Red,
          BqrPrologue pro) {
  bqr_prologue<256>(pro);
  __shared__ T vbuf[4][ROWS];
  __shared__ T tbuf[4];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t it = (int64_t)blockIdx.x * 4 + wv; it < count; it += nwaves) {
    const int64_t blk = blk_list ? (int64_t)blk_list[begin + it] : begin + it;
    const int pi = blk_prob == nullptr ? 0 : __builtin_amdgcn_readfirstlane(blk_prob[blk]);
    const ProbDesc& P = probs[pi];
    const int64_t r0 = row_off[blk];
    const int m = (int)(row_off[blk + 1] - r0);
    const int64_t lb = blk - P.koff;
    const int64_t rl = r0 - P.moff;
    const int64_t ldr = P.ldr;
    T* red = Red + P.redoff + rl * ldr;
    block_qr_wave<T, ROWS, SLOTS>(n, P.nB, m, A + r0 * n, B + P.boff + rl * P.ldb, P.ldb, bvec + r0,
                                  d + P.noff + lb * n, sqrt(pro.lam_out ? pro.lam_val : lam[pi]), Rblk + blk * n * n,
                                  Sc + P.soff + lb * n * P.L, vbuf[wv], &tbuf[wv], lane,
                                  [&](int r, int col, T val) { red[r * ldr + col] = val; }, cam ? cam + r0 : nullptr);
  }
}

template <typename T>
hipError_t launch_blockqr(const int32_t* blk_list, int64_t begin, int64_t count, int cls, int n, int probs_count,
                          const ProbDesc* probs, const int32_t* blk_prob, const int64_t* row_off, const T* A,
                          const T* B, const int32_t* cam, const T* b, const double* d, const double* lam, T* Rblk, T* Sc, T* Red,
                          const BqrPrologue& pro, const QKeep& qk, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int32_t* bp = probs_count == 1 ? nullptr : blk_prob;
  const int rows = block_class_rows(cls), slots = block_class_slots(cls);
  if (!block_class_short(cls)) {
    switch (n) {
#define QRK_N(NN) \
  case NN:        \
    return launch_blockqr_n<T, NN>(blk_list, begin, count, rows, slots, probs, bp, row_off, A, B, cam, b, d, lam, Rblk, Sc, Red, pro, qk, st);
      QRK_N(1) QRK_N(2) QRK_N(3) QRK_N(4) QRK_N(5) QRK_N(6) QRK_N(7) QRK_N(8)
#undef QRK_N
      default:
        return hipErrorInvalidValue;
    }
  }
  // blocks with fewer rows than columns: run-time n, 16 register rows (their reflectors are not
  // kept: the handle refuses a stored Q when it has such blocks)
  if (qk.vd) return hipErrorInvalidValue;
  const int grid = (int)((count + 3) / 4 < 2048 ? (count + 3) / 4 : 2048);
  if (slots == 1)
    hipLaunchKernelGGL((k_blockqr<T, 16, 1>), dim3(grid), dim3(256), 0, st, blk_list, begin, count, n, probs, bp,
                       row_off, A, B, cam, b, d, lam, Rblk, Sc, Red, pro);
  else
    hipLaunchKernelGGL((k_blockqr<T, 16, 2>), dim3(grid), dim3(256), 0, st, blk_list, begin, count, n, probs, bp,
                       row_off, A, B, cam, b, d, lam, Rblk, Sc, Red, pro);
  return hipGetLastError();
}

#define QRK_INST(T)                                                                                   \
  template hipError_t launch_blockqr<T>(const int32_t*, int64_t, int64_t, int, int, int, const ProbDesc*, \
                                        const int32_t*, const int64_t*, const T*, const T*, const int32_t*, \
                                        const T*,                                                           \
                                        const double*, const double*, T*, T*, T*, const BqrPrologue&,       \
                                        const QKeep&, hipStream_t);
QRK_INST(float)
QRK_INST(double)
#undef QRK_INST

}  // namespace qrk
