// Launch of the pipelined dense-part merge tree (see tsqr_tree.hpp), one instantiation per
// column-block count up to kTreeMaxNCB = 8 (the kept panels of a wave fit in LDS four waves at a
// time up to 7 column blocks, 150.5 KiB per workgroup at 7; three at 8, 138 KiB).
#include "qrk_launch.hpp"
#include "tsqr_tree.hpp"

namespace qrk {

hipError_t launch_tsqr_tree(int ncb, const ProbDesc* probs, const int32_t* node_l, const int32_t* node_r,
                            int nnodes, float* slots, int* flags, float* RB, int* status, const QStore& qs,
                            hipStream_t st) {
  if (nnodes < 1) return hipSuccess;
  switch (ncb) {
#define QRK_TREE(N)                                                                                          \
  case N: {                                                                                                  \
    constexpr int wpg = tree_waves(N);                                                                       \
    const dim3 grid((unsigned)((nnodes + wpg - 1) / wpg)), blk(64 * wpg);                                    \
    if (qs.qn)                                                                                               \
      hipLaunchKernelGGL((k_tsqr_tree_keep<N>), grid, blk, 0, st, probs, node_l, node_r, nnodes, slots, flags, \
                         RB, status, qs);                                                                    \
    else                                                                                                     \
      hipLaunchKernelGGL((k_tsqr_tree<N>), grid, blk, 0, st, probs, node_l, node_r, nnodes, slots, flags, RB,  \
                         status);                                                                            \
    break;                                                                                                   \
  }
    QRK_TREE(1) QRK_TREE(2) QRK_TREE(3) QRK_TREE(4) QRK_TREE(5) QRK_TREE(6) QRK_TREE(7) QRK_TREE(8)
#undef QRK_TREE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qrk
