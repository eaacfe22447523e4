// Launch of the pipelined dense-part merge tree (see tsqr_tree.hpp), one instantiation per
// column-block count up to 6 (the kept panels of a wave then fit in LDS four waves at a time).
#include "qrk_launch.hpp"
#include "tsqr_tree.hpp"

namespace qrk {

hipError_t launch_tsqr_tree(int ncb, const ProbDesc* probs, const int32_t* node_l, const int32_t* node_r,
                            int nnodes, float* slots, int* flags, float* RB, int* status, const QStore& qs,
                            hipStream_t st) {
  if (nnodes < 1) return hipSuccess;
  const dim3 grid((unsigned)((nnodes + 3) / 4)), blk(256);
  switch (ncb) {
#define QRK_TREE(N)                                                                                         \
  case N:                                                                                                   \
    if (qs.qn)                                                                                              \
      hipLaunchKernelGGL((k_tsqr_tree_keep<N>), grid, blk, 0, st, probs, node_l, node_r, nnodes, slots, flags,  \
                         RB, status, qs);                                                                   \
    else                                                                                                    \
      hipLaunchKernelGGL((k_tsqr_tree<N>), grid, blk, 0, st, probs, node_l, node_r, nnodes, slots, flags, RB, \
                         status);                                                                           \
    break;
    QRK_TREE(1) QRK_TREE(2) QRK_TREE(3) QRK_TREE(4) QRK_TREE(5) QRK_TREE(6)
#undef QRK_TREE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qrk
