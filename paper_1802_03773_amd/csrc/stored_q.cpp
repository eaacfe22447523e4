// Stored Q entry points: the reflectors a float32 block-angular factorisation keeps when asked
// (qrk_set_keep_q), and Q^T applied to new right-hand sides (qrk_apply_qt, qrk_solve_qt).  The
// kernels are in stored_q.hip; the storage layout is set with the dense-part leaves.
#include <hip/hip_runtime.h>

#include "block_classes.hpp"
#include "qrk_host.hpp"
#include "qrk_launch.hpp"
#include "qrkit.h"

using namespace qrk;

namespace {

hipError_t apply(qrk_handle h, const void* b, double* c, hipStream_t st) {
  return launch_apply_qt(blockangular_view(h), h->cls_begin, h->cls_count, h->leaf_prob, h->leaf_idx,
                         static_cast<const float*>(b), h->qk, QStore{h->q_tiles, h->q_nodes, h->qoff_d}, h->q_xr,
                         h->q_u, h->counters, h->nctr, c, st);
}

}  // namespace

extern "C" {

qrk_status qrk_set_keep_q(qrk_handle h, int32_t keep) {
  if (!h) return QRK_EINVAL;
  if (keep) {
    if (h->kind != KIND_BLOCKANGULAR || h->dtype != QRK_F32 || h->max_rows > 64 || h->ragged) return QRK_EINVAL;
    for (int c = 0; c < kBlockClasses; ++c)
      if (block_class_short(c) && h->bq_count[c] > 0) return QRK_EINVAL;
  }
  h->keep_q = keep != 0;
  h->q_valid = false;
  ++h->shape_gen;  // an LM graph captured before now factors without (or with) the stored Q
  return ensure_q_storage(h);
}

qrk_status qrk_apply_qt(qrk_handle h, const void* b, double* c, void* stream) {
  if (!h || !b || !c || !h->factored || !h->q_valid) return QRK_EINVAL;
  return apply(h, b, c, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? QRK_OK : QRK_EHIP;
}

qrk_status qrk_solve_qt(qrk_handle h, const void* b, double* p, int32_t sweeps, void* stream) {
  if (!h || !b || !p || sweeps < 0 || sweeps > 8 || !h->factored || !h->q_valid) return QRK_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const BatchView bv = blockangular_view(h);
  const float* Rblk = static_cast<const float*>(h->Rblk);
  const float* Sc = static_cast<const float*>(h->Sc);
  const float* RB = static_cast<const float*>(h->RB);
  if (apply(h, b, h->q_c, st) != hipSuccess ||
      launch_backsub_dense<float>(bv, RB, p, h->status, st, h->q_c) != hipSuccess ||
      launch_backsub_blocks<float>(bv, Rblk, Sc, p, h->status, st, h->q_c) != hipSuccess)
    return QRK_EHIP;
  return sweeps > 0 ? blockangular_refine(h, p, sweeps, b, st) : QRK_OK;
}

}  // extern "C"
