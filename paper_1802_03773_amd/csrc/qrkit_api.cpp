// Host side of the qrkit C ABI: argument validation, workspace ownership, launch
// selection and the device status word.  See include/qrkit.h for the contract.
#include "qrkit.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "qrk_launch.hpp"
#include "qrk_device.hpp"
#include "block_classes.hpp"
#include "qrk_host.hpp"
#include "qrk_layout.hpp"
#include "tune_cache.hpp"

using namespace qrk;

namespace {

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

qrk_status check_device(int* cus = nullptr, char* arch = nullptr, size_t arch_len = 0) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return QRK_ENODEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return QRK_ENODEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return QRK_ENODEVICE;
  if (cus) *cus = prop.multiProcessorCount;
  if (arch && arch_len) {
    // the base name (gfx950), without the feature suffixes
    size_t i = 0;
    while (i + 1 < arch_len && prop.gcnArchName[i] && prop.gcnArchName[i] != ':') {
      arch[i] = prop.gcnArchName[i];
      ++i;
    }
    arch[i] = 0;
  }
  return QRK_OK;
}

BatchView view(qrk_handle h) {
  BatchView bv;
  bv.P = h->P;
  bv.n = h->n;
  bv.Ktot = h->K;
  bv.max_L = h->max_L;
  bv.max_rows = h->max_rows;
  bv.probs = h->probs_d;
  bv.blk_prob = h->blk_prob;
  bv.row_off = h->row_off_d;
  bv.pack_blk = h->pack_blk;
  bv.wg_prob = h->wg_prob;
  bv.nwg = h->nwg;
  bv.lam = h->lam_ptr;
  bv.grid_blocks = h->grid_blocks;
  return bv;
}

// lam_host: lambda of a single problem given by value (stored to the handle's device copy by
// the first launch); null when lambda is already on the device.
template <typename T>
qrk_status factor_ba(qrk_handle h, hipStream_t st, const double* lam_host = nullptr) {
  const T* A = static_cast<const T*>(h->A);
  const T* B = static_cast<const T*>(h->B);
  const T* b = static_cast<const T*>(h->b);
  T* Rblk = static_cast<T*>(h->Rblk);
  T* Sc = static_cast<T*>(h->Sc);
  T* Red = static_cast<T*>(h->Red);
  T* RB = static_cast<T*>(h->RB);
  // the first launch clears the status words and the merge-tree arrival counters
  BqrPrologue pro;
  pro.z0 = h->status;
  pro.n0 = h->P;
  if (std::is_same<T, float>::value) {
    pro.z1 = h->counters;
    pro.n1 = h->nctr;
  }
  if (lam_host) {
    pro.lam_out = h->lam_d;
    pro.lam_val = *lam_host;
  }
  h->vparts.clear();  // a new factor of this handle's own rows
  // the stored Q (float32 only): per-block reflectors, tile and node panels
  const bool keep = std::is_same<T, float>::value && h->keep_q && h->qk.vd != nullptr;
  QStore qs;
  if (keep) {
    qs.qt = h->q_tiles;
    qs.qn = h->q_nodes;
    qs.qo = h->qoff_d;
  }
  h->q_valid = false;
  int pr = prof_begin(h, 0, st);
  // without a list, the one class present covers blocks 0 .. K-1 in order
  const int32_t* list = h->blk_list_n > 0 ? h->blk_list : nullptr;
  const int64_t extent = h->blk_list_n > 0 ? h->blk_list_n : h->K;
  for (int c = 0; c < kBlockClasses; ++c) {
    if (h->bq_count[c] == 0) continue;
    if (h->bq_begin[c] < 0 || h->bq_begin[c] + h->bq_count[c] > extent) return QRK_EINVAL;
    if (launch_blockqr<T>(list, h->bq_begin[c], h->bq_count[c], c, h->n, h->P, h->probs_d, h->blk_prob,
                          h->row_off_d, A, B, h->camb ? h->cam : nullptr, b, h->d, h->lam_ptr, Rblk, Sc, Red, pro,
                          keep ? h->qk : QKeep(), st) != hipSuccess)
      return QRK_EHIP;
    pro = BqrPrologue();  // later launches: nothing to clear, lambda on the device
  }
  prof_end(h, pr, st);
  if constexpr (std::is_same<T, float>::value) {
    // dense parts on the matrix cores: leaves and merge trees, one launch per column-block count
    pr = prof_begin(h, 1, st);
    if (launch_tsqr_mfma(h->mode == QRK_BF16X3, h->cls_begin, h->cls_count, h->queue_begin, h->leaf_queue != 0, h->cus,
                         h->leaf_prob, h->leaf_idx, h->probs_d, h->n, Red, h->d, h->lam_ptr, h->slots, h->counters,
                         h->nctr, h->counters + h->qhead_off, RB, qs, st) != hipSuccess)
      return QRK_EHIP;
    if (h->nnodes > 0 &&
        launch_tsqr_tree((h->probs_h[0].L + 15) / 16, h->probs_d, h->node_l, h->node_r, h->nnodes, h->slots,
                         h->counters, RB, h->status, qs, st) != hipSuccess)
      return QRK_EHIP;
    prof_end(h, pr, st);
    h->q_valid = keep;
    return QRK_OK;
  }
  // float64 dense parts: the leaves of every problem in one launch, then one launch per merge
  // level over every problem still merging (the last level of each writes its R_B | c_B)
  T* P0 = static_cast<T*>(h->part0);
  T* P1 = static_cast<T*>(h->part1);
  for (size_t lv = 0; lv < h->tsqr_lvl_begin.size(); ++lv) {
    pr = prof_begin(h, lv == 0 ? 1 : 2, st);
    if (launch_tsqr_stream<T>(h->tsqr_wg + h->tsqr_lvl_begin[lv], h->tsqr_lvl_count[lv], h->max_L, h->probs_d,
                              h->n, Red, h->d, h->lam_ptr, P0, P1, RB, st) != hipSuccess)
      return QRK_EHIP;
    prof_end(h, pr, st);
  }
  return QRK_OK;
}

// `sweeps` corrected semi-normal sweeps for the right-hand side b: r = b - J p,
// g = J^T r - lam D^2 p, p += (R^T R)^{-1} g.
template <typename T>
qrk_status refine_ba(qrk_handle h, double* p, int sweeps, const T* b, hipStream_t st) {
  const T* Rblk = static_cast<const T*>(h->Rblk);
  const T* Sc = static_cast<const T*>(h->Sc);
  const T* RB = static_cast<const T*>(h->RB);
  const BatchView bv = view(h);
  int pr = sweeps > 0 ? prof_begin(h, 4, st) : -1;
  const int64_t Kn = h->K * h->n;
  for (int s = 0; s < sweeps; ++s) {
    if (launch_refine_residual<T>(bv, static_cast<const T*>(h->A), static_cast<const T*>(h->B),
                                  h->camb ? h->cam : nullptr, b, h->d, Rblk, Sc, p, h->ybuf, h->refpart,
                                  st) != hipSuccess)
      return QRK_EHIP;
    // rows added by vertical concatenation: each part's residual terms with the stacked factor
    for (qrk_handle q : h->vparts)
      if (launch_refine_residual<T>(view(q), static_cast<const T*>(q->A), static_cast<const T*>(q->B), nullptr,
                                    static_cast<const T*>(q->b), q->d, Rblk, Sc, p, q->ybuf, q->refpart,
                                    st) != hipSuccess ||
          launch_vcat_merge(Kn, h->ybuf, q->ybuf, h->refpart, q->refpart, q->nwg, h->nB, q->lam_ptr, q->d + Kn,
                            p + Kn, st) != hipSuccess)
        return QRK_EHIP;
    if (launch_refine_dense<T>(bv, h->refpart, RB, h->d, p, h->deltaB, st) != hipSuccess ||
        launch_refine_blocks<T>(bv, Rblk, Sc, h->ybuf, h->deltaB, p, st) != hipSuccess)
      return QRK_EHIP;
  }
  prof_end(h, pr, st);
  return QRK_OK;
}

template <typename T>
qrk_status solve_ba(qrk_handle h, double* p, int sweeps, hipStream_t st) {
  const T* Rblk = static_cast<const T*>(h->Rblk);
  const T* Sc = static_cast<const T*>(h->Sc);
  const T* RB = static_cast<const T*>(h->RB);
  const BatchView bv = view(h);
  int pr = prof_begin(h, 3, st);
  if (launch_backsub_dense<T>(bv, RB, p, h->status, st) != hipSuccess) return QRK_EHIP;
  if (launch_backsub_blocks<T>(bv, Rblk, Sc, p, h->status, st) != hipSuccess) return QRK_EHIP;
  prof_end(h, pr, st);
  return refine_ba<T>(h, p, sweeps, static_cast<const T*>(h->b), st);
}

void prof_free(qrk_handle h) {
  for (auto& r : h->prof_pool) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  h->prof_pool.clear();
  h->prof_used = 0;
  h->prof_on = false;
}

void free_all(qrk_handle h) {
  if (h->lam_stage) {
    free_all(h->lam_stage);
    delete h->lam_stage;
    h->lam_stage = nullptr;
  }
  if (h->vcat_stage) {
    free_all(h->vcat_stage);
    delete h->vcat_stage;
    h->vcat_stage = nullptr;
  }
  prof_free(h);
  for (void* ptr : h->allocs) (void)hipFree(ptr);
  h->allocs.clear();
}

template <typename P>
qrk_status dalloc(qrk_handle h, P** out, size_t bytes) {
  void* ptr = nullptr;
  bytes = std::max<size_t>(bytes, 256);
  if (hipMalloc(&ptr, bytes) != hipSuccess) return QRK_ENOMEM;
  h->allocs.push_back(ptr);
  h->ws_bytes += (int64_t)bytes;
  *out = static_cast<P*>(ptr);
  return QRK_OK;
}

void dfree(qrk_handle h, void* ptr) {
  if (!ptr) return;
  for (size_t i = 0; i < h->allocs.size(); ++i)
    if (h->allocs[i] == ptr) {
      (void)hipFree(ptr);
      h->allocs.erase(h->allocs.begin() + (long)i);
      return;
    }
}

// Slots and arrival counters a merge tree over `leaves` leaves touches: level k has n_k
// nodes (n_0 = leaves, n_{k+1} = ceil(n_k / 2)); its stored triangles sit at slots
// [sum_{j<k} n_j, sum_{j<=k} n_j) and its counters at [sum_{j<k} n_{j+1}, ...).
struct TreeSize {
  int64_t slots, counters;
};
TreeSize tree_size(int64_t leaves) {
  TreeSize t{0, 0};
  for (int64_t nl = leaves; nl > 1; nl = (nl + 1) / 2) {
    t.slots += nl;
    t.counters += (nl + 1) / 2;
  }
  t.slots = std::max<int64_t>(t.slots, 1);
  t.counters = std::max<int64_t>(t.counters, 1);
  return t;
}

// Dense-part leaves of every problem.  float32: leaves are single waves; per 16-column-block
// class c the default is about max(128, rows_c / 4096) rows per leaf (rows_c: the class's
// reduced plus damping rows), scaled by leaf_scale, at most 1024 leaves per problem; a
// single-problem handle may fix the count (h->leaves > 0).  Leaves are listed class by class
// for the per-class launches, and each problem's merge tree gets the slots and arrival
// counters of tree_size.  float64: leaves are workgroups of about 256 rows.
qrk_status assign_leaves(qrk_handle h) {
  std::vector<ProbDesc>& pd = h->probs_h;
  const int P = h->P;
  if (h->dtype == QRK_F64) {
    // leaves of about 256 rows (at most 1024 per problem; a batch's problems share about 4096
    // in proportion to their rows)
    double rows_all = 0.0;
    for (const auto& D : pd) rows_all += (double)(D.M + D.nB);
    for (auto& D : pd) {
      int64_t def = std::max<int64_t>(1, std::min<int64_t>(ceil_div(D.M + D.nB, 256), 1024));
      if (P > 1) def = std::min<int64_t>(def, std::max<int64_t>(1, std::llround(4096.0 * (D.M + D.nB) / rows_all)));
      D.leaves = (int)(h->leaves > 0 ? h->leaves : def);
      D.rows_per_leaf = std::max<int64_t>(1, ceil_div(D.M, D.leaves));
    }
    // the workgroups of every level, all problems together: level 0 streams each problem's
    // reduced rows into its leaves' triangles, each later level merges fanin triangles of the
    // level below (stacked as rows); a problem's last level writes its R_B | c_B.  Levels
    // alternate between the two partial buffers.
    std::vector<TsqrWg> wl;
    h->tsqr_lvl_begin.clear();
    h->tsqr_lvl_count.clear();
    std::vector<int64_t> G((size_t)P), in_off((size_t)P, 0);
    for (int q = 0; q < P; ++q) G[(size_t)q] = pd[(size_t)q].leaves;
    int64_t need[2] = {0, 0};
    for (int level = 0;; ++level) {
      const int buf = 1 + (level & 1);  // this level's output buffer when not the root
      int64_t off = 0;
      const int begin = (int)wl.size();
      bool any = false;
      for (int q = 0; q < P; ++q) {
        const ProbDesc& D = pd[(size_t)q];
        const int64_t L = D.L;
        if (level > 0 && G[(size_t)q] <= 1) continue;  // done
        const int64_t nout = level == 0 ? G[(size_t)q] : ceil_div(G[(size_t)q], (int64_t)h->fanin);
        for (int64_t k = 0; k < nout; ++k) {
          TsqrWg w{};
          w.L = (int32_t)L;
          if (level == 0) {
            w.x_off = D.redoff;
            w.ldx = (int32_t)D.ldr;
            w.r0 = std::min<int64_t>(k * D.rows_per_leaf, D.M);
            w.r1 = std::min<int64_t>((k + 1) * D.rows_per_leaf, D.M);
            w.seed = k == 0 ? q : -1;
            w.in_buf = 0;
          } else {
            w.x_off = in_off[(size_t)q];
            w.ldx = (int32_t)L;
            w.r0 = k * h->fanin * L;
            w.r1 = std::min<int64_t>((k + 1) * h->fanin, G[(size_t)q]) * L;
            w.seed = -1;
            w.in_buf = (int8_t)(1 + ((level - 1) & 1));
          }
          if (nout == 1) {
            w.out_buf = 0;
            w.out_off = D.rboff;
          } else {
            w.out_buf = (int8_t)buf;
            w.out_off = off + k * L * L;
          }
          wl.push_back(w);
        }
        if (nout > 1) {
          in_off[(size_t)q] = off;
          off += nout * L * L;
        }
        G[(size_t)q] = nout;
        any = true;
      }
      if (!any) break;
      h->tsqr_lvl_begin.push_back(begin);
      h->tsqr_lvl_count.push_back((int)wl.size() - begin);
      need[buf - 1] = std::max(need[buf - 1], off);
    }
    qrk_status s;
    const size_t es = sizeof(double);
    if ((int64_t)wl.size() > h->tsqr_wg_cap) {
      dfree(h, h->tsqr_wg);
      h->tsqr_wg = nullptr;
      h->tsqr_wg_cap = 0;
      if ((s = dalloc(h, &h->tsqr_wg, sizeof(TsqrWg) * wl.size())) != QRK_OK) return s;
      h->tsqr_wg_cap = (int64_t)wl.size();
    }
    for (int b = 0; b < 2; ++b) {
      void*& part = b == 0 ? h->part0 : h->part1;
      int64_t& cap = b == 0 ? h->part_cap0 : h->part_cap1;
      if (need[b] > cap) {
        dfree(h, part);
        part = nullptr;
        cap = 0;
        if ((s = dalloc(h, reinterpret_cast<char**>(&part), es * (size_t)need[b])) != QRK_OK) return s;
        cap = need[b];
      }
    }
    if (!wl.empty() &&
        hipMemcpy(h->tsqr_wg, wl.data(), sizeof(TsqrWg) * wl.size(), hipMemcpyHostToDevice) != hipSuccess)
      return QRK_EHIP;
  } else {
    double rows_cls[9] = {0};
    for (auto& D : pd) rows_cls[(D.L + 15) / 16] += (double)(D.M + D.nB);
    for (auto& D : pd) {
      const int c = (D.L + 15) / 16;
      const double per = std::max(128.0, rows_cls[c] / 4096.0) * h->leaf_scale;
      const int64_t def = std::max<int64_t>(
          1, std::min<int64_t>((int64_t)std::ceil((double)(D.M + D.nB) / std::max(per, 1.0)), 1024));
      D.leaves = (int)(h->leaves > 0 ? h->leaves : def);
      D.rows_per_leaf = std::max<int64_t>(1, ceil_div(D.M, D.leaves));
    }
    // widest classes first: classes 8 and 7 have launches of their own, classes 6 .. 1 form the
    // persistent queue launch's item list (the suffix starting at cls_begin of the widest of them)
    std::vector<int32_t> lp, li;
    for (int c = 8; c >= 1; --c) {
      h->cls_begin[c] = (int)lp.size();
      for (int q = 0; q < P; ++q)
        if ((pd[q].L + 15) / 16 == c)
          for (int k = 0; k < pd[q].leaves; ++k) {
            lp.push_back(q);
            li.push_back(k);
          }
      h->cls_count[c] = (int)lp.size() - h->cls_begin[c];
    }
    // a single problem of at most kTreeMaxNCB column blocks merges its leaves in a separate
    // launch, pipelined over column blocks; otherwise the merges run inside the leaf launch
    std::vector<int32_t> nl, nr;
    const bool sep = P == 1 && pd[0].leaves > 1 && (pd[0].L + 15) / 16 <= kTreeMaxNCB;
    if (sep) {
      std::vector<int32_t> items((size_t)pd[0].leaves);
      for (int i = 0; i < pd[0].leaves; ++i) items[(size_t)i] = -1 - i;
      while (items.size() > 1) {
        std::vector<int32_t> next;
        for (size_t i = 0; i + 1 < items.size(); i += 2) {
          nl.push_back(items[i]);
          nr.push_back(items[i + 1]);
          next.push_back((int32_t)nl.size() - 1);
        }
        if (items.size() & 1) next.push_back(items.back());
        items.swap(next);
      }
    }
    h->nnodes = (int)nl.size();
    int64_t slot = 0, ctr = 0;
    for (auto& D : pd) {
      D.slot0 = slot;
      D.ctr0 = ctr;
      D.tree_sep = sep ? 1 : 0;
      if (sep) {
        slot += (int64_t)(D.leaves + h->nnodes) * tsqr_mfma_slot_floats(D.L);
        ctr += std::max<int64_t>(1, (int64_t)h->nnodes * ((D.L + 15) / 16) * 2);  // two flags per column block
      } else {
        const TreeSize ts = tree_size(D.leaves);
        slot += ts.slots * tsqr_mfma_slot_floats(D.L);
        ctr += ts.counters;
      }
    }
    // stored Q: tile panels of every leaf, node panels of the leaves - 1 merges, and the
    // application's merge vectors (128 floats per tree slot)
    int64_t qt = 0, qn = 0, qu = 0;
    h->qoff_h.resize((size_t)P);
    for (int q = 0; q < P; ++q) {
      const ProbDesc& D = pd[(size_t)q];
      QOff& O = h->qoff_h[(size_t)q];
      const int ncb = (D.L + 15) / 16;
      O.qtiles = ceil_div(D.rows_per_leaf, (int64_t)leaf_tile_rows_keep(ncb));
      O.qt0 = qt;
      qt += (int64_t)D.leaves * O.qtiles * ncb * tile_panel_floats(leaf_tile_rows_keep(ncb) / 16);
      O.qn0 = qn;
      qn += (int64_t)(D.leaves - 1) * node_panel_off(ncb);
      O.qc0 = qu;
      qu += tree_size(D.leaves).slots * 128;
    }
    h->q_tiles_n = std::max<int64_t>(qt, 1);
    h->q_nodes_n = std::max<int64_t>(qn, 1);
    h->q_u_n = std::max<int64_t>(qu, 1);
    h->qhead_off = ctr;  // the persistent leaf launch's queue head, cleared with the counters
    ctr += 1;
    h->nctr = ctr;
    h->queue_begin = (int)lp.size();
    for (int c = kQueueNCB; c >= 1; --c)
      if (h->cls_count[c] > 0) h->queue_begin = std::min(h->queue_begin, h->cls_begin[c]);
    if (h->nnodes > h->node_cap) {
      dfree(h, h->node_l);
      dfree(h, h->node_r);
      h->node_l = h->node_r = nullptr;
      h->node_cap = 0;
      qrk_status s2;
      if ((s2 = dalloc(h, &h->node_l, sizeof(int32_t) * h->nnodes)) != QRK_OK ||
          (s2 = dalloc(h, &h->node_r, sizeof(int32_t) * h->nnodes)) != QRK_OK)
        return s2;
      h->node_cap = h->nnodes;
    }
    if (h->nnodes > 0 &&
        (hipMemcpy(h->node_l, nl.data(), sizeof(int32_t) * nl.size(), hipMemcpyHostToDevice) != hipSuccess ||
         hipMemcpy(h->node_r, nr.data(), sizeof(int32_t) * nr.size(), hipMemcpyHostToDevice) != hipSuccess))
      return QRK_EHIP;
    const int64_t nleaf = (int64_t)lp.size();
    qrk_status s;
    if (nleaf > h->leaf_cap) {
      dfree(h, h->leaf_prob);
      dfree(h, h->leaf_idx);
      h->leaf_prob = h->leaf_idx = nullptr;
      h->leaf_cap = 0;
      if ((s = dalloc(h, &h->leaf_prob, sizeof(int32_t) * nleaf)) != QRK_OK ||
          (s = dalloc(h, &h->leaf_idx, sizeof(int32_t) * nleaf)) != QRK_OK)
        return s;
      h->leaf_cap = nleaf;
    }
    if (slot > h->slot_cap) {
      dfree(h, h->slots);
      h->slots = nullptr;
      h->slot_cap = 0;
      if ((s = dalloc(h, &h->slots, sizeof(float) * slot)) != QRK_OK) return s;
      h->slot_cap = slot;
    }
    if (ctr > h->ctr_cap) {
      dfree(h, h->counters);
      h->counters = nullptr;
      h->ctr_cap = 0;
      if ((s = dalloc(h, &h->counters, sizeof(int) * ctr)) != QRK_OK) return s;
      h->ctr_cap = ctr;
    }
    if (hipMemcpy(h->leaf_prob, lp.data(), sizeof(int32_t) * nleaf, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->leaf_idx, li.data(), sizeof(int32_t) * nleaf, hipMemcpyHostToDevice) != hipSuccess)
      return QRK_EHIP;
  }
  if (hipMemcpy(h->probs_d, pd.data(), sizeof(ProbDesc) * P, hipMemcpyHostToDevice) != hipSuccess)
    return QRK_EHIP;
  ++h->shape_gen;
  h->q_valid = false;
  return ensure_q_storage(h);
}

}  // namespace

qrk_status ensure_q_storage(qrk_handle h) {
  if (!h->keep_q) return QRK_OK;
  qrk_status s;
  const size_t es = sizeof(float);
  if (!h->qk.vd) {
    void *vd = nullptr, *vp = nullptr, *g = nullptr;
    if ((s = dalloc(h, &h->qoff_d, sizeof(QOff) * (size_t)h->P)) != QRK_OK) return s;
    if ((s = dalloc(h, &vd, es * (size_t)std::max<int64_t>(h->M * h->n, 1))) != QRK_OK ||
        (s = dalloc(h, &vp, es * (size_t)std::max<int64_t>(h->K * h->n * h->n, 1))) != QRK_OK ||
        (s = dalloc(h, &g, es * (size_t)std::max<int64_t>(h->K * h->n, 1))) != QRK_OK ||
        (s = dalloc(h, &h->q_xr, es * (size_t)std::max<int64_t>(h->M, 1))) != QRK_OK ||
        (s = dalloc(h, &h->q_c, sizeof(double) * (size_t)std::max<int64_t>(h->N, 1))) != QRK_OK)
      return s;
    h->qk.vd = vd;
    h->qk.vp = vp;
    h->qk.g = g;
  }
  auto grow = [&](float** ptr, int64_t* cap, int64_t need) -> qrk_status {
    if (need <= *cap) return QRK_OK;
    dfree(h, *ptr);
    *ptr = nullptr;
    *cap = 0;
    const qrk_status s2 = dalloc(h, ptr, es * (size_t)need);
    if (s2 == QRK_OK) *cap = need;
    return s2;
  };
  if ((s = grow(&h->q_tiles, &h->q_tiles_cap, h->q_tiles_n)) != QRK_OK ||
      (s = grow(&h->q_nodes, &h->q_nodes_cap, h->q_nodes_n)) != QRK_OK ||
      (s = grow(&h->q_u, &h->q_u_cap, h->q_u_n)) != QRK_OK)
    return s;
  if (h->qoff_h.size() != (size_t)h->P ||
      hipMemcpy(h->qoff_d, h->qoff_h.data(), sizeof(QOff) * (size_t)h->P, hipMemcpyHostToDevice) != hipSuccess)
    return QRK_EHIP;
  return QRK_OK;
}

qrk_status handle_alloc(qrk_handle h, void** out, size_t bytes) { return dalloc(h, out, bytes); }

qrk_status blockangular_factor(qrk_handle h, hipStream_t st) {
  return h->dtype == QRK_F32 ? factor_ba<float>(h, st) : factor_ba<double>(h, st);
}

qrk_status blockangular_refine(qrk_handle h, double* p, int sweeps, const void* b, hipStream_t st) {
  return h->dtype == QRK_F32 ? refine_ba<float>(h, p, sweeps, static_cast<const float*>(b), st)
                             : refine_ba<double>(h, p, sweeps, static_cast<const double*>(b), st);
}

qrk_status blockangular_solve(qrk_handle h, double* p, int sweeps, hipStream_t st) {
  return h->dtype == QRK_F32 ? solve_ba<float>(h, p, sweeps, st) : solve_ba<double>(h, p, sweeps, st);
}

BatchView blockangular_view(qrk_handle h) { return view(h); }
void handle_free(qrk_handle h) { free_all(h); }

template <typename T>
qrk_status adjoint_ba(qrk_handle h, const double* p, const double* g, void* dA, void* dB, void* db,
                      double* dlam, double* dd, hipStream_t st) {
  const T* Rblk = static_cast<const T*>(h->Rblk);
  const T* Sc = static_cast<const T*>(h->Sc);
  const T* RB = static_cast<const T*>(h->RB);
  const BatchView bv = view(h);
  // u = (R^T R)^{-1} g through the structured R
  if (launch_adjoint_fwd_blocks<T>(h->K, h->n, h->nB, Rblk, Sc, g, h->ybuf, h->refpart, h->nwg, st) != hipSuccess)
    return QRK_EHIP;
  if (h->nB > 0 && launch_adjoint_dense<T>(bv, h->refpart, RB, g, h->ubuf, st) != hipSuccess) return QRK_EHIP;
  if (launch_adjoint_blocks<T>(bv, Rblk, Sc, h->ybuf, h->ubuf, st) != hipSuccess) return QRK_EHIP;
  if ((dA || dB || db) &&
      launch_adjoint_rows<T>(h->npacks, h->pack_blk, h->K, h->n, h->nB, h->row_off_d,
                             static_cast<const T*>(h->A), static_cast<const T*>(h->B), h->ldb,
                             static_cast<const T*>(h->b), p, h->ubuf, static_cast<T*>(dA),
                             static_cast<T*>(dB), static_cast<T*>(db), h->nwg, st) != hipSuccess)
    return QRK_EHIP;
  if ((dlam || dd) &&
      launch_adjoint_vec(1, h->N, h->ubuf, h->d, p, h->lam, dd, dlam, h->vecpart, st) != hipSuccess)
    return QRK_EHIP;
  return QRK_OK;
}

qrk_status blockangular_adjoint(qrk_handle h, const double* p, const double* g, void* dA, void* dB,
                                void* db, double* dlam, double* dd, hipStream_t st) {
  return h->dtype == QRK_F32 ? adjoint_ba<float>(h, p, g, dA, dB, db, dlam, dd, st)
                             : adjoint_ba<double>(h, p, g, dA, dB, db, dlam, dd, st);
}

int prof_begin(qrk_handle h, int phase, hipStream_t st) {
  if (!h->prof_on || h->prof_used >= (int)h->prof_pool.size()) return -1;
  const int i = h->prof_used++;
  h->prof_pool[i].phase = phase;
  (void)hipEventRecord(h->prof_pool[i].start, st);
  return i;
}

void prof_end(qrk_handle h, int rec, hipStream_t st) {
  if (rec >= 0) (void)hipEventRecord(h->prof_pool[rec].stop, st);
}

// Largest refinement workgroup scale the autotuner tries (its buffers are sized for it).
constexpr double kMaxRefineScale = 2.0;

// The handle's key in the autotuner cache.
std::string handle_tune_key(qrk_handle h) {
  return tune_key(h->arch, (int)h->dtype, (int)h->mode, h->P, h->n, h->M, h->max_L, h->widths);
}

// Refinement workgroups of every problem, in proportion to its packs: 512 in all (two waves per
// SIMD in one round at the refinement's register use), about eight per problem for batches,
// times refine_scale; never more than the capacity reserved at create.
qrk_status assign_refine(qrk_handle h, bool upload) {
  std::vector<ProbDesc>& pd = h->probs_h;
  const int P = h->P;
  const double base = (double)std::min<int64_t>(ceil_div(h->npacks, 4), std::max<int64_t>(512, 8 * (int64_t)P));
  const int64_t target = std::max<int64_t>(1, (int64_t)std::llround(base * h->refine_scale));
  std::vector<int32_t> wg_prob;
  for (int32_t q = 0; q < P; ++q) {
    ProbDesc& D = pd[q];
    int64_t w = (int64_t)std::llround((double)D.npacks * (double)target / (double)h->npacks);
    w = std::max<int64_t>(1, std::min<int64_t>(w, ceil_div(D.npacks, 4)));
    D.wg0 = (int32_t)wg_prob.size();
    D.nwg = (int32_t)w;
    for (int64_t k = 0; k < w; ++k) wg_prob.push_back(q);
  }
  if ((int64_t)wg_prob.size() > h->nwg_cap) return QRK_EINVAL;
  h->nwg = (int)wg_prob.size();
  h->refine_grid = h->nwg;
  if (upload) {
    if (hipMemcpy(h->wg_prob, wg_prob.data(), sizeof(int32_t) * wg_prob.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->probs_d, pd.data(), sizeof(ProbDesc) * P, hipMemcpyHostToDevice) != hipSuccess)
      return QRK_EHIP;
    ++h->shape_gen;
  }
  return QRK_OK;
}

// Validate a batch description and build the handle: per-problem descriptors, the
// block -> problem map, packs of whole blocks (at most 64 rows and 64 blocks, never across
// problems), refinement workgroups per problem (in proportion to the packs, at most 1024 in
// all), dense-part leaves, and all workspace.  ldb_single >= 0: one problem whose B has that
// row stride; -1: B packed problem after problem with row stride nB_p.
qrk_status create_ba(int32_t P, int32_t n, const int32_t* Kp, const int32_t* nBp, const int64_t* row_off_host,
                     int64_t ldb_single, qrk_dtype dtype, qrk_mode mode, qrk_handle* out) {
  if (P < 1 || !Kp || !nBp || !row_off_host) return QRK_EINVAL;
  if (n < 1 || n > QRK_MAX_BLOCK_COLS || (dtype != QRK_F32 && dtype != QRK_F64)) return QRK_EINVAL;
  if (mode != QRK_PLAIN && mode != QRK_BF16X3) return QRK_EINVAL;
  if (mode == QRK_BF16X3 && dtype != QRK_F32) return QRK_EINVAL;
  int64_t Ktot = 0;
  for (int32_t q = 0; q < P; ++q) {
    if (Kp[q] < 1 || nBp[q] < 0 || nBp[q] > QRK_MAX_DENSE_COLS) return QRK_EINVAL;
    Ktot += Kp[q];
  }
  if (row_off_host[0] != 0) return QRK_EINVAL;
  int max_m = 0;
  for (int64_t i = 0; i < Ktot; ++i) {
    const int64_t m = row_off_host[i + 1] - row_off_host[i];
    if (m < 0 || m > QRK_MAX_BLOCK_ROWS) return QRK_EINVAL;
    max_m = std::max<int>(max_m, (int)m);
  }
  int cus = 256;
  char arch[32] = {0};
  qrk_status ds = check_device(&cus, arch, sizeof(arch));
  if (ds != QRK_OK) return ds;

  qrk_handle h = new (std::nothrow) qrk_handle_s();
  if (!h) return QRK_ENOMEM;
  h->kind = KIND_BLOCKANGULAR;
  h->cus = cus;
  std::memcpy(h->arch, arch, sizeof(arch));
  h->dtype = dtype;
  h->mode = mode;
  h->P = P;
  h->K = Ktot;
  h->n = n;
  h->nB = nBp[0];
  h->M = row_off_host[Ktot];
  h->max_rows = max_m + n;
  h->ldb = ldb_single >= 0 ? ldb_single : nBp[0];
  h->ldr = reduced_row_stride(nBp[0] + 1, dtype == QRK_F32 ? 4 : 8);
  const size_t es = dtype == QRK_F32 ? 4 : 8;

  // per-problem descriptors and packs
  std::vector<ProbDesc>& pd = h->probs_h;
  pd.resize(P);
  std::vector<int64_t> packs{0};
  std::vector<int32_t> blk_prob((size_t)Ktot);
  int64_t koff = 0, noff = 0, boff = 0, soff = 0, redoff = 0, rboff = 0;
  for (int32_t q = 0; q < P; ++q) {
    ProbDesc& D = pd[q];
    std::memset(&D, 0, sizeof(D));
    D.koff = koff;
    D.K = Kp[q];
    D.moff = row_off_host[koff];
    D.M = row_off_host[koff + D.K] - D.moff;
    D.noff = noff;
    D.nB = nBp[q];
    D.L = D.nB + 1;
    D.boff = boff;
    D.ldb = ldb_single >= 0 ? ldb_single : D.nB;
    D.soff = soff;
    D.ldr = reduced_row_stride(D.L, dtype == QRK_F32 ? 4 : 8);
    D.redoff = redoff;
    D.rboff = rboff;
    D.pack0 = (int64_t)packs.size() - 1;
    int64_t rows = 0;
    int nbp = 0;
    for (int64_t i = koff; i < koff + D.K; ++i) {
      blk_prob[(size_t)i] = q;
      const int64_t m = row_off_host[i + 1] - row_off_host[i];
      if (nbp > 0 && (rows + m > 64 || nbp == 64)) {
        packs.push_back(i);
        rows = 0;
        nbp = 0;
      }
      rows += m;
      ++nbp;
    }
    packs.push_back(koff + D.K);
    D.npacks = (int64_t)packs.size() - 1 - D.pack0;
    h->max_L = std::max(h->max_L, (int)D.L);
    koff += D.K;
    noff += D.K * n + D.nB;
    boff += D.M * D.ldb;
    soff += D.K * n * D.L;
    redoff += D.M * D.ldr;
    rboff += (int64_t)D.L * D.L;
  }
  h->N = noff;
  h->npacks = (int64_t)packs.size() - 1;
  // per-block QR classes (register rows x column slots)
  BlockClasses bq;
  if (!group_block_classes(row_off_host, Ktot, n, [&](int64_t i) { return (int)pd[blk_prob[(size_t)i]].L; }, bq)) {
    delete h;
    return QRK_EINVAL;
  }
  for (int c = 0; c < kBlockClasses; ++c) {
    h->bq_begin[c] = bq.begin[c];
    h->bq_count[c] = bq.count[c];
  }
  h->blk_list_n = (int64_t)bq.list.size();
  const std::vector<int32_t>& blk_list = bq.list;
  // float32 leaf widths present (for the cache key and the leaf queue)
  {
    bool seen[9] = {false};
    for (auto& D : pd) seen[(D.L + 15) / 16] = true;
    h->widths = 0;
    for (int c = 1; c <= kQueueNCB; ++c) h->widths += seen[c];
  }
  // launch-shape knobs: a remembered autotuner choice for this shape, else the defaults; the
  // refinement workgroup buffers are sized for the largest scale the autotuner tries
  {
    TuneChoice tc;
    if (tune_lookup(handle_tune_key(h), &tc)) {
      h->leaf_scale = tc.leaf_scale;
      h->leaf_queue = tc.leaf_queue;
      h->refine_scale = tc.refine_scale;
    }
    const double keep = h->refine_scale;
    h->nwg_cap = 1 << 30;
    h->refine_scale = std::max(keep, kMaxRefineScale);
    qrk_status s0 = assign_refine(h, false);
    if (s0 != QRK_OK) {
      delete h;
      return s0;
    }
    h->nwg_cap = h->nwg;
    h->refine_scale = keep;
    s0 = assign_refine(h, false);
    if (s0 != QRK_OK) {
      delete h;
      return s0;
    }
  }
  std::vector<int32_t> wg_prob;
  for (int32_t q = 0; q < P; ++q)
    for (int32_t k = 0; k < pd[q].nwg; ++k) wg_prob.push_back(q);
  h->grid_blocks = (int)std::min<int64_t>(ceil_div(Ktot, 4), 2048);
  h->max_leaves = dtype == QRK_F32 ? 4096 : 1024;
  h->leaves = 0;
  h->fanin = 8;

  qrk_status s = QRK_OK;
  const int Lm = h->max_L;
  if ((s = dalloc(h, &h->row_off_d, sizeof(int64_t) * (Ktot + 1))) != QRK_OK ||
      (s = dalloc(h, &h->pack_blk, sizeof(int64_t) * packs.size())) != QRK_OK ||
      (s = dalloc(h, &h->blk_prob, sizeof(int32_t) * Ktot)) != QRK_OK ||
      (!blk_list.empty() && (s = dalloc(h, &h->blk_list, sizeof(int32_t) * blk_list.size())) != QRK_OK) ||
      (s = dalloc(h, &h->wg_prob, sizeof(int32_t) * (size_t)h->nwg_cap)) != QRK_OK ||
      (s = dalloc(h, &h->probs_d, sizeof(ProbDesc) * P)) != QRK_OK ||
      (s = dalloc(h, &h->Rblk, es * (size_t)Ktot * n * n)) != QRK_OK ||
      (s = dalloc(h, &h->Sc, es * (size_t)soff)) != QRK_OK ||
      (s = dalloc(h, &h->Red, es * (size_t)std::max<int64_t>(redoff, 1))) != QRK_OK ||
      (s = dalloc(h, &h->RB, es * (size_t)rboff)) != QRK_OK ||
      (s = dalloc(h, &h->ybuf, sizeof(double) * (size_t)Ktot * n)) != QRK_OK ||
      (s = dalloc(h, &h->ubuf, sizeof(double) * (size_t)h->N)) != QRK_OK ||
      (s = dalloc(h, &h->vecpart, sizeof(double) * (size_t)1024 * std::max(Lm - 1, 1))) != QRK_OK ||
      (s = dalloc(h, &h->refpart, sizeof(double) * (size_t)h->nwg_cap * kMaxDense)) != QRK_OK ||
      (s = dalloc(h, &h->deltaB, sizeof(double) * (size_t)P * kMaxDense)) != QRK_OK ||
      (s = dalloc(h, &h->lam_d, sizeof(double) * (size_t)P)) != QRK_OK ||
      (s = dalloc(h, &h->status, sizeof(int) * (size_t)std::max(P, 4))) != QRK_OK) {
    free_all(h);
    delete h;
    return s;
  }
  h->lam_ptr = h->lam_d;
  if (hipMemcpy(h->row_off_d, row_off_host, sizeof(int64_t) * (Ktot + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->pack_blk, packs.data(), sizeof(int64_t) * packs.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->blk_prob, blk_prob.data(), sizeof(int32_t) * Ktot, hipMemcpyHostToDevice) != hipSuccess ||
      (!blk_list.empty() && hipMemcpy(h->blk_list, blk_list.data(), sizeof(int32_t) * blk_list.size(),
                                      hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(h->wg_prob, wg_prob.data(), sizeof(int32_t) * wg_prob.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemset(h->status, 0, sizeof(int) * (size_t)std::max(P, 4)) != hipSuccess ||
      hipMemset(h->lam_d, 0, sizeof(double) * (size_t)P) != hipSuccess) {
    free_all(h);
    delete h;
    return QRK_EHIP;
  }
  if ((s = assign_leaves(h)) != QRK_OK) {
    free_all(h);
    delete h;
    return s;
  }
  *out = h;
  return QRK_OK;
}

extern "C" {

const char* qrk_strerror(qrk_status s) {
  switch (s) {
    case QRK_OK: return "success";
    case QRK_EINVAL: return "invalid argument";
    case QRK_ENOMEM: return "device memory allocation failed";
    case QRK_EHIP: return "HIP runtime error";
    case QRK_ESINGULAR: return "R has a numerically zero pivot";
    case QRK_ENONFINITE: return "non-finite value in inputs or factor";
    case QRK_ENODEVICE: return "no gfx950 device available";
    case QRK_ETOOLARGE: return "request exceeds the fixed scratch array of the no-allocation entry point";
    case QRK_ENOTCONVERGED: return "refinement sweeps exhausted above the requested tolerance";
  }
  return "unknown status";
}

qrk_status qrk_create_blockangular(int32_t K, int32_t n, int32_t nB, const int64_t* row_off_host,
                                   int64_t ldb, qrk_dtype dtype, qrk_mode mode, qrk_handle* out) {
  if (!out) return QRK_EINVAL;
  *out = nullptr;
  if (ldb < nB || ldb > QRK_MAX_LDB) return QRK_EINVAL;
  return create_ba(1, n, &K, &nB, row_off_host, ldb, dtype, mode, out);
}

qrk_status qrk_create_blockangular_ncol(int32_t K, const int32_t* ncol_host, int32_t nB, const int64_t* row_off_host,
                                        int64_t ldb, qrk_dtype dtype, qrk_mode mode, qrk_handle* out) {
  if (!out) return QRK_EINVAL;
  *out = nullptr;
  if (K < 1 || !ncol_host || !row_off_host) return QRK_EINVAL;
  int nmax = 0;
  for (int32_t i = 0; i < K; ++i) {
    if (ncol_host[i] < 1 || ncol_host[i] > QRK_MAX_BLOCK_COLS) return QRK_EINVAL;
    nmax = std::max(nmax, (int)ncol_host[i]);
  }
  qrk_status s = qrk_create_blockangular(K, nmax, nB, row_off_host, ldb, dtype, mode, out);
  if (s != QRK_OK) return s;
  qrk_handle h = *out;
  std::vector<int64_t> aoff((size_t)K + 1, 0), poff((size_t)K + 1, 0);
  for (int32_t i = 0; i < K; ++i) {
    aoff[(size_t)i + 1] = aoff[(size_t)i] + (row_off_host[i + 1] - row_off_host[i]) * ncol_host[i];
    poff[(size_t)i + 1] = poff[(size_t)i] + ncol_host[i];
  }
  const size_t es = dtype == QRK_F32 ? 4 : 8;
  if ((s = dalloc(h, &h->rg_ncol, sizeof(int32_t) * (size_t)K)) != QRK_OK ||
      (s = dalloc(h, &h->rg_aoff, sizeof(int64_t) * aoff.size())) != QRK_OK ||
      (s = dalloc(h, &h->rg_poff, sizeof(int64_t) * poff.size())) != QRK_OK ||
      (s = dalloc(h, &h->rg_A, es * (size_t)h->M * (size_t)nmax)) != QRK_OK ||
      (s = dalloc(h, &h->rg_d, sizeof(double) * (size_t)h->N)) != QRK_OK ||
      (s = dalloc(h, &h->rg_p, sizeof(double) * (size_t)h->N)) != QRK_OK) {
    qrk_destroy(h);
    *out = nullptr;
    return s;
  }
  if (hipMemcpy(h->rg_ncol, ncol_host, sizeof(int32_t) * (size_t)K, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->rg_aoff, aoff.data(), sizeof(int64_t) * aoff.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->rg_poff, poff.data(), sizeof(int64_t) * poff.size(), hipMemcpyHostToDevice) != hipSuccess) {
    qrk_destroy(h);
    *out = nullptr;
    return QRK_EHIP;
  }
  h->ragged = true;
  h->rg_N = poff[(size_t)K] + nB;
  return QRK_OK;
}

qrk_status qrk_create_blockangular_batched(int32_t P, int32_t n, const int32_t* K_host, const int32_t* nB_host,
                                           const int64_t* row_off_host, qrk_dtype dtype, qrk_mode mode,
                                           qrk_handle* out) {
  if (!out) return QRK_EINVAL;
  *out = nullptr;
  return create_ba(P, n, K_host, nB_host, row_off_host, -1, dtype, mode, out);
}

qrk_status qrk_factor_blockangular(qrk_handle h, const void* A, const void* B, const void* b,
                                   const double* d, double lambda, void* stream) {
  if (!h || h->kind != KIND_BLOCKANGULAR || h->P != 1 || h->camb) return QRK_EINVAL;
  if (!A || !b || !d || (h->nB > 0 && !B)) return QRK_EINVAL;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return QRK_EINVAL;
  if (h->ragged) {  // the blocks at n columns: zero columns past n_i with unit damping
    if (!(lambda > 0.0)) return QRK_EINVAL;
    const hipError_t e =
        h->dtype == QRK_F32
            ? launch_ragged_in<float>(h->K, h->n, h->nB, h->row_off_d, h->rg_ncol, h->rg_aoff, h->rg_poff,
                                      static_cast<const float*>(A), d, static_cast<float*>(h->rg_A), h->rg_d,
                                      S(stream))
            : launch_ragged_in<double>(h->K, h->n, h->nB, h->row_off_d, h->rg_ncol, h->rg_aoff, h->rg_poff,
                                       static_cast<const double*>(A), d, static_cast<double*>(h->rg_A), h->rg_d,
                                       S(stream));
    if (e != hipSuccess) return QRK_EHIP;
    A = h->rg_A;
    d = h->rg_d;
  }
  h->A = A;
  h->B = B;
  h->b = b;
  h->d = d;
  h->lam = lambda;
  h->lam_ptr = h->lam_d;
  h->factored = true;
  h->lam_base_saved = false;
  return h->dtype == QRK_F32 ? factor_ba<float>(h, S(stream), &lambda) : factor_ba<double>(h, S(stream), &lambda);
}

// Camera columns: B's rows in the compressed form (cw values and a camera index per row); the
// per-block QR and the refinement read them in place.
qrk_status qrk_create_blockangular_cam(int32_t K, int32_t n, int32_t ncam, int32_t cw, const int64_t* row_off_host,
                                       qrk_dtype dtype, qrk_mode mode, qrk_handle* out) {
  if (!out) return QRK_EINVAL;
  *out = nullptr;
  if (ncam < 1 || cw < 1 || (int64_t)ncam * cw > QRK_MAX_DENSE_COLS) return QRK_EINVAL;
  const int32_t nB = ncam * cw;
  const qrk_status s = create_ba(1, n, &K, &nB, row_off_host, cw, dtype, mode, out);
  if (s != QRK_OK) return s;
  (*out)->camb = true;
  (*out)->ncam = ncam;
  (*out)->cw = cw;
  return QRK_OK;
}

qrk_status qrk_factor_blockangular_cam(qrk_handle h, const void* A, const void* Bv, const int32_t* cam,
                                       const void* b, const double* d, double lambda, void* stream) {
  if (!h || h->kind != KIND_BLOCKANGULAR || h->P != 1 || !h->camb) return QRK_EINVAL;
  if (!A || !Bv || !cam || !b || !d) return QRK_EINVAL;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return QRK_EINVAL;
  h->A = A;
  h->B = Bv;
  h->cam = cam;
  h->b = b;
  h->d = d;
  h->lam = lambda;
  h->lam_ptr = h->lam_d;
  h->factored = true;
  h->lam_base_saved = false;
  return h->dtype == QRK_F32 ? factor_ba<float>(h, S(stream), &lambda) : factor_ba<double>(h, S(stream), &lambda);
}

// Moré's two-stage damping (Section 5.2, Eq. LMTwoStep): J = Q R once, then per damping value
// the QR of [R; sqrt(lambda) D].  With the damping rows of each block permuted next to its R_i,
// that second QR is again the structured factorisation of Sections 4.1 and 4.2, now of a
// problem whose blocks are the n rows of R_i (coupled rows S_i | c_i) and whose dense part also
// takes the rows of R_B | c_B; it runs on an internal handle of that shape.
qrk_status qrk_factor_lambda(qrk_handle h, double lambda, void* stream) {
  if (h && h->ragged) return QRK_EINVAL;  // needs the factor at lambda = 0
  if (!h || h->kind != KIND_BLOCKANGULAR || h->P != 1 || !h->factored) return QRK_EINVAL;
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return QRK_EINVAL;
  hipStream_t st = S(stream);
  const size_t es = h->dtype == QRK_F32 ? 4 : 8;
  const int n = h->n;
  const int L = h->nB + 1;
  const int64_t Kn = h->K * n;
  qrk_status s;
  if (!h->vparts.empty()) return QRK_EINVAL;  // a stacked factor: its base is not J alone
  h->q_valid = false;  // the stored Q is that of J alone, not of the new factor
  if (!h->lam_base_saved) {
    if (h->lam != 0.0) return QRK_EINVAL;  // the current factor must be that of J alone
    if (!h->lam_stage) {
      if ((s = dalloc(h, &h->Rblk0, es * (size_t)Kn * n)) != QRK_OK ||
          (s = dalloc(h, &h->Sc0, es * (size_t)Kn * L)) != QRK_OK ||
          (s = dalloc(h, &h->RB0, es * (size_t)L * L)) != QRK_OK ||
          (s = dalloc(h, &h->c0, es * (size_t)Kn)) != QRK_OK)
        return s;
      // second-stage problem: K blocks of n rows (R_i), coupled rows of stride L (S_i | c_i)
      std::vector<int64_t> ro((size_t)h->K + 1);
      for (int64_t i = 0; i <= h->K; ++i) ro[(size_t)i] = i * n;
      const int32_t K32 = (int32_t)h->K, nB32 = h->nB;
      qrk_handle h2 = nullptr;
      if ((s = create_ba(1, n, &K32, &nB32, ro.data(), L, h->dtype, h->mode, &h2)) != QRK_OK) return s;
      // its dense part also takes the L rows of R_B | c_B, after the blocks' reduced rows
      h2->probs_h[0].M += L;
      h2->M += L;
      dfree(h2, h2->Red);
      h2->Red = nullptr;
      if ((s = dalloc(h2, &h2->Red, es * (size_t)(Kn + L) * h2->ldr)) != QRK_OK ||
          (s = assign_leaves(h2)) != QRK_OK) {
        free_all(h2);
        delete h2;
        return s;
      }
      h->lam_stage = h2;
    }
    // keep the factor of J aside; c as a contiguous vector (column nB of S | c)
    if (hipMemcpyAsync(h->Rblk0, h->Rblk, es * (size_t)Kn * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h->Sc0, h->Sc, es * (size_t)Kn * L, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h->RB0, h->RB, es * (size_t)L * L, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpy2DAsync(h->c0, es, static_cast<char*>(h->Sc0) + es * (size_t)h->nB, es * (size_t)L, es,
                         (size_t)Kn, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return QRK_EHIP;
    h->lam_base_saved = true;
  }
  qrk_handle h2 = h->lam_stage;
  if (hipMemcpy2DAsync(static_cast<char*>(h2->Red) + es * (size_t)Kn * h2->ldr, es * (size_t)h2->ldr, h->RB0,
                       es * (size_t)L, es * (size_t)L, (size_t)L, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return QRK_EHIP;
  h2->A = h->Rblk0;
  h2->B = h->Sc0;
  h2->b = h->c0;
  h2->d = h->d;
  h2->lam = lambda;
  h2->lam_ptr = h2->lam_d;
  h2->factored = true;
  if ((s = h->dtype == QRK_F32 ? factor_ba<float>(h2, st, &lambda) : factor_ba<double>(h2, st, &lambda)) != QRK_OK)
    return s;
  // the second-stage factor is the factor of [J; sqrt(lambda) D]: solves and refinement use it
  // with the original J
  if (hipMemcpyAsync(h->Rblk, h2->Rblk, es * (size_t)Kn * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h->Sc, h2->Sc, es * (size_t)Kn * L, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h->RB, h2->RB, es * (size_t)L * L, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h->status, h2->status, sizeof(int) * 4, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      launch_fill_double(h->lam_d, 1, lambda, st) != hipSuccess)
    return QRK_EHIP;
  h->lam = lambda;
  h->lam_ptr = h->lam_d;
  return QRK_OK;
}

}  // extern "C"

namespace {

template <typename T>
qrk_status factor_vcat(qrk_handle h, qrk_handle h2, hipStream_t st) {
  const size_t es = sizeof(T);
  const int n = h->n;
  const int L = h->nB + 1;
  const int64_t K = h->K, Kn = K * n;
  qrk_status s;
  if (!h->vcat_stage) {
    // the stage problem: K blocks of 2n rows ([R1_i; R2_i]) with coupled rows of stride L
    // ([S1_i | c1_i; S2_i | c2_i]); its dense part also takes the 2L rows of the two triangles
    // R1_B | c1_B and R2_B | c2_B after the blocks' reduced rows (2n per block: n of them are the
    // block's damping rows, zero here)
    std::vector<int64_t> ro((size_t)K + 1);
    for (int64_t i = 0; i <= K; ++i) ro[(size_t)i] = i * 2 * n;
    const int32_t K32 = (int32_t)K, nB32 = h->nB;
    qrk_handle hs = nullptr;
    if ((s = create_ba(1, n, &K32, &nB32, ro.data(), L, h->dtype, h->mode, &hs)) != QRK_OK) return s;
    hs->probs_h[0].M += 2 * L;
    hs->M += 2 * L;
    dfree(hs, hs->Red);
    hs->Red = nullptr;
    if ((s = dalloc(hs, &hs->Red, es * (size_t)(2 * Kn + 2 * L) * hs->ldr)) != QRK_OK ||
        (s = assign_leaves(hs)) != QRK_OK || (s = dalloc(h, &h->vA, es * (size_t)(2 * Kn * n))) != QRK_OK ||
        (s = dalloc(h, &h->vB, es * (size_t)(2 * Kn * L))) != QRK_OK ||
        (s = dalloc(h, &h->vb, es * (size_t)(2 * Kn))) != QRK_OK) {
      free_all(hs);
      delete hs;
      return s;
    }
    h->vcat_stage = hs;
  }
  qrk_handle hs = h->vcat_stage;
  if (launch_vcat_gather<T>(K, n, L, static_cast<const T*>(h->Rblk), static_cast<const T*>(h2->Rblk),
                            static_cast<const T*>(h->Sc), static_cast<const T*>(h2->Sc),
                            static_cast<const T*>(h->RB), static_cast<const T*>(h2->RB), static_cast<T*>(h->vA),
                            static_cast<T*>(h->vB), static_cast<T*>(h->vb), static_cast<T*>(hs->Red), 2 * Kn,
                            hs->ldr, st) != hipSuccess)
    return QRK_EHIP;
  hs->A = h->vA;
  hs->B = h->vB;
  hs->b = h->vb;
  hs->d = h->d;  // the stage's damping rows are zero (lambda = 0)
  hs->lam = 0.0;
  hs->lam_ptr = hs->lam_d;
  hs->factored = true;
  const double zero = 0.0;
  if ((s = factor_ba<T>(hs, st, &zero)) != QRK_OK) return s;
  // the stage's factor is the factor of the stacked rows
  if (hipMemcpyAsync(h->Rblk, hs->Rblk, es * (size_t)Kn * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h->Sc, hs->Sc, es * (size_t)Kn * L, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h->RB, hs->RB, es * (size_t)L * L, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h->status, hs->status, sizeof(int), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return QRK_EHIP;
  return QRK_OK;
}

}  // namespace

extern "C" {

qrk_status qrk_factor_vcat(qrk_handle h, qrk_handle h2, void* stream) {
  if (!h || !h2 || h == h2 || h->kind != KIND_BLOCKANGULAR || h2->kind != KIND_BLOCKANGULAR || h->P != 1 ||
      h2->P != 1 || !h->factored || !h2->factored || h->K != h2->K || h->n != h2->n || h->nB != h2->nB ||
      h->dtype != h2->dtype || !h2->vparts.empty() || h->vparts.size() >= 64 || h->ragged || h2->ragged ||
      h->camb || h2->camb)
    return QRK_EINVAL;
  for (qrk_handle q : h->vparts)
    if (q == h2) return QRK_EINVAL;
  hipStream_t st = S(stream);
  const qrk_status s = h->dtype == QRK_F32 ? factor_vcat<float>(h, h2, st) : factor_vcat<double>(h, h2, st);
  if (s != QRK_OK) return s;
  h->vparts.push_back(h2);
  h->q_valid = false;
  return QRK_OK;
}

qrk_status qrk_factor_blockangular_batched(qrk_handle h, const void* A, const void* B, const void* b,
                                           const double* d, const double* lambda_dev, void* stream) {
  if (!h || h->kind != KIND_BLOCKANGULAR || h->ragged || h->camb || !A || !b || !d || !lambda_dev)
    return QRK_EINVAL;
  if (h->max_L > 1 && !B) return QRK_EINVAL;
  h->A = A;
  h->B = B;
  h->b = b;
  h->d = d;
  h->lam_ptr = lambda_dev;
  h->factored = true;
  return h->dtype == QRK_F32 ? factor_ba<float>(h, S(stream)) : factor_ba<double>(h, S(stream));
}

qrk_status qrk_solve(qrk_handle h, double* p, int32_t sweeps, void* stream) {
  if (!h || !p || sweeps < 0 || sweeps > 8 || !h->factored) return QRK_EINVAL;
  if (h->ragged) {
    const qrk_status s = h->dtype == QRK_F32 ? solve_ba<float>(h, h->rg_p, sweeps, S(stream))
                                             : solve_ba<double>(h, h->rg_p, sweeps, S(stream));
    if (s != QRK_OK) return s;
    return launch_ragged_out(h->K, h->n, h->nB, h->rg_ncol, h->rg_poff, h->rg_p, p, S(stream)) == hipSuccess
               ? QRK_OK
               : QRK_EHIP;
  }
  if (h->kind == KIND_BLOCKANGULAR)
    return h->dtype == QRK_F32 ? solve_ba<float>(h, p, sweeps, S(stream))
                               : solve_ba<double>(h, p, sweeps, S(stream));
  return banded_solve(h, p, sweeps, S(stream));
}

qrk_status qrk_solve_rhs(qrk_handle h, const void* b, double* p, int32_t sweeps, void* stream) {
  if (!h || !b || !p || sweeps < 1 || sweeps > 8 || !h->factored || !h->vparts.empty() || h->ragged)
    return QRK_EINVAL;
  hipStream_t st = S(stream);
  const int64_t np = h->kind == KIND_BLOCKANGULAR ? h->N : (int64_t)h->P * h->N;
  if (launch_fill_double(p, np, 0.0, st) != hipSuccess) return QRK_EHIP;
  if (h->kind == KIND_BLOCKANGULAR)
    return h->dtype == QRK_F32 ? refine_ba<float>(h, p, sweeps, static_cast<const float*>(b), st)
                               : refine_ba<double>(h, p, sweeps, static_cast<const double*>(b), st);
  return banded_refine(h, p, sweeps, b, st);
}

qrk_status qrk_solve_adjoint(qrk_handle h, const double* p, const double* g, void* dA, void* dB,
                             void* db, double* dlambda, double* dd, void* stream) {
  if (!h || !h->factored || !p || !g || !h->vparts.empty() || h->ragged || h->camb) return QRK_EINVAL;
  if (h->kind == KIND_BLOCKANGULAR) {
    if (h->P != 1 || (dB && h->nB == 0)) return QRK_EINVAL;
    return blockangular_adjoint(h, p, g, dA, dB, db, dlambda, dd, S(stream));
  }
  if (dB) return QRK_EINVAL;
  return banded_adjoint(h, p, g, dA, db, dlambda, dd, S(stream));
}

static qrk_status colnorms_ba(qrk_handle h, const void* A, const void* B, const int32_t* cam, double* d,
                              void* stream) {
  const int nparts = (int)std::min<int64_t>(std::max<int64_t>(1, ceil_div(h->M, 512)), 1024);
  hipError_t e = h->dtype == QRK_F32
                     ? launch_colnorms<float>(h->K, h->n, h->nB, h->M, h->row_off_d,
                                              static_cast<const float*>(A), static_cast<const float*>(B),
                                              h->ldb, cam, d, h->vecpart, nparts, S(stream))
                     : launch_colnorms<double>(h->K, h->n, h->nB, h->M, h->row_off_d,
                                               static_cast<const double*>(A),
                                               static_cast<const double*>(B), h->ldb, cam, d, h->vecpart,
                                               nparts, S(stream));
  return e == hipSuccess ? QRK_OK : QRK_EHIP;
}

qrk_status qrk_colnorms_blockangular(qrk_handle h, const void* A, const void* B, double* d, void* stream) {
  if (!h || h->kind != KIND_BLOCKANGULAR || h->P != 1 || h->ragged || h->camb || !A || !d || (h->nB > 0 && !B))
    return QRK_EINVAL;
  return colnorms_ba(h, A, B, nullptr, d, stream);
}

qrk_status qrk_colnorms_blockangular_cam(qrk_handle h, const void* A, const void* Bv, const int32_t* cam, double* d,
                                         void* stream) {
  if (!h || h->kind != KIND_BLOCKANGULAR || h->P != 1 || !h->camb || !A || !Bv || !cam || !d) return QRK_EINVAL;
  return colnorms_ba(h, A, Bv, cam, d, stream);
}

qrk_status qrk_get_factor(qrk_handle h, void* Rblk, void* Sc, void* RB, void* stream) {
  if (!h || !h->factored) return QRK_EINVAL;
  const size_t es = h->dtype == QRK_F32 ? 4 : 8;
  hipStream_t st = S(stream);
  if (h->kind == KIND_BLOCKANGULAR) {
    if (h->P != 1) return QRK_EINVAL;
    const int L = h->nB + 1;
    if (Rblk && hipMemcpyAsync(Rblk, h->Rblk, es * (size_t)h->K * h->n * h->n,
                               hipMemcpyDeviceToDevice, st) != hipSuccess)
      return QRK_EHIP;
    if (Sc && hipMemcpyAsync(Sc, h->Sc, es * (size_t)h->K * h->n * L, hipMemcpyDeviceToDevice, st) !=
                  hipSuccess)
      return QRK_EHIP;
    if (RB && hipMemcpyAsync(RB, h->RB, es * (size_t)L * L, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return QRK_EHIP;
  } else {
    if (Rblk && hipMemcpyAsync(Rblk, h->bandR, es * (size_t)h->P * h->N * h->w,
                               hipMemcpyDeviceToDevice, st) != hipSuccess)
      return QRK_EHIP;
    if (Sc && hipMemcpyAsync(Sc, h->bandc, es * (size_t)h->P * h->N, hipMemcpyDeviceToDevice, st) !=
                  hipSuccess)
      return QRK_EHIP;
  }
  return hipStreamSynchronize(st) == hipSuccess ? QRK_OK : QRK_EHIP;
}

qrk_status qrk_status_get(qrk_handle h, int32_t* detail_host, void* stream) {
  if (!h) return QRK_EINVAL;
  const int nw = h->kind == KIND_BLOCKANGULAR ? h->P : 1;
  std::vector<int> words((size_t)nw, 0);
  hipStream_t st = S(stream);
  if (hipMemcpyAsync(words.data(), h->status, sizeof(int) * (size_t)nw, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QRK_EHIP;
  int bits = 0;
  for (int w : words) bits |= w;
  if (detail_host) *detail_host = bits;
  // a zero pivot also makes p non-finite, so singularity is reported first
  if (bits & ST_BADINPUT) return QRK_EINVAL;
  if (bits & ST_STALL) return QRK_EHIP;
  if (bits & ST_SINGULAR) return QRK_ESINGULAR;
  if (bits & ST_NONFINITE) return QRK_ENONFINITE;
  if (bits & ST_NOTCONVERGED) return QRK_ENOTCONVERGED;
  return QRK_OK;
}

qrk_status qrk_status_get_problems(qrk_handle h, int32_t* bits_host, void* stream) {
  if (!h || !bits_host) return QRK_EINVAL;
  const int nw = h->kind == KIND_BLOCKANGULAR ? h->P : 1;
  hipStream_t st = S(stream);
  if (hipMemcpyAsync(bits_host, h->status, sizeof(int) * (size_t)nw, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QRK_EHIP;
  return QRK_OK;
}

qrk_status qrk_set_tsqr_shape(qrk_handle h, int32_t leaves, int32_t fanin) {
  if (!h || leaves < 0 || fanin < 0 || fanin == 1 || fanin > 64) return QRK_EINVAL;
  if (h->kind != KIND_BLOCKANGULAR || h->P != 1 || leaves > h->max_leaves) return QRK_EINVAL;
  // the leaf tables and the merge-tree workspace are rewritten (and may be reallocated) below,
  // so nothing that reads them may still be in flight on any stream
  if (hipDeviceSynchronize() != hipSuccess) return QRK_EHIP;
  h->leaves = leaves;
  h->fanin = fanin ? fanin : 8;
  return assign_leaves(h);
}

qrk_status qrk_autotune_blockangular(qrk_handle h, double* scale_host, void* stream) {
  if (!h || h->kind != KIND_BLOCKANGULAR || !h->factored || h->dtype != QRK_F32) return QRK_EINVAL;
  hipStream_t st = S(stream);
  // as in qrk_set_tsqr_shape: no earlier work on any stream may still read the tables rewritten
  if (hipDeviceSynchronize() != hipSuccess) return QRK_EHIP;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return QRK_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return QRK_EHIP;
  }
  const int fixed = h->leaves;
  h->leaves = 0;
  const bool prof = h->prof_on;
  h->prof_on = false;
  qrk_status s = QRK_OK;
  // one timed configuration: the factor and a one-sweep solve (the step the LM loop takes),
  // best of two after a warm-up; p goes to the adjoint's scratch vector
  auto time_config = [&](double* ms_out) -> qrk_status {
    qrk_status r;
    if ((r = assign_leaves(h)) != QRK_OK || (r = assign_refine(h, true)) != QRK_OK) return r;
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) return QRK_EHIP;
      if ((r = factor_ba<float>(h, st)) != QRK_OK) return r;
      if ((r = blockangular_solve(h, h->ubuf, 1, st)) != QRK_OK) return r;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return QRK_EHIP;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return QRK_EHIP;
      if (rep > 0) best = std::min(best, ms);
    }
    *ms_out = best;
    return QRK_OK;
  };
  // coordinate search: rows per leaf, then the leaf queue (batches of several widths), then the
  // refinement workgroups, each from the best of the previous ones
  TuneChoice best;
  best.leaf_scale = h->leaf_scale;
  best.leaf_queue = h->leaf_queue;
  best.refine_scale = h->refine_scale;
  best.ms = 1e300;
  auto try_config = [&](double ls, int lq, double rs) {
    if (s != QRK_OK) return;
    h->leaf_scale = ls;
    h->leaf_queue = lq;
    h->refine_scale = rs;
    double ms = 0.0;
    s = time_config(&ms);
    if (s == QRK_OK && ms < best.ms) {
      best.leaf_scale = ls;
      best.leaf_queue = lq;
      best.refine_scale = rs;
      best.ms = ms;
    }
  };
  for (double ls : {0.5, 1.0, 2.0, 4.0}) try_config(ls, best.leaf_queue, best.refine_scale);
  if (h->widths > 1)
    for (int lq : {1, 0}) try_config(best.leaf_scale, lq, best.refine_scale);
  for (double rs : {0.5, 1.0, kMaxRefineScale}) try_config(best.leaf_scale, best.leaf_queue, rs);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->prof_on = prof;
  h->leaf_scale = best.leaf_scale;
  h->leaf_queue = best.leaf_queue;
  h->refine_scale = best.refine_scale;
  h->leaves = fixed;
  if (s == QRK_OK) s = assign_leaves(h);
  if (s == QRK_OK) s = assign_refine(h, true);
  if (s == QRK_OK) s = factor_ba<float>(h, st);
  if (s == QRK_OK) (void)tune_store(handle_tune_key(h), best);  // the file is best effort
  if (scale_host) *scale_host = best.leaf_scale;
  return s;
}

qrk_status qrk_tune_get(qrk_handle h, double* leaf_scale, int32_t* leaf_queue, double* refine_scale) {
  if (!h || h->kind != KIND_BLOCKANGULAR) return QRK_EINVAL;
  if (leaf_scale) *leaf_scale = h->leaf_scale;
  if (leaf_queue) *leaf_queue = h->leaf_queue;
  if (refine_scale) *refine_scale = h->refine_scale;
  return QRK_OK;
}

qrk_status qrk_tune_cache_file(const char* path) { return tune_set_file(path) ? QRK_OK : QRK_EINVAL; }

qrk_status qrk_profile_enable(qrk_handle h, int32_t max_calls) {
  if (!h || max_calls < 0 || max_calls > 100000) return QRK_EINVAL;
  prof_free(h);
  for (int i = 0; i < QRK_NPHASES; ++i) {
    h->prof_ms[i] = 0.0;
    h->prof_cnt[i] = 0;
  }
  if (max_calls == 0) return QRK_OK;
  const int nrec = max_calls * QRK_NPHASES;
  h->prof_pool.resize(nrec);
  for (auto& r : h->prof_pool) {
    if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) {
      prof_free(h);
      return QRK_EHIP;
    }
  }
  h->prof_on = true;
  return QRK_OK;
}

qrk_status qrk_profile_read(qrk_handle h, double* ms_host, int32_t* count_host, int32_t nphase) {
  if (!h || nphase < 0) return QRK_EINVAL;
  for (int i = 0; i < h->prof_used; ++i) {
    auto& r = h->prof_pool[i];
    if (hipEventSynchronize(r.stop) != hipSuccess) return QRK_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return QRK_EHIP;
    h->prof_ms[r.phase] += ms;
    h->prof_cnt[r.phase] += 1;
  }
  h->prof_used = 0;
  for (int i = 0; i < nphase && i < QRK_NPHASES; ++i) {
    if (ms_host) ms_host[i] = h->prof_ms[i];
    if (count_host) count_host[i] = h->prof_cnt[i];
    h->prof_ms[i] = 0.0;
    h->prof_cnt[i] = 0;
  }
  return QRK_OK;
}

int64_t qrk_workspace_bytes(qrk_handle h) { return h ? h->ws_bytes : 0; }

void qrk_destroy(qrk_handle h) {
  if (!h) return;
  free_all(h);
  delete h;
}

}  // extern "C"
