// Host side of the Levenberg-Marquardt driver (block-angular and banded handles): state ownership, one iteration as a sequence
// of stream-ordered launches (model evaluation, the structured factor and solve, gain ratio
// and damping update), and its capture into a HIP graph that is replayed per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "qrk_banded.hpp"
#include "qrk_device.hpp"
#include "qrk_host.hpp"
#include "qrk_launch.hpp"
#include "qrk_lm.hpp"
#include "qrkit.h"

using namespace qrk;

struct qrk_lm_s {
  qrk_handle h = nullptr;
  const void* A0 = nullptr;  // block-angular: A0; banded: vals0
  const void* B0 = nullptr;
  const int32_t* row_start = nullptr;  // banded
  const void* y = nullptr;
  double c = 0.0;
  int sweeps = 1;
  int max_log = 0;
  void* A = nullptr;  // J(x), the handle's layouts and storage type
  void* B = nullptr;
  void* b = nullptr;  // -f(x)
  double *x = nullptr, *p = nullptr, *d = nullptr, *gJ = nullptr;
  double *F = nullptr, *Fnew = nullptr, *pred = nullptr, *lam = nullptr, *nu = nullptr;
  double *part = nullptr, *fpart = nullptr, *log = nullptr;
  double* predpart = nullptr;  // per-workgroup parts of the predicted decrease
  int64_t maxN = 0;            // unknowns of the largest problem
  double* f = nullptr;  // banded: f(x) per row
  int *acc = nullptr, *iter = nullptr;
  int64_t* noff = nullptr;
  std::vector<void*> allocs;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t shape_gen = 0;  // the handle's leaf-layout generation the graph was captured with
};

namespace {

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Unknowns over all problems (banded handles keep N per problem).
int64_t lm_unknowns(qrk_lm lm) { return lm->h->kind == KIND_BANDED ? (int64_t)lm->h->P * lm->h->N : lm->h->N; }

template <typename P>
qrk_status lm_alloc(qrk_lm lm, P** out, size_t bytes) {
  void* ptr = nullptr;
  if (hipMalloc(&ptr, bytes < 256 ? 256 : bytes) != hipSuccess) return QRK_ENOMEM;
  lm->allocs.push_back(ptr);
  *out = static_cast<P*>(ptr);
  return QRK_OK;
}

void lm_free(qrk_lm lm) {
  if (lm->exec) (void)hipGraphExecDestroy(lm->exec);
  if (lm->graph) (void)hipGraphDestroy(lm->graph);
  if (lm->cap) (void)hipStreamDestroy(lm->cap);
  for (void* ptr : lm->allocs) (void)hipFree(ptr);
  lm->allocs.clear();
}

// One LM iteration, enqueued on st (eagerly, or into a graph under capture).
template <typename T>
qrk_status lm_iteration(qrk_lm lm, hipStream_t st) {
  qrk_handle h = lm->h;
  BatchView bv = blockangular_view(h);
  bv.lam = lm->lam;
  T* A = static_cast<T*>(lm->A);
  T* B = static_cast<T*>(lm->B);
  T* b = static_cast<T*>(lm->b);
  const T* A0 = static_cast<const T*>(lm->A0);
  const T* B0 = static_cast<const T*>(lm->B0);
  const T* y = static_cast<const T*>(lm->y);
  if (launch_lmba_eval<T>(bv, true, A0, B0, y, lm->c, lm->x, nullptr, A, B, b, lm->d, lm->gJ, lm->part, lm->fpart,
                          lm->F, st) != hipSuccess)
    return QRK_EHIP;
  h->A = A;
  h->B = B;
  h->b = b;
  h->d = lm->d;
  h->lam_ptr = lm->lam;
  h->factored = true;
  qrk_status s;
  if ((s = blockangular_factor(h, st)) != QRK_OK) return s;
  if ((s = blockangular_solve(h, lm->p, lm->sweeps, st)) != QRK_OK) return s;
  if (launch_lm_control(h->P, lm->maxN, lm->noff, lm->p, lm->d, lm->gJ, lm->lam, lm->nu, lm->F, lm->Fnew, lm->pred,
                        lm->predpart, lm->acc,
                        lm->iter, lm->log, lm->max_log, lm->x, st, 0) != hipSuccess)
    return QRK_EHIP;
  if (launch_lmba_eval<T>(bv, false, A0, B0, y, lm->c, lm->x, lm->p, A, B, b, lm->d, lm->gJ, lm->part, lm->fpart,
                          lm->Fnew, st) != hipSuccess)
    return QRK_EHIP;
  if (launch_lm_control(h->P, lm->maxN, lm->noff, lm->p, lm->d, lm->gJ, lm->lam, lm->nu, lm->F, lm->Fnew, lm->pred,
                        lm->predpart, lm->acc,
                        lm->iter, lm->log, lm->max_log, lm->x, st, 1) != hipSuccess)
    return QRK_EHIP;
  return QRK_OK;
}

// One LM iteration on a banded handle (P stacked problems).
template <typename T>
qrk_status lm_iteration_banded(qrk_lm lm, hipStream_t st) {
  qrk_handle h = lm->h;
  T* vals = static_cast<T*>(lm->A);
  T* b = static_cast<T*>(lm->b);
  const T* vals0 = static_cast<const T*>(lm->A0);
  const T* y = static_cast<const T*>(lm->y);
  if (launch_band_first_row(h->P, h->M, h->N, h->w, lm->row_start, h->bandfr, st) != hipSuccess ||
      launch_lmbd_eval<T>(h->P, h->M, h->N, h->w, true, lm->row_start, h->bandfr, vals0, y, lm->c, lm->x, nullptr,
                          vals, b, lm->f, lm->d, lm->gJ, lm->fpart, lm->F, st) != hipSuccess)
    return QRK_EHIP;
  h->row_start = lm->row_start;
  h->A = vals;
  h->b = b;
  h->d = lm->d;
  h->lam_ptr = lm->lam;
  h->factored = true;
  qrk_status s;
  if ((s = banded_factor(h, st)) != QRK_OK) return s;
  if ((s = banded_solve(h, lm->p, lm->sweeps, st)) != QRK_OK) return s;
  if (launch_lm_control(h->P, lm->maxN, lm->noff, lm->p, lm->d, lm->gJ, lm->lam, lm->nu, lm->F, lm->Fnew, lm->pred,
                        lm->predpart, lm->acc,
                        lm->iter, lm->log, lm->max_log, lm->x, st, 0) != hipSuccess)
    return QRK_EHIP;
  if (launch_lmbd_eval<T>(h->P, h->M, h->N, h->w, false, lm->row_start, h->bandfr, vals0, y, lm->c, lm->x, lm->p,
                          vals, b, lm->f, lm->d, lm->gJ, lm->fpart, lm->Fnew, st) != hipSuccess)
    return QRK_EHIP;
  if (launch_lm_control(h->P, lm->maxN, lm->noff, lm->p, lm->d, lm->gJ, lm->lam, lm->nu, lm->F, lm->Fnew, lm->pred,
                        lm->predpart, lm->acc,
                        lm->iter, lm->log, lm->max_log, lm->x, st, 1) != hipSuccess)
    return QRK_EHIP;
  return QRK_OK;
}

qrk_status lm_enqueue(qrk_lm lm, hipStream_t st) {
  if (lm->h->kind == KIND_BANDED)
    return lm->h->dtype == QRK_F32 ? lm_iteration_banded<float>(lm, st) : lm_iteration_banded<double>(lm, st);
  return lm->h->dtype == QRK_F32 ? lm_iteration<float>(lm, st) : lm_iteration<double>(lm, st);
}

// State shared by both structures: x, p, d, J^T f (N_tot), per-problem scalars, the log and
// the unknown offsets of the problems.
qrk_status lm_alloc_common(qrk_lm lm, const std::vector<int64_t>& noff) {
  const size_t P = (size_t)noff.size() - 1, N = (size_t)noff.back();
  qrk_status s;
  if ((s = lm_alloc(lm, &lm->x, sizeof(double) * N)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->p, sizeof(double) * N)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->d, sizeof(double) * N)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->gJ, sizeof(double) * N)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->F, sizeof(double) * P)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->Fnew, sizeof(double) * P)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->pred, sizeof(double) * P)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->lam, sizeof(double) * P)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->nu, sizeof(double) * P)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->acc, sizeof(int) * P)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->iter, sizeof(int))) != QRK_OK ||
      (s = lm_alloc(lm, &lm->log, sizeof(double) * (size_t)(lm->max_log > 0 ? lm->max_log : 1) * P * 4)) !=
          QRK_OK ||
      (s = lm_alloc(lm, &lm->noff, sizeof(int64_t) * (P + 1))) != QRK_OK)
    return s;
  for (size_t q = 0; q < P; ++q) lm->maxN = std::max<int64_t>(lm->maxN, noff[q + 1] - noff[q]);
  if ((s = lm_alloc(lm, &lm->predpart, sizeof(double) * (size_t)P * lm_pred_blocks(lm->maxN))) != QRK_OK) return s;
  if (hipMemcpy(lm->noff, noff.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipStreamCreateWithFlags(&lm->cap, hipStreamNonBlocking) != hipSuccess)
    return QRK_EHIP;
  return QRK_OK;
}

}  // namespace

extern "C" {

qrk_status qrk_lm_create_blockangular(qrk_handle h, const void* A0, const void* B0, const void* y, double c,
                                      int32_t sweeps, int32_t max_log, qrk_lm* out) {
  if (!out) return QRK_EINVAL;
  *out = nullptr;
  if (!h || h->kind != KIND_BLOCKANGULAR || h->ragged || h->camb || !A0 || !y || (h->max_L > 1 && !B0))
    return QRK_EINVAL;
  if (!std::isfinite(c) || sweeps < 0 || sweeps > 8 || max_log < 0) return QRK_EINVAL;
  qrk_lm lm = new (std::nothrow) qrk_lm_s();
  if (!lm) return QRK_ENOMEM;
  lm->h = h;
  lm->A0 = A0;
  lm->B0 = B0;
  lm->y = y;
  lm->c = c;
  lm->sweeps = sweeps;
  lm->max_log = max_log;
  const size_t es = h->dtype == QRK_F32 ? 4 : 8;
  int64_t btot = 0;
  std::vector<int64_t> noff(h->P + 1, 0);
  for (int q = 0; q < h->P; ++q) {
    const ProbDesc& D = h->probs_h[q];
    btot += D.M * D.ldb;
    noff[q + 1] = D.noff + D.K * h->n + D.nB;
  }
  qrk_status s;
  if ((s = lm_alloc(lm, &lm->A, es * (size_t)h->M * h->n)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->B, es * (size_t)btot)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->b, es * (size_t)h->M)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->part, sizeof(double) * (size_t)h->nwg_cap * 2 * kMaxDense)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->fpart, sizeof(double) * (size_t)std::max<int64_t>(h->npacks, 1))) != QRK_OK ||
      (s = lm_alloc_common(lm, noff)) != QRK_OK) {
    lm_free(lm);
    delete lm;
    return s;
  }
  *out = lm;
  return QRK_OK;
}

qrk_status qrk_lm_create_banded(qrk_handle h, const int32_t* row_start, const void* vals0, const void* y, double c,
                                int32_t sweeps, int32_t max_log, qrk_lm* out) {
  if (!out) return QRK_EINVAL;
  *out = nullptr;
  if (!h || h->kind != KIND_BANDED || !row_start || !vals0 || !y || h->M < 1) return QRK_EINVAL;
  if (!std::isfinite(c) || sweeps < 0 || sweeps > 8 || max_log < 0) return QRK_EINVAL;
  qrk_lm lm = new (std::nothrow) qrk_lm_s();
  if (!lm) return QRK_ENOMEM;
  lm->h = h;
  lm->A0 = vals0;
  lm->row_start = row_start;
  lm->y = y;
  lm->c = c;
  lm->sweeps = sweeps;
  lm->max_log = max_log;
  const size_t es = h->dtype == QRK_F32 ? 4 : 8;
  const size_t PM = (size_t)h->P * h->M;
  std::vector<int64_t> noff(h->P + 1, 0);
  for (int q = 0; q < h->P; ++q) noff[q + 1] = noff[q] + h->N;
  const size_t nblk = (size_t)((h->M + 255) / 256);
  qrk_status s;
  if ((s = lm_alloc(lm, &lm->A, es * PM * h->w)) != QRK_OK || (s = lm_alloc(lm, &lm->b, es * PM)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->f, sizeof(double) * PM)) != QRK_OK ||
      (s = lm_alloc(lm, &lm->fpart, sizeof(double) * nblk * h->P)) != QRK_OK ||
      (s = lm_alloc_common(lm, noff)) != QRK_OK) {
    lm_free(lm);
    delete lm;
    return s;
  }
  *out = lm;
  return QRK_OK;
}

qrk_status qrk_lm_reset(qrk_lm lm, const double* x0, const double* lambda0, void* stream) {
  if (!lm || !x0 || !lambda0) return QRK_EINVAL;
  hipStream_t st = S(stream);
  const int P = lm->h->P;
  if (hipMemcpyAsync(lm->x, x0, sizeof(double) * (size_t)lm_unknowns(lm), hipMemcpyDeviceToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(lm->lam, lambda0, sizeof(double) * (size_t)P, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      launch_lm_init(P, lm->nu, lm->iter, st) != hipSuccess ||
      launch_fill_double(lm->log, (int64_t)(lm->max_log > 0 ? lm->max_log : 1) * P * 4, 0.0, st) != hipSuccess)
    return QRK_EHIP;
  return QRK_OK;
}

qrk_status qrk_lm_run(qrk_lm lm, int32_t iters, int32_t use_graph, void* stream) {
  if (!lm || iters < 0) return QRK_EINVAL;
  hipStream_t st = S(stream);
  qrk_handle h = lm->h;
  if (!use_graph) {
    for (int k = 0; k < iters; ++k) {
      qrk_status s = lm_enqueue(lm, st);
      if (s != QRK_OK) return s;
    }
    return QRK_OK;
  }
  if (lm->exec && lm->shape_gen != h->shape_gen) {
    // the leaf layout changed since the capture (qrk_set_tsqr_shape / qrk_autotune_blockangular):
    // the graph holds the old launch geometry and workspace pointers, so capture again
    if (hipStreamSynchronize(st) != hipSuccess) return QRK_EHIP;
    (void)hipGraphExecDestroy(lm->exec);
    (void)hipGraphDestroy(lm->graph);
    lm->exec = nullptr;
    lm->graph = nullptr;
  }
  if (!lm->exec) {
    // capture one iteration on the driver's own stream (phase timing off: no event nodes)
    lm->shape_gen = h->shape_gen;
    const bool prof = h->prof_on;
    h->prof_on = false;
    if (hipStreamBeginCapture(lm->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      h->prof_on = prof;
      return QRK_EHIP;
    }
    qrk_status s = lm_enqueue(lm, lm->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(lm->cap, &g);
    h->prof_on = prof;
    if (s != QRK_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return s != QRK_OK ? s : QRK_EHIP;
    }
    lm->graph = g;
    if (hipGraphInstantiate(&lm->exec, lm->graph, nullptr, nullptr, 0) != hipSuccess) {
      lm->exec = nullptr;
      return QRK_EHIP;
    }
  }
  for (int k = 0; k < iters; ++k)
    if (hipGraphLaunch(lm->exec, st) != hipSuccess) return QRK_EHIP;
  return QRK_OK;
}

qrk_status qrk_lm_get(qrk_lm lm, double* x, double* lambda, double* log, int32_t* iters_host, void* stream) {
  if (!lm) return QRK_EINVAL;
  hipStream_t st = S(stream);
  const size_t P = (size_t)lm->h->P;
  if (x && hipMemcpyAsync(x, lm->x, sizeof(double) * (size_t)lm_unknowns(lm), hipMemcpyDeviceToDevice, st) !=
               hipSuccess)
    return QRK_EHIP;
  if (lambda && hipMemcpyAsync(lambda, lm->lam, sizeof(double) * P, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return QRK_EHIP;
  if (log && lm->max_log > 0 &&
      hipMemcpyAsync(log, lm->log, sizeof(double) * (size_t)lm->max_log * P * 4, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    return QRK_EHIP;
  if (iters_host) {
    int it = 0;
    if (hipMemcpyAsync(&it, lm->iter, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return QRK_EHIP;
    *iters_host = it;
  }
  return QRK_OK;
}

void qrk_lm_destroy(qrk_lm lm) {
  if (!lm) return;
  lm_free(lm);
  delete lm;
}

}  // extern "C"
