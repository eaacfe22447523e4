// Host side of the qrkit C ABI: argument validation, workspace ownership, launch
// selection and the device status word.  See include/qrkit.h for the contract.
#include "qrkit.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "qrk_launch.hpp"
#include "qrk_device.hpp"
#include "qrk_host.hpp"

using namespace qrk;

namespace {

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

qrk_status check_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return QRK_ENODEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return QRK_ENODEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return QRK_ENODEVICE;
  return QRK_OK;
}

template <typename T>
qrk_status factor_ba(qrk_handle h, hipStream_t st) {
  const T* A = static_cast<const T*>(h->A);
  const T* B = static_cast<const T*>(h->B);
  const T* b = static_cast<const T*>(h->b);
  T* Rblk = static_cast<T*>(h->Rblk);
  T* Sc = static_cast<T*>(h->Sc);
  T* Red = static_cast<T*>(h->Red);
  T* RB = static_cast<T*>(h->RB);
  T* P0 = static_cast<T*>(h->part0);
  T* P1 = static_cast<T*>(h->part1);
  const int L = h->nB + 1;
  const double sq = std::sqrt(h->lam);
  if (launch_fill_int(h->status, 0, st) != hipSuccess) return QRK_EHIP;
  int pr = prof_begin(h, 0, st);
  if (launch_blockqr<T>(h->K, h->n, h->nB, h->max_rows, h->row_off_d, A, B, h->ldb, b, h->d, sq,
                        Rblk, Sc, Red, h->ldr, h->grid_blocks, st) != hipSuccess)
    return QRK_EHIP;
  prof_end(h, pr, st);
  if constexpr (std::is_same<T, float>::value) {
    // dense part on the matrix cores: leaves and the merge tree in one launch
    pr = prof_begin(h, 1, st);
    if (launch_tsqr_mfma(Red, h->ldr, h->M, L, h->leaves, h->d + h->K * h->n, sq, h->slots,
                         h->counters, RB, st) != hipSuccess)
      return QRK_EHIP;
    prof_end(h, pr, st);
    return QRK_OK;
  }
  // dense part: leaves, then the reduction tree (ping-pong buffers, last level -> RB)
  int G = h->leaves;
  const int64_t rows_per = std::max<int64_t>(1, ceil_div(h->M, G));
  T* out = (G == 1) ? RB : P0;
  pr = prof_begin(h, 1, st);
  if (launch_tsqr_stream<T>(Red, h->ldr, h->M, L, rows_per, G, h->d + h->K * h->n, sq, out, st) !=
      hipSuccess)
    return QRK_EHIP;
  prof_end(h, pr, st);
  T* cur = out;
  T* other = P1;
  pr = prof_begin(h, 2, st);
  while (G > 1) {
    const int Gn = (int)ceil_div(G, h->fanin);
    T* dst = (Gn == 1) ? RB : other;
    if (launch_tsqr_stream<T>(cur, L, (int64_t)G * L, L, (int64_t)h->fanin * L, Gn, nullptr, 0.0,
                              dst, st) != hipSuccess)
      return QRK_EHIP;
    other = cur;
    cur = dst;
    G = Gn;
  }
  prof_end(h, pr, st);
  return QRK_OK;
}

template <typename T>
qrk_status solve_ba(qrk_handle h, double* p, int sweeps, hipStream_t st) {
  const T* Rblk = static_cast<const T*>(h->Rblk);
  const T* Sc = static_cast<const T*>(h->Sc);
  const T* RB = static_cast<const T*>(h->RB);
  const int L = h->nB + 1;
  const int64_t off = h->K * h->n;
  int pr = prof_begin(h, 3, st);
  if (launch_backsub_dense<T>(RB, L, p, off, h->status, st) != hipSuccess) return QRK_EHIP;
  if (launch_backsub_blocks<T>(h->K, h->n, h->nB, Rblk, Sc, p, h->status, h->solve_grid, st) !=
      hipSuccess)
    return QRK_EHIP;
  prof_end(h, pr, st);
  pr = sweeps > 0 ? prof_begin(h, 4, st) : -1;
  for (int s = 0; s < sweeps; ++s) {
    if (launch_refine_residual<T>(h->npacks, h->pack_blk, h->K, h->n, h->nB, h->row_off_d,
                                  static_cast<const T*>(h->A),
                                  static_cast<const T*>(h->B), h->ldb, static_cast<const T*>(h->b),
                                  h->d, h->lam, Rblk, Sc, p, h->ybuf, h->refpart, h->refine_grid,
                                  st) != hipSuccess)
      return QRK_EHIP;
    if (launch_refine_dense<T>(h->refine_grid, h->nB, h->refpart, RB, h->d, h->lam, p, off,
                               h->deltaB, st) != hipSuccess)
      return QRK_EHIP;
    if (launch_refine_blocks<T>(h->K, h->n, h->nB, Rblk, Sc, h->ybuf, h->deltaB, p,
                                h->solve_grid, st) != hipSuccess)
      return QRK_EHIP;
  }
  prof_end(h, pr, st);
  return QRK_OK;
}

// Leaf count of the dense-part QR: float32 leaves are single waves (about 128 rows
// each, at most 2048); float64 leaves are workgroups (about 256 rows, at most 1024).
int default_leaves(qrk_handle h) {
  const int64_t per = h->dtype == QRK_F32 ? 128 : 256;  // rows per leaf before the cap
  return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(h->M + h->nB, per), h->max_leaves));
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

}  // namespace

qrk_status handle_alloc(qrk_handle h, void** out, size_t bytes) { return dalloc(h, out, bytes); }
void handle_free(qrk_handle h) { free_all(h); }

template <typename T>
qrk_status adjoint_ba(qrk_handle h, const double* p, const double* g, void* dA, void* dB, void* db,
                      double* dlam, double* dd, hipStream_t st) {
  const T* Rblk = static_cast<const T*>(h->Rblk);
  const T* Sc = static_cast<const T*>(h->Sc);
  const T* RB = static_cast<const T*>(h->RB);
  const int64_t Kn = h->K * h->n;
  // u = (R^T R)^{-1} g through the structured R
  if (launch_adjoint_fwd_blocks<T>(h->K, h->n, h->nB, Rblk, Sc, g, h->ybuf, h->refpart, h->refine_grid,
                                   st) != hipSuccess)
    return QRK_EHIP;
  if (h->nB > 0 && launch_adjoint_dense<T>(h->refine_grid, h->nB, h->refpart, RB, g + Kn, h->ubuf + Kn,
                                           st) != hipSuccess)
    return QRK_EHIP;
  if (launch_adjoint_blocks<T>(h->K, h->n, h->nB, Rblk, Sc, h->ybuf, h->ubuf + Kn, h->ubuf, h->solve_grid,
                               st) != hipSuccess)
    return QRK_EHIP;
  if ((dA || dB || db) &&
      launch_adjoint_rows<T>(h->npacks, h->pack_blk, h->K, h->n, h->nB, h->row_off_d,
                             static_cast<const T*>(h->A), static_cast<const T*>(h->B), h->ldb,
                             static_cast<const T*>(h->b), p, h->ubuf, static_cast<T*>(dA),
                             static_cast<T*>(dB), static_cast<T*>(db), h->refine_grid, st) != hipSuccess)
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
  }
  return "unknown status";
}

qrk_status qrk_create_blockangular(int32_t K, int32_t n, int32_t nB, const int64_t* row_off_host,
                                   int64_t ldb, qrk_dtype dtype, qrk_mode mode, qrk_handle* out) {
  if (!out) return QRK_EINVAL;
  *out = nullptr;
  if (K < 1 || n < 1 || n > QRK_MAX_BLOCK_COLS || nB < 0 || nB > QRK_MAX_DENSE_COLS) return QRK_EINVAL;
  if (!row_off_host || ldb < nB || (dtype != QRK_F32 && dtype != QRK_F64)) return QRK_EINVAL;
  if (mode != QRK_PLAIN && mode != QRK_BF16X3) return QRK_EINVAL;
  if (mode == QRK_BF16X3 && dtype != QRK_F32) return QRK_EINVAL;
  if (row_off_host[0] != 0) return QRK_EINVAL;
  int max_m = 0;
  for (int32_t i = 0; i < K; ++i) {
    const int64_t m = row_off_host[i + 1] - row_off_host[i];
    if (m < 0 || m > QRK_MAX_BLOCK_ROWS) return QRK_EINVAL;
    max_m = std::max<int>(max_m, (int)m);
  }
  qrk_status ds = check_device();
  if (ds != QRK_OK) return ds;

  qrk_handle h = new (std::nothrow) qrk_handle_s();
  if (!h) return QRK_ENOMEM;
  h->kind = KIND_BLOCKANGULAR;
  h->dtype = dtype;
  h->mode = mode;
  h->K = K;
  h->n = n;
  h->nB = nB;
  h->M = row_off_host[K];
  h->N = (int64_t)K * n + nB;
  h->ldb = ldb;
  h->max_rows = max_m + n;
  const size_t es = dtype == QRK_F32 ? 4 : 8;
  const int L = nB + 1;
  h->ldr = ((L + 3) / 4) * 4;
  // packs of consecutive whole blocks, at most 64 rows and 64 blocks each (refinement)
  std::vector<int64_t> packs{0};
  {
    int64_t rows = 0;
    int nbp = 0;
    for (int32_t i = 0; i < K; ++i) {
      const int64_t m = row_off_host[i + 1] - row_off_host[i];
      if (nbp > 0 && (rows + m > 64 || nbp == 64)) {
        packs.push_back(i);
        rows = 0;
        nbp = 0;
      }
      rows += m;
      ++nbp;
    }
    packs.push_back(K);
  }
  h->npacks = (int64_t)packs.size() - 1;
  h->grid_blocks = (int)std::min<int64_t>(ceil_div(K, 4), 2048);
  h->solve_grid = (int)std::min<int64_t>(ceil_div(K, 16), 2048);
  h->refine_grid = (int)std::min<int64_t>(ceil_div(h->npacks, 4), 1024);
  h->max_leaves = 1024;  // float32: one leaf wave per SIMD of the 256-CU chip
  h->leaves = default_leaves(h);
  h->fanin = 8;
  qrk_status s = QRK_OK;
  if ((s = dalloc(h, &h->row_off_d, sizeof(int64_t) * (K + 1))) != QRK_OK ||
      (s = dalloc(h, &h->pack_blk, sizeof(int64_t) * packs.size())) != QRK_OK ||
      (s = dalloc(h, &h->Rblk, es * (size_t)K * n * n)) != QRK_OK ||
      (s = dalloc(h, &h->Sc, es * (size_t)K * n * L)) != QRK_OK ||
      (s = dalloc(h, &h->Red, es * (size_t)std::max<int64_t>(h->M, 1) * h->ldr)) != QRK_OK ||
      (s = dalloc(h, &h->RB, es * (size_t)L * L)) != QRK_OK ||
      (s = dalloc(h, &h->part0, dtype == QRK_F64 ? es * (size_t)1024 * L * L : 0)) != QRK_OK ||
      (s = dalloc(h, &h->part1, dtype == QRK_F64 ? es * (size_t)1024 * L * L : 0)) != QRK_OK ||
      (s = dalloc(h, &h->slots, dtype == QRK_F32 ? sizeof(float) * (size_t)2 * h->max_leaves *
                                                       tsqr_mfma_slot_floats(L)
                                                 : 0)) != QRK_OK ||
      (s = dalloc(h, &h->counters, sizeof(int) * (size_t)(2 * h->max_leaves + 2))) != QRK_OK ||
      (s = dalloc(h, &h->ybuf, sizeof(double) * (size_t)K * n)) != QRK_OK ||
      (s = dalloc(h, &h->ubuf, sizeof(double) * (size_t)h->N)) != QRK_OK ||
      (s = dalloc(h, &h->vecpart, sizeof(double) * (size_t)1024 * std::max(nB, 1))) != QRK_OK ||
      (s = dalloc(h, &h->refpart, sizeof(double) * (size_t)h->refine_grid * std::max(nB, 1))) != QRK_OK ||
      (s = dalloc(h, &h->deltaB, sizeof(double) * (size_t)std::max(nB, 1))) != QRK_OK ||
      (s = dalloc(h, &h->status, sizeof(int) * 4)) != QRK_OK) {
    free_all(h);
    delete h;
    return s;
  }
  if (hipMemcpy(h->row_off_d, row_off_host, sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(h->pack_blk, packs.data(), sizeof(int64_t) * packs.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemset(h->status, 0, sizeof(int) * 4) != hipSuccess) {
    free_all(h);
    delete h;
    return QRK_EHIP;
  }
  *out = h;
  return QRK_OK;
}

qrk_status qrk_factor_blockangular(qrk_handle h, const void* A, const void* B, const void* b,
                                   const double* d, double lambda, void* stream) {
  if (!h || h->kind != KIND_BLOCKANGULAR) return QRK_EINVAL;
  if (!A || !b || !d || (h->nB > 0 && !B)) return QRK_EINVAL;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return QRK_EINVAL;
  h->A = A;
  h->B = B;
  h->b = b;
  h->d = d;
  h->lam = lambda;
  h->factored = true;
  return h->dtype == QRK_F32 ? factor_ba<float>(h, S(stream)) : factor_ba<double>(h, S(stream));
}

qrk_status qrk_solve(qrk_handle h, double* p, int32_t sweeps, void* stream) {
  if (!h || !p || sweeps < 0 || sweeps > 8 || !h->factored) return QRK_EINVAL;
  if (h->kind == KIND_BLOCKANGULAR)
    return h->dtype == QRK_F32 ? solve_ba<float>(h, p, sweeps, S(stream))
                               : solve_ba<double>(h, p, sweeps, S(stream));
  return banded_solve(h, p, sweeps, S(stream));
}

qrk_status qrk_solve_adjoint(qrk_handle h, const double* p, const double* g, void* dA, void* dB,
                             void* db, double* dlambda, double* dd, void* stream) {
  if (!h || !h->factored || !p || !g) return QRK_EINVAL;
  if (h->kind == KIND_BLOCKANGULAR) {
    if (dB && h->nB == 0) return QRK_EINVAL;
    return blockangular_adjoint(h, p, g, dA, dB, db, dlambda, dd, S(stream));
  }
  if (dB) return QRK_EINVAL;
  return banded_adjoint(h, p, g, dA, db, dlambda, dd, S(stream));
}

qrk_status qrk_colnorms_blockangular(qrk_handle h, const void* A, const void* B, double* d, void* stream) {
  if (!h || h->kind != KIND_BLOCKANGULAR || !A || !d || (h->nB > 0 && !B)) return QRK_EINVAL;
  const int nparts = (int)std::min<int64_t>(std::max<int64_t>(1, ceil_div(h->M, 512)), 1024);
  hipError_t e = h->dtype == QRK_F32
                     ? launch_colnorms<float>(h->K, h->n, h->nB, h->M, h->row_off_d,
                                              static_cast<const float*>(A), static_cast<const float*>(B),
                                              h->ldb, d, h->vecpart, nparts, S(stream))
                     : launch_colnorms<double>(h->K, h->n, h->nB, h->M, h->row_off_d,
                                               static_cast<const double*>(A),
                                               static_cast<const double*>(B), h->ldb, d, h->vecpart,
                                               nparts, S(stream));
  return e == hipSuccess ? QRK_OK : QRK_EHIP;
}

qrk_status qrk_get_factor(qrk_handle h, void* Rblk, void* Sc, void* RB, void* stream) {
  if (!h || !h->factored) return QRK_EINVAL;
  const size_t es = h->dtype == QRK_F32 ? 4 : 8;
  hipStream_t st = S(stream);
  if (h->kind == KIND_BLOCKANGULAR) {
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
  int bits = 0;
  hipStream_t st = S(stream);
  if (hipMemcpyAsync(&bits, h->status, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QRK_EHIP;
  if (detail_host) *detail_host = bits;
  // a zero pivot also makes p non-finite, so singularity is reported first
  if (bits & ST_BADINPUT) return QRK_EINVAL;
  if (bits & ST_SINGULAR) return QRK_ESINGULAR;
  if (bits & ST_NONFINITE) return QRK_ENONFINITE;
  return QRK_OK;
}

qrk_status qrk_set_tsqr_shape(qrk_handle h, int32_t leaves, int32_t fanin) {
  if (!h || leaves < 0 || fanin < 0 || fanin == 1 || fanin > 64) return QRK_EINVAL;
  if (h->kind != KIND_BLOCKANGULAR || leaves > h->max_leaves) return QRK_EINVAL;
  h->leaves = leaves ? leaves : default_leaves(h);
  h->fanin = fanin ? fanin : 8;
  return QRK_OK;
}

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
