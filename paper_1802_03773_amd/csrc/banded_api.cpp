// Host side of the banded-J entry points (Givens QR of [J; sqrt(lam) D], banded solve,
// float64-residual refinement, adjoint).  P problems of identical shape may share one
// handle; their arrays are stacked (see include/qrkit.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

#include "qrk_banded.hpp"
#include "qrk_device.hpp"
#include "qrk_host.hpp"
#include "qrk_launch.hpp"
#include "qrkit.h"

using namespace qrk;

namespace {

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <typename T>
qrk_status banded_refine_t(qrk_handle h, double* p, int sweeps, const T* b, hipStream_t st);

template <typename T>
qrk_status banded_solve_t(qrk_handle h, double* p, int sweeps, hipStream_t st) {
  const T* R = static_cast<const T*>(h->bandR);
  const T* c = static_cast<const T*>(h->bandc);
  int pr = prof_begin(h, 3, st);
  const T* R16 = static_cast<const T*>(h->bandR16);
  if (launch_banded_backsub<T>(h->P, h->N, h->w, R, R16, h->bandinv, c, p, h->status, st) != hipSuccess)
    return QRK_EHIP;
  prof_end(h, pr, st);
  return banded_refine_t<T>(h, p, sweeps, static_cast<const T*>(h->b), st);
}

// `sweeps` corrected semi-normal sweeps for the right-hand side b.
template <typename T>
qrk_status banded_refine_t(qrk_handle h, double* p, int sweeps, const T* b, hipStream_t st) {
  const T* R = static_cast<const T*>(h->bandR);
  const T* R16 = static_cast<const T*>(h->bandR16);
  int pr = sweeps > 0 ? prof_begin(h, 4, st) : -1;
  for (int s = 0; s < sweeps; ++s) {
    // r = b - J p; g = J^T r - lam D^2 p; y = R^{-T} g; p += R^{-1} y
    if (launch_banded_apply<T>(h->P, h->M, h->N, h->w, h->row_start, static_cast<const T*>(h->A), b, p, h->rbuf,
                               st) != hipSuccess ||
        launch_banded_jt<T>(h->P, h->M, h->N, h->w, h->row_start, h->bandfr, static_cast<const T*>(h->A), h->rbuf,
                            h->d, h->lam_ptr, p, h->gbuf, st) != hipSuccess ||
        launch_banded_fwd<T>(h->P, h->N, h->w, R, R16, h->bandinv, h->gbuf, h->gbuf, st) != hipSuccess ||
        launch_banded_solve_add<T>(h->P, h->N, h->w, R, R16, h->bandinv, h->gbuf, p, st) != hipSuccess)
      return QRK_EHIP;
  }
  prof_end(h, pr, st);
  return QRK_OK;
}

template <typename T>
qrk_status banded_adjoint_t(qrk_handle h, const double* p, const double* g, void* dvals, void* db,
                            double* dlam, double* dd, hipStream_t st) {
  const T* R = static_cast<const T*>(h->bandR);
  const T* R16 = static_cast<const T*>(h->bandR16);
  const int64_t PN = (int64_t)h->P * h->N, PM = (int64_t)h->P * h->M;
  // u = R^{-1} R^{-T} g
  if (launch_banded_fwd<T>(h->P, h->N, h->w, R, R16, h->bandinv, g, h->gbuf, st) != hipSuccess ||
      launch_fill_double(h->ubuf, PN, 0.0, st) != hipSuccess ||
      launch_banded_solve_add<T>(h->P, h->N, h->w, R, R16, h->bandinv, h->gbuf, h->ubuf, st) != hipSuccess)
    return QRK_EHIP;
  const T* vals = static_cast<const T*>(h->A);
  if (dvals || db) {
    if (launch_banded_apply<T>(h->P, h->M, h->N, h->w, h->row_start, vals, nullptr, h->ubuf, h->jubuf, st) !=
        hipSuccess)
      return QRK_EHIP;
  }
  if (dvals) {
    if (launch_banded_apply<T>(h->P, h->M, h->N, h->w, h->row_start, vals, static_cast<const T*>(h->b), p,
                               h->rbuf, st) != hipSuccess ||
        launch_banded_dvals<T>(h->P, h->M, h->N, h->w, h->row_start, h->rbuf, h->jubuf, h->ubuf, p,
                               static_cast<T*>(dvals), st) != hipSuccess)
      return QRK_EHIP;
  }
  if (db && launch_to_type<T>(h->jubuf, static_cast<T*>(db), PM, st) != hipSuccess) return QRK_EHIP;
  if ((dlam || dd) &&
      launch_adjoint_vec(h->P, h->N, h->ubuf, h->d, p, h->lam, dd, dlam, h->vecpart, st) != hipSuccess)
    return QRK_EHIP;
  return QRK_OK;
}

qrk_status create_banded(int32_t P, int64_t M, int64_t N, int32_t w, qrk_dtype dtype, qrk_handle* out) {
  if (!out) return QRK_EINVAL;
  *out = nullptr;
  if (P < 1 || M < 0 || N < 1 || w < 1 || w > QRK_MAX_BAND || w > N) return QRK_EINVAL;
  if (dtype != QRK_F32 && dtype != QRK_F64) return QRK_EINVAL;
  int dev = -1;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
    return QRK_ENODEVICE;
  qrk_handle h = new (std::nothrow) qrk_handle_s();
  if (!h) return QRK_ENOMEM;
  h->kind = KIND_BANDED;
  h->dtype = dtype;
  h->P = P;
  h->M = M;
  h->N = N;
  h->w = w;
  const size_t es = dtype == QRK_F32 ? 4 : 8;
  const size_t PN = (size_t)P * N, PM = (size_t)P * (M > 0 ? M : 1);
  qrk_status s;
  if ((s = handle_alloc(h, &h->bandR, es * PN * w)) != QRK_OK ||
      (s = handle_alloc(h, &h->bandc, es * PN)) != QRK_OK ||
      (s = handle_alloc(h, reinterpret_cast<void**>(&h->bandinv), sizeof(double) * PN)) != QRK_OK ||
      (s = handle_alloc(h, reinterpret_cast<void**>(&h->bandfr), sizeof(int32_t) * (size_t)P * (N + 1))) != QRK_OK ||
      (s = handle_alloc(h, reinterpret_cast<void**>(&h->rbuf), sizeof(double) * PM)) != QRK_OK ||
      (s = handle_alloc(h, reinterpret_cast<void**>(&h->jubuf), sizeof(double) * PM)) != QRK_OK ||
      (s = handle_alloc(h, reinterpret_cast<void**>(&h->gbuf), sizeof(double) * PN)) != QRK_OK ||
      (s = handle_alloc(h, reinterpret_cast<void**>(&h->ubuf), sizeof(double) * PN)) != QRK_OK ||
      (s = handle_alloc(h, reinterpret_cast<void**>(&h->vecpart),
                        sizeof(double) * (size_t)(P > 1024 ? P : 1024))) != QRK_OK ||
      (s = handle_alloc(h, reinterpret_cast<void**>(&h->lam_d), sizeof(double) * (size_t)P)) != QRK_OK ||
      (s = handle_alloc(h, reinterpret_cast<void**>(&h->status), sizeof(int) * 4)) != QRK_OK) {
    handle_free(h);
    delete h;
    return s;
  }
  if (hipMemset(h->status, 0, sizeof(int) * 4) != hipSuccess) {
    handle_free(h);
    delete h;
    return QRK_EHIP;
  }
  // bands up to 15 keep a padded sweep copy of R (zeroed once; the padding stays zero)
  if (bsweep_w_fits(P, N, w, es)) {
    void* r16 = nullptr;
    const size_t bytes = es * 16 * ((size_t)P * N + 2 * kBandPad);
    if ((s = handle_alloc(h, &r16, bytes)) != QRK_OK || hipMemset(r16, 0, bytes) != hipSuccess) {
      handle_free(h);
      delete h;
      return s != QRK_OK ? s : QRK_EHIP;
    }
    h->bandR16 = static_cast<char*>(r16) + es * 16 * kBandPad;
  }
  *out = h;
  return QRK_OK;
}

}  // namespace

qrk_status banded_solve(qrk_handle h, double* p, int sweeps, hipStream_t st) {
  return h->dtype == QRK_F32 ? banded_solve_t<float>(h, p, sweeps, st) : banded_solve_t<double>(h, p, sweeps, st);
}

qrk_status banded_refine(qrk_handle h, double* p, int sweeps, const void* b, hipStream_t st) {
  return h->dtype == QRK_F32 ? banded_refine_t<float>(h, p, sweeps, static_cast<const float*>(b), st)
                             : banded_refine_t<double>(h, p, sweeps, static_cast<const double*>(b), st);
}

qrk_status banded_adjoint(qrk_handle h, const double* p, const double* g, void* dvals, void* db,
                          double* dlam, double* dd, hipStream_t st) {
  return h->dtype == QRK_F32 ? banded_adjoint_t<float>(h, p, g, dvals, db, dlam, dd, st)
                             : banded_adjoint_t<double>(h, p, g, dvals, db, dlam, dd, st);
}

extern "C" {

qrk_status qrk_create_banded(int64_t M, int64_t N, int32_t w, qrk_dtype dtype, qrk_handle* out) {
  return create_banded(1, M, N, w, dtype, out);
}

qrk_status qrk_create_banded_batched(int32_t P, int64_t M, int64_t N, int32_t w, qrk_dtype dtype,
                                     qrk_handle* out) {
  return create_banded(P, M, N, w, dtype, out);
}

qrk_status qrk_set_banded_method(qrk_handle h, int32_t method) {
  if (!h || h->kind != KIND_BANDED || method < 0 || method > 2) return QRK_EINVAL;
  if (method != 0 && (h->dtype != QRK_F32 || h->w > 15)) return QRK_EINVAL;
  h->band_method = method;
  return QRK_OK;
}

qrk_status qrk_factor_banded(qrk_handle h, const int32_t* row_start, const void* vals, const void* b,
                             const double* d, double lambda, void* stream) {
  if (!h || h->kind != KIND_BANDED) return QRK_EINVAL;
  if ((h->M > 0 && (!row_start || !vals || !b)) || !d) return QRK_EINVAL;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return QRK_EINVAL;
  h->row_start = row_start;
  h->A = vals;
  h->b = b;
  h->d = d;
  h->lam = lambda;
  h->factored = true;
  hipStream_t st = S(stream);
  if (launch_fill_double(h->lam_d, h->P, lambda, st) != hipSuccess) return QRK_EHIP;
  h->lam_ptr = h->lam_d;
  return banded_factor(h, st);
}

}  // extern "C"

// Givens QR of every problem of a banded handle with its current (borrowed) inputs and
// the damping at h->lam_ptr ([P], device).
qrk_status banded_factor(qrk_handle h, hipStream_t st) {
  if (launch_fill_int(h->status, 0, st) != hipSuccess) return QRK_EHIP;
  const int32_t* row_start = h->row_start;
  const void* vals = h->A;
  const void* b = h->b;
  const double* d = h->d;
  int pr = prof_begin(h, 5, st);
  if (launch_band_first_row(h->P, h->M, h->N, h->w, row_start, h->bandfr, st) != hipSuccess) return QRK_EHIP;
  if (h->band_method != 0) {
    const hipError_t ew = launch_bwy<float>(h->band_method == 2, h->P, h->M, h->N, h->w, row_start,
                                            static_cast<const float*>(vals), static_cast<const float*>(b), d,
                                            h->lam_ptr, static_cast<float*>(h->bandR), static_cast<float*>(h->bandc),
                                            h->bandinv, static_cast<float*>(h->bandR16), h->status, st);
    prof_end(h, pr, st);
    return ew == hipSuccess ? QRK_OK : QRK_EHIP;
  }
  hipError_t e = h->dtype == QRK_F32
                     ? launch_banded_givens<float>(h->P, h->M, h->N, h->w, row_start,
                                                   static_cast<const float*>(vals),
                                                   static_cast<const float*>(b), d, h->lam_ptr,
                                                   static_cast<float*>(h->bandR),
                                                   static_cast<float*>(h->bandc), h->bandinv,
                                                   static_cast<float*>(h->bandR16), h->status, st)
                     : launch_banded_givens<double>(h->P, h->M, h->N, h->w, row_start,
                                                    static_cast<const double*>(vals),
                                                    static_cast<const double*>(b), d, h->lam_ptr,
                                                    static_cast<double*>(h->bandR),
                                                    static_cast<double*>(h->bandc), h->bandinv,
                                                    static_cast<double*>(h->bandR16), h->status, st);
  prof_end(h, pr, st);
  return e == hipSuccess ? QRK_OK : QRK_EHIP;
}
