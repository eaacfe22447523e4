// Launchers of the banded-J kernels (internal to libqrkit.so).  P problems of identical
// shape are stacked: row_start [P][M], vals [P][M][w], b [P][M], d and p [P][N],
// R band [P][N][w] (row j holds R[j][j .. j+w-1]), c [P][N].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrk {

template <typename T>
hipError_t launch_banded_givens(int P, int64_t M, int64_t N, int w, const int32_t* row_start,
                                const T* vals, const T* b, const double* d, const double* lam, T* Rb,
                                T* cb, double* binv, T* R16, int* status, hipStream_t st);
// p = R^{-1} c (status: singular pivots, non-finite results)
template <typename T>
hipError_t launch_banded_backsub(int P, int64_t N, int w, const T* Rb, const T* R16, const double* binv, const T* cb,
                                 double* p, int* status, hipStream_t st);
// out += R^{-1} rhs
template <typename T>
hipError_t launch_banded_solve_add(int P, int64_t N, int w, const T* Rb, const T* R16, const double* binv,
                                   const double* rhs, double* out, hipStream_t st);
// y = R^{-T} g
template <typename T>
hipError_t launch_banded_fwd(int P, int64_t N, int w, const T* Rb, const T* R16, const double* binv, const double* g,
                             double* y, hipStream_t st);
// r = b - J v (or J v when b is null), float64, [P][M]
template <typename T>
hipError_t launch_banded_apply(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                               const T* b, const double* v, double* r, hipStream_t st);
// first-row table fr [P][N+1]: fr[c] = first row whose start is >= c
hipError_t launch_band_first_row(int P, int64_t M, int64_t N, int w, const int32_t* row_start, int32_t* fr,
                                 hipStream_t st);
// g = J^T r - lam d^2 v, float64, [P][N] (fr: the first-row table of row_start)
template <typename T>
hipError_t launch_banded_jt(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const int32_t* fr,
                            const T* vals, const double* r, const double* d, const double* lam, const double* v,
                            double* g, hipStream_t st);
// dvals[i][l] = r_i u_{s_i+l} - (J u)_i p_{s_i+l}
template <typename T>
hipError_t launch_banded_dvals(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const double* r,
                               const double* Ju, const double* u, const double* p, T* dvals, hipStream_t st);

// Block-banded QR on the matrix cores (w <= 15, float32 only; banded_wy.hip): the same outputs
// as launch_banded_givens; bf16x3 selects BF16x3 products for the compact-WY updates.
template <typename T>
hipError_t launch_bwy(bool bf16x3, int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                      const T* b, const double* d, const double* lam, T* Rb, T* cb, double* binv, T* R16,
                      int* status, hipStream_t st);

// Rows of padding before and after the sweep copy of the band (R16), and the band sizes the
// compile-time-width sweeps accept (their per-lane offsets into R16 are 32-bit).
constexpr int kBandPad = 128;
inline bool bsweep_w_fits(int64_t P, int64_t N, int w, size_t es) {
  return w >= 1 && w <= 15 && (P * N + 2 * kBandPad) * 16 * (int64_t)es < ((int64_t)1 << 32);
}

// The compile-time-width kernels (w <= 15, banded_w.hpp); binv: reciprocal pivots [P][N].
template <typename T>
hipError_t launch_bgivens_w(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                            const T* b, const double* d, const double* lam, T* Rb, T* cb, double* binv, T* R16,
                            int* status, hipStream_t st);
template <typename T>
hipError_t launch_bapply_w(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals, const T* b,
                           const double* v, double* r, hipStream_t st);
template <typename T>
hipError_t launch_bsweep_w(int kind, int P, int64_t N, int w, const T* R16, const double* binv, const T* rhsT,
                           const double* rhsD, double* out, int* status, hipStream_t st);

}  // namespace qrk
