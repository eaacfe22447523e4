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
                                T* cb, int* status, hipStream_t st);
// p = R^{-1} c (status: singular pivots, non-finite results)
template <typename T>
hipError_t launch_banded_backsub(int P, int64_t N, int w, const T* Rb, const T* cb, double* p, int* status,
                                 hipStream_t st);
// out += R^{-1} rhs
template <typename T>
hipError_t launch_banded_solve_add(int P, int64_t N, int w, const T* Rb, const double* rhs, double* out,
                                   hipStream_t st);
// y = R^{-T} g
template <typename T>
hipError_t launch_banded_fwd(int P, int64_t N, int w, const T* Rb, const double* g, double* y,
                             hipStream_t st);
// r = b - J v (or J v when b is null), float64, [P][M]
template <typename T>
hipError_t launch_banded_apply(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                               const T* b, const double* v, double* r, hipStream_t st);
// g = J^T r - lam d^2 v, float64, [P][N]
template <typename T>
hipError_t launch_banded_jt(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                            const double* r, const double* d, const double* lam, const double* v, double* g,
                            hipStream_t st);
// dvals[i][l] = r_i u_{s_i+l} - (J u)_i p_{s_i+l}
template <typename T>
hipError_t launch_banded_dvals(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const double* r,
                               const double* Ju, const double* u, const double* p, T* dvals, hipStream_t st);

}  // namespace qrk
