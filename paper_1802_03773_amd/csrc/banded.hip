// Banded J (the banded class of QRkit Section 4.4): row i of J holds w values at columns
// s_i .. s_i + w - 1 with s_i nondecreasing.  The QR of [J; sqrt(lam) D] is formed by
// Givens rotations (Section 2): R starts as the upper-triangular diag(sqrt(lam) d), and
// each row of J (with its b_i riding along as one more entry) is rotated into R in row
// order, one rotation per column of the row.  Because the starts are nondecreasing, the
// rows of R that a new row touches have no entries right of column s_i + w - 1, so R keeps
// upper bandwidth w - 1 and a w x w window of R (rows and columns s .. s + w - 1) is all
// that is live while row i is processed.
//
// Layout: one problem per group of G lanes (G = 16: one DPP row; G = 32 for w > 15).
// Lane l < w holds column s + l of the window (its entries in window rows 0..w-1), lane w
// holds the right-hand side c of those rows.  The pivot of rotation k is lane k; its two
// inputs are broadcast to the group, every lane applies the rotation to its own column.
// R is stored banded: row j holds R[j][j .. j + w - 1] (float or double), c is [N].
#include "qrk_device.hpp"
#include "qrk_banded.hpp"

namespace qrk {

// Broadcast lane K of each group; shift lanes of a group by one.
template <int G, int K, typename T>
__device__ __forceinline__ T gbcast(T x) {
  if constexpr (G == 16 && sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x150 + K, 0xF,
                                                          0xF, false));
  } else {
    return __shfl(x, K, G);
  }
}

template <int G, typename T>
__device__ __forceinline__ T gbcast_rt(T x, int k) {
  return __shfl(x, k, G);
}

template <int G, typename T>
__device__ __forceinline__ T gsum(T x) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) x += __shfl_xor(x, off, G);
  return x;
}

// lane l receives lane l + 1's value (within the group; the last lane keeps its own)
template <int G, typename T>
__device__ __forceinline__ T from_next(T x) {
  return __shfl_down(x, 1, G);
}

// lane l receives lane l - 1's value (the first lane keeps its own)
template <int G, typename T>
__device__ __forceinline__ T from_prev(T x) {
  return __shfl_up(x, 1, G);
}

template <typename T, int G>
__global__ void __launch_bounds__(256)
k_banded_givens(int P, int64_t M, int64_t N, int w, const int32_t* __restrict__ row_start,
                const T* __restrict__ vals, const T* __restrict__ bvec, const double* __restrict__ d,
                const double* __restrict__ lam, T* __restrict__ Rb, T* __restrict__ cb, int* __restrict__ status) {
  constexpr int W = G - 1;
  const int lane = threadIdx.x % G;
  const int64_t prob = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (prob >= P) return;
  const double sqrt_lam = sqrt(lam[prob]);
  const int32_t* rs = row_start + prob * M;
  const T* V = vals + prob * M * w;
  const T* bb = bvec + prob * M;
  const double* dd = d + prob * N;
  T* R = Rb + prob * N * w;
  T* cc = cb + prob * N;

  T Rw[W];
  const T diag0 = (lane < w) ? (T)(sqrt_lam * dd[lane < w ? lane : 0]) : T(0);
#pragma unroll
  for (int k = 0; k < W; ++k) Rw[k] = (k == lane) ? diag0 : T(0);
  int64_t s = 0;
  bool bad = false;

  auto shift = [&]() {
    // window row 0 (= row s of R) is final
    if (lane < w) R[s * w + lane] = Rw[0];
    if (lane == w) cc[s] = Rw[0];
#pragma unroll
    for (int k = 0; k + 1 < W; ++k) Rw[k] = Rw[k + 1];
    Rw[W - 1] = T(0);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const T nx = from_next<G>(Rw[k]);
      if (lane < w - 1) Rw[k] = nx;
      else if (lane == w - 1) Rw[k] = T(0);
    }
    // the new bottom row s + w enters with its damping diagonal
    if (lane == w - 1) {
#pragma unroll
      for (int k = 0; k < W; ++k)
        if (k == w - 1) Rw[k] = (T)(sqrt_lam * dd[s + w]);
    }
    ++s;
  };

  for (int64_t i = 0; i < M; ++i) {
    int64_t si = rs[i];
    if (si < s || si > N - w) {
      bad = true;
      si = si < s ? s : (N - w);
    }
    while (s < si) shift();
    T x = T(0);
    if (lane < w)
      x = V[i * w + lane];
    else if (lane == w)
      x = bb[i];
    static_for<0, W>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      if (k < w) {
        const T a = gbcast<G, k>(Rw[k]);
        const T xk = gbcast<G, k>(x);
        const T rr = sqrt(a * a + xk * xk);
        T cs = T(1), sn = T(0);
        if (rr != T(0)) {
          const T inv = T(1) / rr;
          cs = a * inv;
          sn = xk * inv;
        }
        const T Rk = Rw[k];
        Rw[k] = cs * Rk + sn * x;
        x = cs * x - sn * Rk;
        if (lane == k) {
          Rw[k] = rr;
          x = T(0);
        }
      }
    });
  }
  while (s < N - w) shift();
  // flush the last window: row s + k holds columns s + k .. s + w - 1 here, zeros beyond
#pragma unroll
  for (int k = 0; k < W; ++k) {
    if (k < w) {
      if (lane < w) {
        if (lane >= k) R[(s + k) * w + (lane - k)] = Rw[k];
        if (lane < k) R[(s + k) * w + (w - k + lane)] = T(0);
      }
      if (lane == w) cc[s + k] = Rw[k];
    }
  }
  if (bad) set_status(status, ST_BADINPUT);
}

// x = R^{-1} rhs for the banded R of every problem (backward sweep).
//   rhs: c (T, ADD = false, output set) or a float64 vector (ADD = true, output added).
template <typename T, int G, bool ADD>
__global__ void __launch_bounds__(256)
k_banded_bwd(int P, int64_t N, int w, const T* __restrict__ Rb, const T* __restrict__ cT,
             const double* __restrict__ rhs, double* __restrict__ out, int* __restrict__ status) {
  const int lane = threadIdx.x % G;
  const int64_t prob = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (prob >= P) return;
  const T* R = Rb + prob * N * w;
  double pw = 0.0;  // lane l holds x[j + l]
  double dmax = 0.0;
  bool bad = false, nonfinite = false;
  if (!ADD) {
    for (int64_t j = lane; j < N; j += G) dmax = fmax(dmax, fabs((double)R[j * w]));
    for (int off = G / 2; off >= 1; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, G));
  }
  for (int64_t j = N - 1; j >= 0; --j) {
    double part = (lane >= 1 && lane < w && j + lane < N) ? (double)R[j * w + lane] * pw : 0.0;
    part = gsum<G>(part);
    const double base = ADD ? rhs[prob * N + j] : (double)cT[prob * N + j];
    const double piv = (double)R[j * w];
    const double xj = (base - part) / piv;
    if (!ADD && is_finite(piv) && !(fabs(piv) > (double)N * Eps<T>::value * dmax)) bad = true;
    if (lane == 0) {
      if (ADD)
        out[prob * N + j] += xj;
      else
        out[prob * N + j] = xj;
      nonfinite |= !is_finite(xj);
    }
    if (lane == 0) pw = xj;
    pw = from_prev<G>(pw);
  }
  if (status) {
    if (bad) set_status(status, ST_SINGULAR);
    if (nonfinite) set_status(status, ST_NONFINITE);
  }
}

// y = R^{-T} g (forward sweep); g and y are float64 [P][N] (may alias).
template <typename T, int G>
__global__ void __launch_bounds__(256)
k_banded_fwd(int P, int64_t N, int w, const T* __restrict__ Rb, const double* g, double* y) {
  const int lane = threadIdx.x % G;
  const int64_t prob = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (prob >= P) return;
  const T* R = Rb + prob * N * w;
  double yw = 0.0;  // lane l holds y[j - l]
  for (int64_t j = 0; j < N; ++j) {
    double part = (lane >= 1 && lane < w && j - lane >= 0) ? (double)R[(j - lane) * w + lane] * yw : 0.0;
    part = gsum<G>(part);
    const double yj = (g[prob * N + j] - part) / (double)R[j * w];
    if (lane == 0) y[prob * N + j] = yj;
    if (lane == 0) yw = yj;
    yw = from_prev<G>(yw);
  }
}

// r = b - J v (float64), one row per lane: r [P][M].  With b == nullptr, r = J v.
template <typename T>
__global__ void __launch_bounds__(256)
k_banded_apply(int P, int64_t M, int64_t N, int w, const int32_t* __restrict__ row_start,
               const T* __restrict__ vals, const T* __restrict__ bvec, const double* __restrict__ v,
               double* __restrict__ r) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)P * M) return;
  const int64_t prob = t / M, i = t % M;
  int64_t si = row_start[prob * M + i];
  si = si < 0 ? 0 : (si > N - w ? N - w : si);
  const T* row = vals + (prob * M + i) * w;
  const double* vp = v + prob * N + si;
  double acc = 0.0;
  for (int l = 0; l < w; ++l) acc += (double)row[l] * vp[l];
  r[t] = bvec ? (double)bvec[t] - acc : acc;
}

// g = J^T r - lam d^2 v (float64) by a sweep over the rows of each problem (deterministic).
template <typename T, int G>
__global__ void __launch_bounds__(256)
k_banded_jt(int P, int64_t M, int64_t N, int w, const int32_t* __restrict__ row_start,
            const T* __restrict__ vals, const double* __restrict__ r, const double* __restrict__ d,
            const double* __restrict__ lamv, const double* __restrict__ v, double* __restrict__ g) {
  const int lane = threadIdx.x % G;
  const int64_t prob = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (prob >= P) return;
  const double lam = lamv[prob];
  const int32_t* rs = row_start + prob * M;
  double acc = 0.0;  // lane l accumulates column s + l
  int64_t s = 0;
  auto flush = [&]() {
    if (lane == 0) {
      const double dj = d[prob * N + s];
      g[prob * N + s] = acc - lam * dj * dj * v[prob * N + s];
    }
    acc = from_next<G>(acc);
    if (lane == G - 1) acc = 0.0;
    ++s;
  };
  for (int64_t i = 0; i < M; ++i) {
    int64_t si = rs[i];
    si = si < s ? s : (si > N - w ? N - w : si);
    while (s < si) flush();
    if (lane < w) acc += (double)vals[(prob * M + i) * w + lane] * r[prob * M + i];
  }
  while (s < N) flush();
}

// Adjoint entries on the structural nonzeros: dvals[i][l] = r_i u_{s_i+l} - (J u)_i p_{s_i+l}.
template <typename T>
__global__ void __launch_bounds__(256)
k_banded_dvals(int P, int64_t M, int64_t N, int w, const int32_t* __restrict__ row_start,
               const double* __restrict__ r, const double* __restrict__ Ju, const double* __restrict__ u,
               const double* __restrict__ p, T* __restrict__ dvals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)P * M * w) return;
  const int64_t row = t / w;
  const int l = (int)(t % w);
  const int64_t prob = row / M;
  int64_t si = row_start[row];
  si = si < 0 ? 0 : (si > N - w ? N - w : si);
  const int64_t col = prob * N + si + l;
  dvals[t] = (T)(r[row] * u[col] - Ju[row] * p[col]);
}

// ---------------------------------------------------------------------------------
#define QRK_G_DISPATCH(KERNEL, T, ...)                                                           \
  do {                                                                                           \
    if (w < 16) {                                                                                \
      const int64_t threads = (int64_t)P * 16;                                                   \
      hipLaunchKernelGGL((KERNEL<T, 16>), dim3((threads + 255) / 256), dim3(256), 0, st, __VA_ARGS__); \
    } else {                                                                                     \
      const int64_t threads = (int64_t)P * 32;                                                   \
      hipLaunchKernelGGL((KERNEL<T, 32>), dim3((threads + 255) / 256), dim3(256), 0, st, __VA_ARGS__); \
    }                                                                                            \
  } while (0)

template <typename T>
hipError_t launch_banded_givens(int P, int64_t M, int64_t N, int w, const int32_t* row_start,
                                const T* vals, const T* b, const double* d, const double* lam, T* Rb,
                                T* cb, int* status, hipStream_t st) {
  if (w < 1 || w > 31) return hipErrorInvalidValue;
  QRK_G_DISPATCH(k_banded_givens, T, P, M, N, w, row_start, vals, b, d, lam, Rb, cb, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_backsub(int P, int64_t N, int w, const T* Rb, const T* cb, double* p, int* status,
                                 hipStream_t st) {
  if (w < 16) {
    const int64_t threads = (int64_t)P * 16;
    hipLaunchKernelGGL((k_banded_bwd<T, 16, false>), dim3((threads + 255) / 256), dim3(256), 0, st, P, N, w,
                       Rb, cb, (const double*)nullptr, p, status);
  } else {
    const int64_t threads = (int64_t)P * 32;
    hipLaunchKernelGGL((k_banded_bwd<T, 32, false>), dim3((threads + 255) / 256), dim3(256), 0, st, P, N, w,
                       Rb, cb, (const double*)nullptr, p, status);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_solve_add(int P, int64_t N, int w, const T* Rb, const double* rhs, double* out,
                                   hipStream_t st) {
  if (w < 16) {
    const int64_t threads = (int64_t)P * 16;
    hipLaunchKernelGGL((k_banded_bwd<T, 16, true>), dim3((threads + 255) / 256), dim3(256), 0, st, P, N, w,
                       Rb, (const T*)nullptr, rhs, out, (int*)nullptr);
  } else {
    const int64_t threads = (int64_t)P * 32;
    hipLaunchKernelGGL((k_banded_bwd<T, 32, true>), dim3((threads + 255) / 256), dim3(256), 0, st, P, N, w,
                       Rb, (const T*)nullptr, rhs, out, (int*)nullptr);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_fwd(int P, int64_t N, int w, const T* Rb, const double* g, double* y,
                             hipStream_t st) {
  QRK_G_DISPATCH(k_banded_fwd, T, P, N, w, Rb, g, y);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_apply(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                               const T* b, const double* v, double* r, hipStream_t st) {
  const int64_t threads = (int64_t)P * M;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL((k_banded_apply<T>), dim3((threads + 255) / 256), dim3(256), 0, st, P, M, N, w, row_start,
                     vals, b, v, r);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_jt(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                            const double* r, const double* d, const double* lam, const double* v, double* g,
                            hipStream_t st) {
  QRK_G_DISPATCH(k_banded_jt, T, P, M, N, w, row_start, vals, r, d, lam, v, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_dvals(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const double* r,
                               const double* Ju, const double* u, const double* p, T* dvals, hipStream_t st) {
  const int64_t threads = (int64_t)P * M * w;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL((k_banded_dvals<T>), dim3((threads + 255) / 256), dim3(256), 0, st, P, M, N, w, row_start,
                     r, Ju, u, p, dvals);
  return hipGetLastError();
}

#define QRK_BINST(T)                                                                                     \
  template hipError_t launch_banded_givens<T>(int, int64_t, int64_t, int, const int32_t*, const T*,        \
                                              const T*, const double*, const double*, T*, T*, int*, hipStream_t); \
  template hipError_t launch_banded_backsub<T>(int, int64_t, int, const T*, const T*, double*, int*,       \
                                               hipStream_t);                                              \
  template hipError_t launch_banded_solve_add<T>(int, int64_t, int, const T*, const double*, double*,      \
                                                 hipStream_t);                                            \
  template hipError_t launch_banded_fwd<T>(int, int64_t, int, const T*, const double*, double*,            \
                                           hipStream_t);                                                  \
  template hipError_t launch_banded_apply<T>(int, int64_t, int64_t, int, const int32_t*, const T*,         \
                                             const T*, const double*, double*, hipStream_t);              \
  template hipError_t launch_banded_jt<T>(int, int64_t, int64_t, int, const int32_t*, const T*,            \
                                          const double*, const double*, const double*, const double*, double*, \
                                          hipStream_t);                                                   \
  template hipError_t launch_banded_dvals<T>(int, int64_t, int64_t, int, const int32_t*, const double*,    \
                                             const double*, const double*, const double*, T*, hipStream_t);
QRK_BINST(float)
QRK_BINST(double)
#undef QRK_BINST

}  // namespace qrk
