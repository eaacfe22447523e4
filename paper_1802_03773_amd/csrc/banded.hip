// Banded J (the banded class of QRkit Section 4.4): row i of J holds w values at columns
// s_i .. s_i + w - 1 with s_i nondecreasing.  The QR of [J; sqrt(lam) D] is formed by
// Givens rotations (Section 2): R starts as the upper-triangular diag(sqrt(lam) d), and
// each row of J (with its b_i riding along as one more entry) is rotated into R in row
// order, one rotation per column of the row.  Because the starts are nondecreasing, the
// rows of R that a new row touches have no entries right of column s_i + w - 1, so R keeps
// upper bandwidth w - 1 and a w x w window of R (rows and columns s .. s + w - 1) is all
// that is live while row i is processed.
//
// This file holds the run-time-width kernels, used for 16 <= w <= 31 (bands up to 15 use
// the compile-time-width kernels of banded_w.hpp), and the kernels shared by every width
// (J v, J^T r, adjoint entries).
// Layout of the run-time-width kernels: one problem per group of G = 32 lanes.  Lane l < w
// holds column s + l of the window (its entries in window rows 0..w-1), lane w holds the
// right-hand side c of those rows.  The pivot of rotation k is lane k; its two inputs are
// broadcast to the group, every lane applies the rotation to its own column.
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

// Row starts clamped to [0, N - w] (the same clamp as the factorisation's for valid input).
__device__ __forceinline__ int64_t band_start(const int32_t* rs, int64_t i, int64_t N, int w) {
  const int64_t s = rs[i];
  return s < 0 ? 0 : (s > N - w ? N - w : s);
}

// First-row table of every problem: fr[c] (c = 0 .. N) = the first row whose start is >= c,
// for nondecreasing starts.  Thread i (0 .. M) fills the columns after row i-1's start up to
// row i's start (thread M: up to N).  Starts out of order leave entries unset; the readers
// clamp what they read.
__global__ void __launch_bounds__(256)
k_band_first_row(int P, int64_t M, int64_t N, int w, const int32_t* __restrict__ row_start,
                 int32_t* __restrict__ fr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)P * (M + 1)) return;
  const int64_t prob = t / (M + 1), i = t % (M + 1);
  const int32_t* rs = row_start + prob * M;
  int32_t* f = fr + prob * (N + 1);
  const int64_t c0 = i == 0 ? 0 : band_start(rs, i - 1, N, w) + 1;
  const int64_t c1 = i == M ? N : band_start(rs, i, N, w);
  for (int64_t c = c0; c <= c1; ++c) f[c] = (int32_t)i;
}

// g = J^T r - lam d^2 v (float64), one thread per column: column j of a problem collects the
// rows whose start lies in [j - w + 1, j] in row order, so the sum is deterministic.  The row
// ranges come from the first-row table.  A workgroup covers 256 consecutive columns of one
// problem: the starts, residuals and values of its rows (one contiguous range) are copied to
// LDS with coalesced loads, eight per thread in flight, and each column then reads only LDS.
// Ranges beyond the LDS capacity read their rows from memory.
template <typename T>
__global__ void __launch_bounds__(256)
k_banded_jt(int P, int64_t M, int64_t N, int w, const int32_t* __restrict__ row_start, const int32_t* __restrict__ fr,
            const T* __restrict__ vals, const double* __restrict__ r, const double* __restrict__ d,
            const double* __restrict__ lamv, const double* __restrict__ v, double* __restrict__ g) {
  constexpr int CAP = 1024;                          // rows
  constexpr int VCAP = 40960 / (int)sizeof(T);       // values
  __shared__ int32_t s_st[CAP];
  __shared__ double s_r[CAP];
  __shared__ T s_v[VCAP];
  const int64_t nb = (N + 255) / 256;
  const int64_t prob = blockIdx.x / nb;
  const int64_t c0 = (int64_t)(blockIdx.x % nb) * 256;
  const int64_t j = c0 + threadIdx.x;
  const int32_t* rs = row_start + prob * M;
  const int32_t* f = fr + prob * (N + 1);
  const double* rp = r + prob * M;
  const T* V = vals + prob * M * w;
  auto row_at = [&](int64_t c) -> int64_t {  // table entry, clamped to [0, M]
    c = c < 0 ? 0 : (c > N ? N : c);
    const int64_t i = f[c];
    return i < 0 ? 0 : (i > M ? M : i);
  };
  const int64_t lo = row_at(c0 - w + 1);
  int64_t hi = row_at(c0 + 256);
  hi = hi < lo ? lo : hi;
  const int64_t n = hi - lo;
  const bool staged = n <= CAP && n * w <= VCAP;
  if (staged) {
    const int64_t nv = n * w;
    const T* Vlo = V + lo * w;
    for (int64_t i0 = 0; i0 < nv; i0 += 256 * 8) {
      T buf[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = i0 + u * 256 + threadIdx.x;
        buf[u] = i < nv ? Vlo[i] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = i0 + u * 256 + threadIdx.x;
        if (i < nv) s_v[i] = buf[u];
      }
    }
    for (int64_t i0 = 0; i0 < n; i0 += 256 * 4) {
      int32_t sb[4];
      double rb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + u * 256 + threadIdx.x;
        sb[u] = i < n ? (int32_t)band_start(rs, lo + i, N, w) : 0;
        rb[u] = i < n ? rp[lo + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + u * 256 + threadIdx.x;
        if (i < n) {
          s_st[i] = sb[u];
          s_r[i] = rb[u];
        }
      }
    }
    __syncthreads();
  }
  if (j >= N) return;
  int64_t a = row_at(j - w + 1), e = row_at(j + 1);
  double acc = 0.0;
  if (staged) {
    a = a < lo ? lo : a;
    e = e > hi ? hi : e;
    // eight rows per batch: their LDS reads are independent, the sum keeps row order
    const int i1 = (int)(e - lo);
    for (int i0 = (int)(a - lo); i0 < i1; i0 += 8) {
      int kk[8];
      double rr[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u < i1 ? i0 + u : i1 - 1;
        kk[u] = (int)(j - s_st[i]);
        rr[u] = s_r[i];
      }
      T vv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u < i1 ? i0 + u : i1 - 1;
        const int k = kk[u] < 0 ? 0 : (kk[u] >= w ? w - 1 : kk[u]);
        vv[u] = s_v[i * w + k];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < i1 && kk[u] >= 0 && kk[u] < w) acc += (double)vv[u] * rr[u];
    }
  } else {
    for (int64_t i = a; i < e; ++i) {
      const int64_t k = j - band_start(rs, i, N, w);
      if (k < 0 || k >= w) continue;
      acc += (double)V[i * w + k] * rp[i];
    }
  }
  const int64_t t = prob * N + j;
  const double dj = d[t];
  g[t] = acc - lamv[prob] * dj * dj * v[t];
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

template <typename T>
hipError_t launch_banded_givens(int P, int64_t M, int64_t N, int w, const int32_t* row_start,
                                const T* vals, const T* b, const double* d, const double* lam, T* Rb,
                                T* cb, double* binv, T* R16, int* status, hipStream_t st) {
  if (w < 1 || w > 31) return hipErrorInvalidValue;
  if (w <= 15) return launch_bgivens_w<T>(P, M, N, w, row_start, vals, b, d, lam, Rb, cb, binv, R16, status, st);
  const int64_t threads = (int64_t)P * 32;
  hipLaunchKernelGGL((k_banded_givens<T, 32>), dim3((threads + 255) / 256), dim3(256), 0, st, P, M, N, w, row_start,
                     vals, b, d, lam, Rb, cb, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_backsub(int P, int64_t N, int w, const T* Rb, const T* R16, const double* binv, const T* cb,
                                 double* p, int* status, hipStream_t st) {
  if (R16) {
    return launch_bsweep_w<T>(0, P, N, w, R16, binv, cb, nullptr, p, status, st);
  } else {
    const int64_t threads = (int64_t)P * 32;
    hipLaunchKernelGGL((k_banded_bwd<T, 32, false>), dim3((threads + 255) / 256), dim3(256), 0, st, P, N, w,
                       Rb, cb, (const double*)nullptr, p, status);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_solve_add(int P, int64_t N, int w, const T* Rb, const T* R16, const double* binv,
                                   const double* rhs, double* out, hipStream_t st) {
  if (R16) {
    return launch_bsweep_w<T>(1, P, N, w, R16, binv, nullptr, rhs, out, nullptr, st);
  } else {
    const int64_t threads = (int64_t)P * 32;
    hipLaunchKernelGGL((k_banded_bwd<T, 32, true>), dim3((threads + 255) / 256), dim3(256), 0, st, P, N, w,
                       Rb, (const T*)nullptr, rhs, out, (int*)nullptr);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_fwd(int P, int64_t N, int w, const T* Rb, const T* R16, const double* binv, const double* g,
                             double* y, hipStream_t st) {
  if (R16) return launch_bsweep_w<T>(2, P, N, w, R16, binv, nullptr, g, y, nullptr, st);
  const int64_t threads = (int64_t)P * 32;
  hipLaunchKernelGGL((k_banded_fwd<T, 32>), dim3((threads + 255) / 256), dim3(256), 0, st, P, N, w, Rb, g, y);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_apply(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                               const T* b, const double* v, double* r, hipStream_t st) {
  const int64_t threads = (int64_t)P * M;
  if (threads == 0) return hipSuccess;
  if (w <= 15) return launch_bapply_w<T>(P, M, N, w, row_start, vals, b, v, r, st);
  hipLaunchKernelGGL((k_banded_apply<T>), dim3((threads + 255) / 256), dim3(256), 0, st, P, M, N, w, row_start,
                     vals, b, v, r);
  return hipGetLastError();
}

hipError_t launch_band_first_row(int P, int64_t M, int64_t N, int w, const int32_t* row_start, int32_t* fr,
                                 hipStream_t st) {
  const int64_t threads = (int64_t)P * (M + 1);
  hipLaunchKernelGGL(k_band_first_row, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, P, M, N, w,
                     row_start, fr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_banded_jt(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const int32_t* fr,
                            const T* vals, const double* r, const double* d, const double* lam, const double* v,
                            double* g, hipStream_t st) {
  const int64_t blocks = (int64_t)P * ((N + 255) / 256);
  hipLaunchKernelGGL((k_banded_jt<T>), dim3((unsigned)blocks), dim3(256), 0, st, P, M, N, w, row_start, fr, vals, r,
                     d, lam, v, g);
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
                                              const T*, const double*, const double*, T*, T*, double*, T*, int*, hipStream_t); \
  template hipError_t launch_banded_backsub<T>(int, int64_t, int, const T*, const T*, const double*, const T*, \
                                               double*, int*, hipStream_t);                               \
  template hipError_t launch_banded_solve_add<T>(int, int64_t, int, const T*, const T*, const double*,     \
                                                 const double*, double*, hipStream_t);                    \
  template hipError_t launch_banded_fwd<T>(int, int64_t, int, const T*, const T*, const double*,           \
                                           const double*, double*, hipStream_t);                          \
  template hipError_t launch_banded_apply<T>(int, int64_t, int64_t, int, const int32_t*, const T*,         \
                                             const T*, const double*, double*, hipStream_t);              \
  template hipError_t launch_banded_jt<T>(int, int64_t, int64_t, int, const int32_t*, const int32_t*, const T*, \
                                          const double*, const double*, const double*, const double*, double*, \
                                          hipStream_t);                                                   \
  template hipError_t launch_banded_dvals<T>(int, int64_t, int64_t, int, const int32_t*, const double*,    \
                                             const double*, const double*, const double*, T*, hipStream_t);
QRK_BINST(float)
QRK_BINST(double)
#undef QRK_BINST

}  // namespace qrk
