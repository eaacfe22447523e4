// Back-substitution through the structured R of a horizontal concatenation
// (QRkit Section 4.2: R = [[blkdiag(R_i), S], [0, R_B]]) and corrected
// semi-normal-equation refinement of the step (Bjorck 1987):
//     r = b - J p,  g = J^T r - lam D^2 p   (float64),
//     R^T y = g,  R delta = y,  p <- p + delta.
// The two triangular solves run through the structure:
//     R_i^T y_i = g_i;   R_B^T y_B = g_B - sum_i S_i^T y_i;
//     R_B delta_B = y_B; R_i delta_i = y_i - S_i delta_B.
// Sums over blocks are deterministic: per-wave partials in registers, per-workgroup
// partials combined in a fixed order, then one workgroup adds the workgroup partials
// in index order.
#include "qrk_device.hpp"
#include "qrk_launch.hpp"

namespace qrk {

// ---------------------------------------------------------------------------------
// Dense part: R_B p_B = c_B, one workgroup (column-sweep back-substitution).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(128)
k_backsub_dense(const T* __restrict__ RB, int L, double* __restrict__ p, int64_t off,
                int* __restrict__ status) {
  __shared__ double pbuf[2];
  __shared__ double dmax[2];
  const int t = threadIdx.x;
  const int nB = L - 1;
  double rhs = (t < nB) ? (double)RB[(int64_t)t * L + nB] : 0.0;
  double dg = (t < nB) ? fabs((double)RB[(int64_t)t * L + t]) : 0.0;
  // max |R_jj| over the workgroup (two waves)
  double wm = wave_allreduce_max(dg);
  if ((t & 63) == 0) dmax[t >> 6] = wm;
  __syncthreads();
  const double rmax = (blockDim.x > 64) ? fmax(dmax[0], dmax[1]) : dmax[0];
  const double tol = (double)nB * Eps<T>::value * rmax;
  bool bad = false;
  for (int i = nB - 1; i >= 0; --i) {
    if (t == i) {
      const double piv = (double)RB[(int64_t)i * L + i];
      if (is_finite(piv) && !(fabs(piv) > tol)) bad = true;
      pbuf[i & 1] = rhs / piv;
    }
    __syncthreads();
    const double pi = pbuf[i & 1];
    if (t < i) rhs -= (double)RB[(int64_t)t * L + i] * pi;
    if (t == i) rhs = pi;
  }
  bool nonfinite = false;
  if (t < nB) {
    p[off + t] = rhs;
    if (!is_finite(rhs)) nonfinite = true;
  }
  if (bad) set_status(status, ST_SINGULAR);
  if (nonfinite) set_status(status, ST_NONFINITE);
}

template <typename T>
hipError_t launch_backsub_dense(const T* RB, int L, double* p, int64_t off, int* status,
                                hipStream_t st) {
  if (L - 1 > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_backsub_dense<T>), dim3(1), dim3(128), 0, st, RB, L, p, off, status);
  return hipGetLastError();
}

// Small triangular solves of one block, evaluated redundantly by every lane.
// Rb is the block's n x n R (row-major).  rhs/out hold up to 8 entries.
template <typename T>
__device__ __forceinline__ void block_backsub(const T* __restrict__ Rb, int n, const double* rhs,
                                              double* out) {
#pragma unroll
  for (int i = 7; i >= 0; --i) {
    if (i < n) {
      double s = rhs[i];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j > i && j < n) s -= (double)Rb[i * n + j] * out[j];
      out[i] = s / (double)Rb[i * n + i];
    }
  }
}

template <typename T>
__device__ __forceinline__ void block_fwdsub_T(const T* __restrict__ Rb, int n, const double* g,
                                               double* out) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if (i < n) {
      double s = g[i];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < i) s -= (double)Rb[j * n + i] * out[j];
      out[i] = s / (double)Rb[i * n + i];
    }
  }
}

// ---------------------------------------------------------------------------------
// Blocks: p_i = R_i^{-1} (c_i - S_i p_B), one wave per block.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_backsub_blocks(int64_t K, int n, int nB, const T* __restrict__ Rblk, const T* __restrict__ Sc,
                 double* __restrict__ p, int* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int L = nB + 1;
  const int64_t base = K * n;
  const double pb0 = (lane < nB) ? p[base + lane] : 0.0;
  const double pb1 = (lane + 64 < nB) ? p[base + 64 + lane] : 0.0;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  bool bad = false, nonfinite = false;
  for (int64_t blk = (int64_t)blockIdx.x * 4 + wv; blk < K; blk += nwaves) {
    double rhs[8], out[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      rhs[k] = 0.0;
      out[k] = 0.0;
      if (k < n) {
        const T* row = Sc + (blk * n + k) * L;
        double s = 0.0;
        if (lane < nB) s += (double)row[lane] * pb0;
        if (lane + 64 < nB) s += (double)row[64 + lane] * pb1;
        s = wave_allreduce_sum(s);
        rhs[k] = (double)row[nB] - s;
      }
    }
    const T* Rb = Rblk + blk * n * n;
    double dmax = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < n) dmax = fmax(dmax, fabs((double)Rb[k * n + k]));
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < n) {
        const double piv = (double)Rb[k * n + k];
        if (is_finite(piv) && !(fabs(piv) > (double)n * Eps<T>::value * dmax)) bad = true;
      }
    block_backsub(Rb, n, rhs, out);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < n && lane == k) {
        p[blk * n + k] = out[k];
        if (!is_finite(out[k])) nonfinite = true;
      }
  }
  if (bad) set_status(status, ST_SINGULAR);
  if (nonfinite) set_status(status, ST_NONFINITE);
}

template <typename T>
hipError_t launch_backsub_blocks(int64_t K, int n, int nB, const T* Rblk, const T* Sc, double* p,
                                 int* status, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_backsub_blocks<T>), dim3(grid), dim3(256), 0, st, K, n, nB, Rblk, Sc, p,
                     status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Refinement pass 1 (one wave per block, float64 arithmetic).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_refine_residual(int64_t K, int n, int nB, const int64_t* __restrict__ row_off,
                  const T* __restrict__ A, const T* __restrict__ B, int64_t ldb,
                  const T* __restrict__ bvec, const double* __restrict__ d, double lam,
                  const T* __restrict__ Rblk, const T* __restrict__ Sc,
                  const double* __restrict__ p, double* __restrict__ y, double* __restrict__ part) {
  __shared__ double red[4][128];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int L = nB + 1;
  const int64_t base = K * n;
  const double pb0 = (lane < nB) ? p[base + lane] : 0.0;
  const double pb1 = (lane + 64 < nB) ? p[base + 64 + lane] : 0.0;
  double t0 = 0.0, t1 = 0.0;  // partial sums of B^T r - S^T y for columns lane, lane+64
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t blk = (int64_t)blockIdx.x * 4 + wv; blk < K; blk += nwaves) {
    const int64_t r0 = row_off[blk];
    const int m = (int)(row_off[blk + 1] - r0);
    double pi[8], g[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      pi[k] = (k < n) ? p[blk * n + k] : 0.0;
      g[k] = 0.0;
    }
    for (int r = 0; r < m; ++r) {
      const int64_t row = r0 + r;
      const double b0 = (lane < nB) ? (double)B[row * ldb + lane] : 0.0;
      const double b1 = (lane + 64 < nB) ? (double)B[row * ldb + 64 + lane] : 0.0;
      double s = wave_allreduce_sum(b0 * pb0 + b1 * pb1);
      double aval[8];
      double ap = 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        aval[k] = (k < n) ? (double)A[row * n + k] : 0.0;
        ap += aval[k] * pi[k];
      }
      const double res = (double)bvec[row] - ap - s;
#pragma unroll
      for (int k = 0; k < 8; ++k) g[k] += aval[k] * res;
      t0 += b0 * res;
      t1 += b1 * res;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < n) {
        const double dk = d[blk * n + k];
        g[k] -= lam * dk * dk * pi[k];
      }
    const T* Rb = Rblk + blk * n * n;
    double yy[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) yy[k] = 0.0;
    block_fwdsub_T(Rb, n, g, yy);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k < n) {
        const T* row = Sc + (blk * n + k) * L;
        if (lane < nB) t0 -= (double)row[lane] * yy[k];
        if (lane + 64 < nB) t1 -= (double)row[64 + lane] * yy[k];
        if (lane == k) y[blk * n + k] = yy[k];
      }
    }
  }
  // workgroup partial: waves combined in fixed order
  red[wv][lane] = t0;
  red[wv][64 + lane] = t1;
  __syncthreads();
  if (threadIdx.x < 128 && threadIdx.x < nB) {
    const int j = threadIdx.x;
    const double s = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
    part[(int64_t)blockIdx.x * nB + j] = s;
  }
}

template <typename T>
hipError_t launch_refine_residual(int64_t K, int n, int nB, const int64_t* row_off, const T* A,
                                  const T* B, int64_t ldb, const T* b, const double* d, double lam,
                                  const T* Rblk, const T* Sc, const double* p, double* y,
                                  double* part, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_refine_residual<T>), dim3(grid), dim3(256), 0, st, K, n, nB, row_off, A, B,
                     ldb, b, d, lam, Rblk, Sc, p, y, part);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Refinement pass 2 (one workgroup): dense-part correction.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(128)
k_refine_dense(int nparts, int nB, const double* __restrict__ part, const T* __restrict__ RB,
               const double* __restrict__ dvec, double lam, double* __restrict__ p, int64_t off,
               double* __restrict__ delta_B) {
  __shared__ double buf[2];
  const int t = threadIdx.x;
  const int L = nB + 1;
  double g = 0.0;
  if (t < nB) {
    for (int w = 0; w < nparts; ++w) g += part[(int64_t)w * nB + t];
    const double dj = dvec[off + t];
    g -= lam * dj * dj * p[off + t];
  }
  // R_B^T y = g (forward, column sweep): y_i = g_i / R_ii; g_t -= R_it y_i for t > i
  for (int i = 0; i < nB; ++i) {
    if (t == i) buf[i & 1] = g / (double)RB[(int64_t)i * L + i];
    __syncthreads();
    const double yi = buf[i & 1];
    if (t > i && t < nB) g -= (double)RB[(int64_t)i * L + t] * yi;
    if (t == i) g = yi;
  }
  __syncthreads();
  // R_B delta = y (backward, column sweep)
  for (int i = nB - 1; i >= 0; --i) {
    if (t == i) buf[i & 1] = g / (double)RB[(int64_t)i * L + i];
    __syncthreads();
    const double di = buf[i & 1];
    if (t < i) g -= (double)RB[(int64_t)t * L + i] * di;
    if (t == i) g = di;
  }
  if (t < nB) {
    delta_B[t] = g;
    p[off + t] += g;
  }
}

template <typename T>
hipError_t launch_refine_dense(int nparts, int nB, const double* part, const T* RB, const double* dvec,
                               double lam, double* p, int64_t off, double* delta_B, hipStream_t st) {
  if (nB > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_refine_dense<T>), dim3(1), dim3(128), 0, st, nparts, nB, part, RB, dvec, lam,
                     p, off, delta_B);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Refinement pass 3: delta_i = R_i^{-1}(y_i - S_i delta_B), p_i += delta_i.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_refine_blocks(int64_t K, int n, int nB, const T* __restrict__ Rblk, const T* __restrict__ Sc,
                const double* __restrict__ y, const double* __restrict__ delta_B,
                double* __restrict__ p) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int L = nB + 1;
  const double db0 = (lane < nB) ? delta_B[lane] : 0.0;
  const double db1 = (lane + 64 < nB) ? delta_B[64 + lane] : 0.0;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t blk = (int64_t)blockIdx.x * 4 + wv; blk < K; blk += nwaves) {
    double rhs[8], out[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      rhs[k] = 0.0;
      out[k] = 0.0;
      if (k < n) {
        const T* row = Sc + (blk * n + k) * L;
        double s = 0.0;
        if (lane < nB) s += (double)row[lane] * db0;
        if (lane + 64 < nB) s += (double)row[64 + lane] * db1;
        s = wave_allreduce_sum(s);
        rhs[k] = y[blk * n + k] - s;
      }
    }
    block_backsub(Rblk + blk * n * n, n, rhs, out);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < n && lane == k) p[blk * n + k] += out[k];
  }
}

template <typename T>
hipError_t launch_refine_blocks(int64_t K, int n, int nB, const T* Rblk, const T* Sc, const double* y,
                                const double* delta_B, double* p, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_refine_blocks<T>), dim3(grid), dim3(256), 0, st, K, n, nB, Rblk, Sc, y,
                     delta_B, p);
  return hipGetLastError();
}

#define QRK_INST(T)                                                                                \
  template hipError_t launch_backsub_dense<T>(const T*, int, double*, int64_t, int*, hipStream_t);  \
  template hipError_t launch_backsub_blocks<T>(int64_t, int, int, const T*, const T*, double*, int*, \
                                               int, hipStream_t);                                   \
  template hipError_t launch_refine_residual<T>(int64_t, int, int, const int64_t*, const T*,         \
                                                const T*, int64_t, const T*, const double*, double,  \
                                                const T*, const T*, const double*, double*, double*, \
                                                int, hipStream_t);                                  \
  template hipError_t launch_refine_dense<T>(int, int, const double*, const T*, const double*,       \
                                             double, double*, int64_t, double*, hipStream_t);       \
  template hipError_t launch_refine_blocks<T>(int64_t, int, int, const T*, const T*, const double*,  \
                                              const double*, double*, int, hipStream_t);
QRK_INST(float)
QRK_INST(double)
#undef QRK_INST

}  // namespace qrk
