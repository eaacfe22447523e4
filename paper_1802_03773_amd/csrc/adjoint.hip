// Adjoint of the LM step through the stored factor (not in the paper; the derivation
// differentiates the paper's Eq. 1, (J^T J + lam D^2) p = J^T b):
//   M dp = dJ^T r + J^T db - J^T dJ p - dlam D^2 p - 2 lam D dD p,   r = b - J p,
// so for a loss with g = dL/dp and u = M^{-1} g = (R^T R)^{-1} g (two triangular solves):
//   dL/db = J u,  dL/dJ_ab = r_a u_b - (J u)_a p_b,  dL/dlam = -u^T D^2 p,
//   dL/dd_j = -2 lam u_j d_j p_j.
// The triangular solves run through the structured R of Section 4.2 exactly as in the
// refinement; this file holds the pieces that differ: the forward pass over the blocks
// with a given g, the row pass that writes the gradients on the structural nonzeros, and
// the vector terms.
#include "qrk_batch.hpp"
#include "qrk_device.hpp"
#include "qrk_launch.hpp"

namespace qrk {

// y_i = R_i^{-T} g_i (one wave per block, redundantly in every lane) and per-workgroup
// partials of -sum_i S_i^T y_i (lanes over the dense columns; row stride kMaxDense).
template <typename T>
__global__ void __launch_bounds__(256)
k_adj_fwd_blocks(int64_t K, int n, int nB, const T* __restrict__ Rblk, const T* __restrict__ Sc,
                 const double* __restrict__ g, double* __restrict__ y, double* __restrict__ part) {
  __shared__ double red[4][128];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int L = nB + 1;
  double t0 = 0.0, t1 = 0.0;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t blk = (int64_t)blockIdx.x * 4 + wv; blk < K; blk += nwaves) {
    const T* Rb = Rblk + blk * n * n;
    double yy[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      yy[i] = 0.0;
      if (i < n) {
        double s = g[blk * n + i];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < i) s -= (double)Rb[j * n + i] * yy[j];
        yy[i] = s / (double)Rb[i * n + i];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k < n) {
        const T* row = Sc + (blk * n + k) * L;
        if (lane < nB) t0 -= (double)row[lane] * yy[k];
        if (lane + 64 < nB) t1 -= (double)row[lane + 64] * yy[k];
        if (lane == k) y[blk * n + k] = yy[k];
      }
    }
  }
  red[wv][lane] = t0;
  red[wv][lane + 64] = t1;
  __syncthreads();
  for (int j = threadIdx.x; j < nB; j += blockDim.x)
    part[(int64_t)blockIdx.x * kMaxDense + j] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
}

template <typename T>
hipError_t launch_adjoint_fwd_blocks(int64_t K, int n, int nB, const T* Rblk, const T* Sc, const double* g,
                                     double* y, double* part, int grid, hipStream_t st) {
  if (nB > 127 || n > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_adj_fwd_blocks<T>), dim3(grid), dim3(256), 0, st, K, n, nB, Rblk, Sc, g, y, part);
  return hipGetLastError();
}

// One wave per pack of whole blocks (at most 64 rows): lane r computes r_r = b_r - J_r p and
// (J u)_r, writes dA's row and db; then the pack's rows of dB are written coalesced.
template <typename T>
__global__ void __launch_bounds__(256)
k_adj_rows(int64_t npacks, const int64_t* __restrict__ pack_blk, int n, int nB,
           const int64_t* __restrict__ row_off, const T* __restrict__ A, const T* __restrict__ B,
           int64_t ldb, const T* __restrict__ bvec, const double* __restrict__ p,
           const double* __restrict__ u, int64_t Kn, T* __restrict__ dA, T* __restrict__ dB,
           T* __restrict__ db) {
  __shared__ double pB[128], uB[128];
  __shared__ double rr[4][64], ju[4][64];
  __shared__ int rowblk[4][64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < nB; j += blockDim.x) {
    pB[j] = p[Kn + j];
    uB[j] = u[Kn + j];
  }
  __syncthreads();
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t pk = (int64_t)blockIdx.x * 4 + wv; pk < npacks; pk += nwaves) {
    const int64_t b0 = pack_blk[pk];
    const int nb = (int)(pack_blk[pk + 1] - b0);
    const int64_t pr0 = row_off[b0];
    const int prows = (int)(row_off[b0 + nb] - pr0);
    if (lane < nb) {
      const int lo = (int)(row_off[b0 + lane] - pr0), hi = (int)(row_off[b0 + lane + 1] - pr0);
      for (int r = lo; r < hi; ++r) rowblk[wv][r] = lane;
    }
    wave_lds_sync();
    if (lane < prows) {
      const int64_t row = pr0 + lane;
      const int64_t blk = b0 + rowblk[wv][lane];
      double a[8], ap = 0.0, au = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        a[c] = (c < n) ? (double)A[row * n + c] : 0.0;
        if (c < n) {
          ap += a[c] * p[blk * n + c];
          au += a[c] * u[blk * n + c];
        }
      }
      const T* Brow = B + row * ldb;
      double bp = 0.0, bu = 0.0;
      for (int j = 0; j < nB; ++j) {
        const double bv = (double)Brow[j];
        bp += bv * pB[j];
        bu += bv * uB[j];
      }
      const double r = (double)bvec[row] - ap - bp;
      const double Ju = au + bu;
      rr[wv][lane] = r;
      ju[wv][lane] = Ju;
      if (dA) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (c < n) dA[row * n + c] = (T)(r * u[blk * n + c] - Ju * p[blk * n + c]);
      }
      if (db) db[row] = (T)Ju;
    }
    wave_lds_sync();
    if (dB) {
      for (int r = 0; r < prows; ++r) {
        const double rv = rr[wv][r], jv = ju[wv][r];
        T* out = dB + (pr0 + r) * ldb;
        if (lane < nB) out[lane] = (T)(rv * uB[lane] - jv * pB[lane]);
        if (lane + 64 < nB) out[lane + 64] = (T)(rv * uB[lane + 64] - jv * pB[lane + 64]);
      }
    }
    wave_lds_sync();
  }
}

template <typename T>
hipError_t launch_adjoint_rows(int64_t npacks, const int64_t* pack_blk, int64_t K, int n, int nB,
                               const int64_t* row_off, const T* A, const T* B, int64_t ldb, const T* b,
                               const double* p, const double* u, T* dA, T* dB, T* db, int grid,
                               hipStream_t st) {
  if (nB > 127 || n > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_adj_rows<T>), dim3(grid), dim3(256), 0, st, npacks, pack_blk, n, nB, row_off, A, B,
                     ldb, b, p, u, K * n, dA, dB, db);
  return hipGetLastError();
}

// dd and per-workgroup partials of -u^T D^2 p for every problem (problem = blockIdx.y).
__global__ void __launch_bounds__(256)
k_adj_vec(int64_t N, const double* __restrict__ u, const double* __restrict__ d,
          const double* __restrict__ p, double lam, double* __restrict__ dd, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t prob = blockIdx.y;
  double s = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (int64_t)gridDim.x * 256) {
    const int64_t e = prob * N + j;
    const double t = u[e] * d[e] * p[e];
    s -= t * d[e];
    if (dd) dd[e] = -2.0 * lam * t;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[prob * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_adj_vec_final(int nparts, const double* __restrict__ part, double* __restrict__ dlam) {
  const int prob = blockIdx.x;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += part[prob * nparts + i];
    dlam[prob] = s;
  }
}

hipError_t launch_adjoint_vec(int P, int64_t N, const double* u, const double* d, const double* p,
                              double lam, double* dd, double* dlam, double* part, hipStream_t st) {
  int grid = (int)((N + 255) / 256);
  const int cap = P > 0 ? 1024 / P : 1;
  if (grid > cap) grid = cap > 0 ? cap : 1;
  hipLaunchKernelGGL(k_adj_vec, dim3(grid, P), dim3(256), 0, st, N, u, d, p, lam, dd, part);
  if (dlam) hipLaunchKernelGGL(k_adj_vec_final, dim3(P), dim3(64), 0, st, grid, part, dlam);
  return hipGetLastError();
}

#define QRK_AINST(T)                                                                                     \
  template hipError_t launch_adjoint_fwd_blocks<T>(int64_t, int, int, const T*, const T*, const double*,   \
                                                   double*, double*, int, hipStream_t);                   \
  template hipError_t launch_adjoint_rows<T>(int64_t, const int64_t*, int64_t, int, int, const int64_t*,   \
                                             const T*, const T*, int64_t, const T*, const double*,         \
                                             const double*, T*, T*, T*, int, hipStream_t);
QRK_AINST(float)
QRK_AINST(double)
#undef QRK_AINST

}  // namespace qrk
