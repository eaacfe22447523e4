// Small utility kernels of libqrkit.so.
#include "qrk_device.hpp"
#include "qrk_host.hpp"

namespace qrk {

// Clear or set a few ints with a kernel (not hipMemsetAsync, so the call can sit inside a
// captured HIP graph).
__global__ void k_fill_int(int* ptr, int value) {
  if (threadIdx.x < 4) ptr[threadIdx.x] = value;
}

hipError_t launch_fill_int(int* ptr, int value, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, ptr, value);
  return hipGetLastError();
}

}  // namespace qrk

namespace qrk {

__global__ void k_fill_double(double* __restrict__ p, int64_t n, double value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

hipError_t launch_fill_double(double* p, int64_t n, double value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_double, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

template <typename T>
__global__ void k_to_type(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

template <typename T>
hipError_t launch_to_type(const double* src, T* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_to_type<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}
template hipError_t launch_to_type<float>(const double*, float*, int64_t, hipStream_t);
template hipError_t launch_to_type<double>(const double*, double*, int64_t, hipStream_t);

// Column norms of a block-angular J (Section 5.2's D = diag(J^T J)^(1/2)), float64, with
// d_j = 1 for an all-zero column.  Block columns: one thread per (block, column).  Dense
// columns: per-workgroup partial sums over row chunks, then a fixed-order final sum.
template <typename T>
__global__ void k_colnorms_blocks(int64_t K, int n, const int64_t* __restrict__ row_off,
                                  const T* __restrict__ A, double* __restrict__ d) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * n) return;
  const int64_t blk = t / n;
  const int c = (int)(t % n);
  double s = 0.0;
  for (int64_t r = row_off[blk]; r < row_off[blk + 1]; ++r) {
    const double a = (double)A[r * n + c];
    s += a * a;
  }
  d[t] = s > 0.0 ? sqrt(s) : 1.0;
}

template <typename T>
__global__ void __launch_bounds__(128)
k_colnorms_dense(int64_t M, int nB, const T* __restrict__ B, int64_t ldb, const int32_t* __restrict__ cam,
                 int64_t rows_per, double* __restrict__ part) {
  const int j = threadIdx.x;
  if (j >= nB) return;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = r0 + rows_per < M ? r0 + rows_per : M;
  double s = 0.0;
  if (cam) {
    // camera columns: row r holds ldb values of camera cam[r] (none outside [0, nB / ldb))
    const uint32_t ncam = (uint32_t)(nB / ldb);
    for (int64_t r = r0; r < r1; ++r) {
      const int cr = cam[r];
      if ((uint32_t)cr >= ncam) continue;
      const uint32_t k = (uint32_t)(j - cr * (int)ldb);
      if (k < (uint32_t)ldb) {
        const double b = (double)B[r * ldb + k];
        s += b * b;
      }
    }
  } else {
    for (int64_t r = r0; r < r1; ++r) {
      const double b = (double)B[r * ldb + j];
      s += b * b;
    }
  }
  part[(int64_t)blockIdx.x * nB + j] = s;
}

__global__ void k_colnorms_final(int nparts, int nB, const double* __restrict__ part,
                                 double* __restrict__ dB) {
  const int j = threadIdx.x;
  if (j >= nB) return;
  double s = 0.0;
  for (int w = 0; w < nparts; ++w) s += part[(int64_t)w * nB + j];
  dB[j] = s > 0.0 ? sqrt(s) : 1.0;
}

template <typename T>
hipError_t launch_colnorms(int64_t K, int n, int nB, int64_t M, const int64_t* row_off, const T* A,
                           const T* B, int64_t ldb, const int32_t* cam, double* d, double* part, int nparts,
                           hipStream_t st) {
  const int64_t kn = K * n;
  if (kn > 0)
    hipLaunchKernelGGL((k_colnorms_blocks<T>), dim3((unsigned)((kn + 255) / 256)), dim3(256), 0, st, K, n,
                       row_off, A, d);
  if (nB > 0) {
    const int64_t rows_per = (M + nparts - 1) / nparts > 0 ? (M + nparts - 1) / nparts : 1;
    hipLaunchKernelGGL((k_colnorms_dense<T>), dim3(nparts), dim3(128), 0, st, M, nB, B, ldb, cam, rows_per,
                       part);
    hipLaunchKernelGGL(k_colnorms_final, dim3(1), dim3(128), 0, st, nparts, nB, part, d + kn);
  }
  return hipGetLastError();
}
template hipError_t launch_colnorms<float>(int64_t, int, int, int64_t, const int64_t*, const float*,
                                           const float*, int64_t, const int32_t*, double*, double*, int,
                                           hipStream_t);
template hipError_t launch_colnorms<double>(int64_t, int, int, int64_t, const int64_t*, const double*,
                                            const double*, int64_t, const int32_t*, double*, double*, int,
                                            hipStream_t);

}  // namespace qrk

namespace qrk {

// Per problem q (one workgroup each, unknowns [noff[q], noff[q+1])): out[2q] = sum (p - pold)^2,
// out[2q+1] = sum p^2, in a fixed order (strided per thread, then a tree in LDS).
__global__ void __launch_bounds__(256) k_rel_change(const int64_t* __restrict__ noff, const double* __restrict__ p,
                                                    const double* __restrict__ pold, double* __restrict__ out) {
  __shared__ double sd[256], sp[256];
  const int q = blockIdx.x;
  const int64_t lo = noff[q], hi = noff[q + 1];
  double a = 0.0, c = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double x = p[i], dx = x - pold[i];
    a += dx * dx;
    c += x * x;
  }
  sd[threadIdx.x] = a;
  sp[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sd[threadIdx.x] += sd[threadIdx.x + h];
      sp[threadIdx.x] += sp[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * q] = sd[0];
    out[2 * q + 1] = sp[0];
  }
}

hipError_t launch_rel_change(int P, const int64_t* noff, const double* p, const double* pold, double* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_rel_change, dim3((unsigned)P), dim3(256), 0, st, noff, p, pold, out);
  return hipGetLastError();
}

}  // namespace qrk
