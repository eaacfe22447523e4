// Tall-skinny QR of the reduced dense rows (QRkit Section 4.2, the factorisation
// Q'R' = qr(Q_1^perp^T A_2)), organised as a communication-avoiding reduction: every
// workgroup streams a contiguous range of rows into its own running triangle (a flat
// tree inside the workgroup), and the triangles are then merged by the same kernel
// level by level, each level one launch over every problem of a batch (the workgroup
// list says where each one reads and writes).  The damping rows sqrt(lam) D_B are already triangular, so they are
// simply the starting triangle of workgroup 0 (sqrt(lam) d_B, lam read on the device).
//
// Merge of a tile of KT rows into the running triangle R (Householder, Section 2):
// for column j, the reflector acting on [R_jj; tile column j] has the form [1; w] so
// only R's row j and the tile change.  Thread c owns column c of R (kept in LDS,
// private to the thread) and column c of the tile (in registers); thread j builds w,
// publishes it through LDS, and every thread c > j updates its own column.
#include "qrk_batch.hpp"
#include "qrk_device.hpp"
#include "qrk_launch.hpp"

namespace qrk {

template <typename T, int KT, int NT>
__global__ void __launch_bounds__(NT)
k_tsqr_stream(const TsqrWg* __restrict__ wgs, const ProbDesc* __restrict__ probs, int n, const T* __restrict__ Red,
              const double* __restrict__ d, const double* __restrict__ lamv, T* __restrict__ part0,
              T* __restrict__ part1, T* __restrict__ RB) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TsqrWg W = wgs[blockIdx.x];
  const T* X = (W.in_buf == 0 ? Red : (W.in_buf == 1 ? part0 : part1)) + W.x_off;
  T* Rout = (W.out_buf == 0 ? RB : (W.out_buf == 1 ? part0 : part1)) + W.out_off;
  const int64_t ldx = W.ldx;
  const int L = W.L;
  const double* dB = nullptr;
  const double* lam = nullptr;
  if (W.seed >= 0) {
    const ProbDesc& P = probs[W.seed];
    dB = d + P.noff + P.K * n;
    lam = lamv + W.seed;
  }
  const int ldc = L + 1;
  T* Rc = reinterpret_cast<T*>(smem_raw);                       // [L][ldc], column-major per thread
  const int rc_elems = ((L * ldc + 3) / 4) * 4;
  T* Wb = Rc + rc_elems;                                          // [2][KT]
  T* Tb = Wb + 2 * KT;                                            // [2]
  const int c = threadIdx.x;
  const bool own = c < L;
  T* Rmy = Rc + c * ldc;

  if (own) {
    for (int j = 0; j < L; ++j) Rmy[j] = T(0);
    if (dB != nullptr && c < L - 1) Rmy[c] = (T)(sqrt(*lam) * dB[c]);
  }
  __syncthreads();

  const int64_t r0 = W.r0;
  const int64_t r1 = W.r1;
  for (int64_t t = r0; t < r1; t += KT) {
    const int kt = (int)((r1 - t) < KT ? (r1 - t) : KT);
    T x[KT];
#pragma unroll
    for (int r = 0; r < KT; ++r) x[r] = (own && r < kt) ? X[(t + r) * ldx + c] : T(0);

    for (int j = 0; j < L; ++j) {
      const int buf = j & 1;
      if (c == j) {
        const T alpha = Rmy[j];
        T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
        for (int r = 0; r < KT; r += 4) {
          s0 += x[r] * x[r];
          if (r + 1 < KT) s1 += x[r + 1] * x[r + 1];
          if (r + 2 < KT) s2 += x[r + 2] * x[r + 2];
          if (r + 3 < KT) s3 += x[r + 3] * x[r + 3];
        }
        const T sigma = (s0 + s1) + (s2 + s3);
        T beta = alpha, tau = T(0), scale = T(0);
        if (sigma != T(0)) {
          const T nrm = sqrt(alpha * alpha + sigma);
          beta = alpha >= T(0) ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scale = T(1) / (alpha - beta);
        }
        Rmy[j] = beta;
#pragma unroll
        for (int r = 0; r < KT; ++r) Wb[buf * KT + r] = x[r] * scale;
        Tb[buf] = tau;
      }
      __syncthreads();
      if (own && c > j) {
        const T tau = Tb[buf];
        if (tau != T(0)) {
          T w[KT];
#pragma unroll
          for (int r = 0; r < KT; ++r) w[r] = Wb[buf * KT + r];
          T s0 = Rmy[j], s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
          for (int r = 0; r < KT; r += 4) {
            s0 += w[r] * x[r];
            if (r + 1 < KT) s1 += w[r + 1] * x[r + 1];
            if (r + 2 < KT) s2 += w[r + 2] * x[r + 2];
            if (r + 3 < KT) s3 += w[r + 3] * x[r + 3];
          }
          const T s = ((s0 + s1) + (s2 + s3)) * tau;
          Rmy[j] -= s;
#pragma unroll
          for (int r = 0; r < KT; ++r) x[r] -= w[r] * s;
        }
      }
    }
    __syncthreads();
  }

  if (own)
    for (int j = 0; j < L; ++j) Rout[(int64_t)j * L + c] = (j <= c) ? Rmy[j] : T(0);
}

template <typename T>
hipError_t launch_tsqr_stream(const TsqrWg* wg, int count, int Lmax, const ProbDesc* probs, int n, const T* Red,
                              const double* d, const double* lam, T* part0, T* part1, T* RB, hipStream_t st) {
  constexpr int KT = 32;
  if (count < 1) return hipSuccess;
  const int rc_elems = ((Lmax * (Lmax + 1) + 3) / 4) * 4;
  const size_t smem = sizeof(T) * (size_t)(rc_elems + 2 * KT + 4);
  if (Lmax <= 64) {
    hipLaunchKernelGGL((k_tsqr_stream<T, KT, 64>), dim3(count), dim3(64), smem, st, wg, probs, n, Red, d, lam, part0,
                       part1, RB);
  } else if (Lmax <= 128) {
    if (smem > 65536) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tsqr_stream<T, KT, 128>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_tsqr_stream<T, KT, 128>), dim3(count), dim3(128), smem, st, wg, probs, n, Red, d, lam,
                       part0, part1, RB);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_tsqr_stream<float>(const TsqrWg*, int, int, const ProbDesc*, int, const float*,
                                              const double*, const double*, float*, float*, float*, hipStream_t);
template hipError_t launch_tsqr_stream<double>(const TsqrWg*, int, int, const ProbDesc*, int, const double*,
                                               const double*, const double*, double*, double*, double*,
                                               hipStream_t);

}  // namespace qrk
