// Self-check entry points: the device primitives of the BF16x3 trailing updates exposed one
// at a time, so that a parity test can compare them with a bit-level emulation.
//
// What they compute (the compact-WY trailing update of Section 2, with each fp32 operand split
// as hi = bf16(x), lo = bf16(x - hi) and a*b ~ hi*hi' + hi*lo' + lo*hi'):
//   qrk_check_bf16_split     hi and lo of every element, by bf_split (the dense-part kernels'
//                            own split);
//   qrk_check_bf16x3_product C = A B for a 16 x k tile A and a k x 16 tile B, on the bf16 matrix
//                            cores with the operand layout and the three-product order of the
//                            dense-part trailing updates (hi*hi into one accumulator, hi*lo and
//                            lo*hi into a second one, the two added at the end).
#include "qrk_host.hpp"
#include "tsqr_mfma.hpp"

namespace qrk {

__global__ void __launch_bounds__(256) k_check_bf16_split(const float* __restrict__ x, float* __restrict__ hi,
                                                          float* __restrict__ lo, int64_t n) {
  const int64_t base = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;
  if (base >= n) return;
  float t[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) t[e] = base + e < n ? x[base + e] : 0.f;
  const BfPair s = bf_split(t);
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (base + e < n) {
      hi[base + e] = (float)s.hi[e];
      lo[base + e] = (float)s.lo[e];
    }
}

// One wave.  Chunk k0 .. k0+31 of the contraction: lane l supplies A[l % 16][k0 + 8(l / 16) + e]
// and B[k0 + 8(l / 16) + e][l % 16], e = 0..7 (the K-slot assignment of the trailing updates);
// C[4(l >> 4) + v][l & 15] is component v of lane l's accumulator.
__global__ void __launch_bounds__(64) k_check_bf16x3_product(const float* __restrict__ A, const float* __restrict__ B,
                                                             float* __restrict__ C, int k) {
  const int lane = threadIdx.x;
  const int r = lane & 15;
  const int kq = 8 * (lane >> 4);
  f4 Y0 = {0.f, 0.f, 0.f, 0.f}, Y1 = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < k; k0 += 32) {
    float a[8], b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = A[(int64_t)r * k + k0 + kq + e];
      b[e] = B[(int64_t)(k0 + kq + e) * 16 + r];
    }
    const BfPair as = bf_split(a);
    const BfPair bs = bf_split(b);
    Y0 = mfma_bf(as.hi, bs.hi, Y0);
    Y1 = mfma_bf(as.hi, bs.lo, Y1);
    Y1 = mfma_bf(as.lo, bs.hi, Y1);
  }
  const f4 Y = Y0 + Y1;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(4 * (lane >> 4) + v) * 16 + r] = Y[v];
}

}  // namespace qrk

using namespace qrk;

extern "C" {

qrk_status qrk_check_bf16_split(const float* x, float* hi, float* lo, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!x || !hi || !lo))) return QRK_EINVAL;
  if (n == 0) return QRK_OK;
  const int64_t threads = (n + 7) / 8;
  hipLaunchKernelGGL(k_check_bf16_split, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, x, hi, lo, n);
  return hipGetLastError() == hipSuccess ? QRK_OK : QRK_EHIP;
}

qrk_status qrk_check_bf16x3_product(const float* A, const float* B, float* C, int32_t k, void* stream) {
  if (!A || !B || !C || k < 32 || k > 4096 || k % 32 != 0) return QRK_EINVAL;
  hipLaunchKernelGGL(k_check_bf16x3_product, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, C, (int)k);
  return hipGetLastError() == hipSuccess ? QRK_OK : QRK_EHIP;
}

}  // extern "C"
