// Device-side helpers shared by the qrkit HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "qrk_batch.hpp"

namespace qrk {

// Status bits recorded in the handle's device status word.
enum : int {
  ST_SINGULAR = 1,
  ST_NONFINITE = 2,
  ST_BADINPUT = 4,
  ST_STALL = 8,  // a dense-part merge did not see its inputs within its wait bound
  ST_NOTCONVERGED = 16,  // qrk_solve_tol used all its sweeps above the requested tolerance
};

constexpr int kWave = 64;

// Compile-time loop: f(std::integral_constant<int, I>) for I in [I0, N).
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Make LDS writes of one lane visible to the other lanes of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_allreduce_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_allreduce_max(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

template <typename T>
__device__ __forceinline__ bool is_finite(T x) {
  return __builtin_isfinite(x);
}

template <typename T>
struct Eps;
template <>
struct Eps<float> {
  static constexpr double value = 5.9604644775390625e-08;  // 2^-24
};
template <>
struct Eps<double> {
  static constexpr double value = 1.1102230246251565e-16;  // 2^-53
};

// The first per-block QR launch's clearing and lambda store (BqrPrologue), by the NT threads
// of workgroup 0.
template <int NT>
__device__ __forceinline__ void bqr_prologue(const BqrPrologue& pro) {
  if (blockIdx.x != 0) return;
  for (int64_t i = threadIdx.x; i < pro.n0; i += NT) pro.z0[i] = 0;
  for (int64_t i = threadIdx.x; i < pro.n1; i += NT) pro.z1[i] = 0;
  if (threadIdx.x == 0 && pro.lam_out) *pro.lam_out = pro.lam_val;
}

__device__ __forceinline__ void set_status(int* status, int bits) {
  if (status) atomicOr(status, bits);
}

}  // namespace qrk
