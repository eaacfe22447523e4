// Banded J with a compile-time band width W <= 15: Givens QR and the banded triangular sweeps
// organised for latency (the banded class of QRkit Section 4.4, rotations of Section 2).
//
// What is computed is that of the run-time-w kernels in banded.hip: R starts as
// diag(sqrt(lam) d), every row of J (its b_i riding along) is rotated into R in row order, one
// rotation per column of the row, and p = R^{-1} c, y = R^{-T} g are banded sweeps.
//
// One problem per 16-lane group (one DPP row), four problems per wave.  Every step of a
// problem is a dependency chain, so what matters is the chain's length, not bandwidth:
//   * the live w x w window of R is held in band-offset layout (register k = window row k =
//     R row s + k, lane l = offset l, i.e. column s + k + l; lane 15 = its c entry).  That is
//     the storage layout of the band, so advancing the window is a rename of registers and a
//     retiring row is stored as it stands;
//   * the incoming row x is held relative to the current pivot (lane l = column s + k + l at
//     rotation k) and moves down one lane per rotation (one DPP), so every rotation's pivot is
//     lane 0 and its operands are DPP broadcasts;
//   * a rotation is c = a / r, s = x_k / r with 1 / r from one reciprocal square root, written
//     as x' = (a x - x_k R_k) / r and R_k' = (a R_k + x_k x) / r so that everything but the
//     final product is independent of the square root;
//   * rows, row starts and damping values are loaded a chunk of rows ahead;
//   * the sweeps keep the pending sums of the next w - 1 unknowns in lanes (lane l = the
//     unknown l steps ahead), so a step is one FMA, one FMA for the next unknown and one DPP
//     broadcast; R's entries and reciprocal pivots are loaded a chunk of steps ahead.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "qrk_banded.hpp"
#include "qrk_device.hpp"

namespace qrk {

// DPP move within each row of 16 lanes: lanes disabled by BANK keep `old`; with BC, lanes
// whose source lies outside the row read 0.
template <int CTRL, int BANK = 0xF, bool BC = true>
__device__ __forceinline__ float bw_dpp(float old, float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, x), CTRL, 0xF, BANK, BC));
}
template <int CTRL, int BANK = 0xF, bool BC = true>
__device__ __forceinline__ double bw_dpp(double old, double x) {
  const uint64_t o = __builtin_bit_cast(uint64_t, old), v = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)v, CTRL, 0xF, BANK, BC);
  const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(v >> 32), CTRL, 0xF, BANK, BC);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// lane K of the row, to every lane of the row
template <int K, typename T>
__device__ __forceinline__ T bw_bcast(T x) {
  return bw_dpp<0x150 + K>(T(0), x);
}
// lane l takes lane l + 1 (lane 15 takes 0)
template <typename T>
__device__ __forceinline__ T bw_down(T x) {
  return bw_dpp<0x101>(T(0), x);
}

__device__ __forceinline__ float bw_rsqrt(float q) { return __builtin_amdgcn_rsqf(q); }
__device__ __forceinline__ double bw_rsqrt(double q) { return 1.0 / sqrt(q); }
template <typename T>
struct BwTiny;
template <>
struct BwTiny<float> {
  static constexpr float value = 0x1p-126f;
};
template <>
struct BwTiny<double> {
  static constexpr double value = 0x1p-1022;
};

// Givens QR of P banded problems (M rows, N columns, W values per row).  Output: band R
// [P][N][W] (row j holds R[j][j .. j+W-1]), c [P][N], and for the sweeps the reciprocal
// pivots 1 / R[j][j] in float64 [P][N] and the sweep copy of the band R16 [P][N][16] (slot l
// of row j = R[j][j+l] for 1 <= l < W, zero elsewhere).  Row starts outside [s, N - W] (s: the previous row's
// start) are clamped and flagged as ST_BADINPUT.
template <typename T, int W>
__global__ void __launch_bounds__(256)
k_bgivens_w(int P, int64_t M, int64_t N, const int32_t* __restrict__ row_start, const T* __restrict__ vals,
            const T* __restrict__ bvec, const double* __restrict__ d, const double* __restrict__ lam,
            T* __restrict__ Rb, T* __restrict__ cb, double* __restrict__ binv, T* __restrict__ R16,
            int* __restrict__ status) {
  static_assert(W >= 1 && W <= 15, "band width");
  constexpr int C = 8;    // rows per prefetch chunk (even: rows are taken in pairs)
  constexpr int RHS = 15; // lane of the right-hand side
  const int lane = threadIdx.x & 15;
  const int64_t prob = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  if (prob >= P) return;
  const T sl = (T)sqrt(lam[prob]);
  const int32_t* rs = row_start + prob * M;
  const T* V = vals + prob * M * W;
  const T* bb = bvec + prob * M;
  const double* dd = d + prob * N;
  T* R = Rb + prob * N * W;
  T* cc = cb + prob * N;
  double* iv = binv + prob * N;
  T* S16 = R16 ? R16 + prob * N * 16 : nullptr;  // the sweep copy, when the handle keeps one
  const int64_t smax = N - W;

  T Rw[W];
#pragma unroll
  for (int k = 0; k < W; ++k) Rw[k] = lane == 0 ? sl * (T)dd[k] : T(0);

  auto load_x = [&](int64_t i) -> T {
    if (i >= M) return T(0);
    if (lane < W) return V[i * W + lane];
    return lane == RHS ? bb[i] : T(0);
  };
  auto load_st = [&](int64_t i) -> int32_t { return i < M ? rs[i] : 0; };
  // damping values of the next columns to enter: lane l -> column s0 + W + l
  auto load_dq = [&](int64_t s0) -> T {
    const int64_t col = s0 + W + lane;
    return (lane < 15 && col < N) ? sl * (T)dd[col] : T(0);
  };

  T cx[C], nx[C];
  int32_t cst[C], nst[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    cst[c] = load_st(c);
    cx[c] = load_x(c);
  }
  T dq = load_dq(0);
  int64_t s = 0;
  bool bad = false;

  auto retire = [&]() {  // window row 0 (R row s) is final
    if (lane < W) R[s * W + lane] = Rw[0];
    if (lane == RHS) cc[s] = Rw[0];
    if (lane == 0) iv[s] = 1.0 / (double)Rw[0];
    if (S16) S16[s * 16 + lane] = (lane >= 1 && lane < W) ? Rw[0] : T(0);
  };

  for (int64_t base = 0; base < M; base += C) {
    // where this chunk leaves the window, and the prefetch of the next chunk
    int64_t s_end = s;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (base + c < M) {
        int64_t si = cst[c];
        si = si < s_end ? s_end : (si > smax ? smax : si);
        s_end = si;
      }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      nst[c] = load_st(base + C + c);
      nx[c] = load_x(base + C + c);
    }
    const T ndq = load_dq(s_end);
    int jsh = 0;  // shifts in this chunk (lane jsh of the chunk's dq is the next to enter)
    auto shift_to = [&](int64_t si) {
      while (s < si) {
        retire();
#pragma unroll
        for (int k = 0; k + 1 < W; ++k) Rw[k] = Rw[k + 1];
        T e;
        if (jsh < 15) {
          e = dq;
        } else {
          e = lane == 0 ? sl * (T)dd[s + W] : T(0);
        }
        Rw[W - 1] = lane == 0 ? e : T(0);
        dq = bw_down(dq);
        ++jsh;
        ++s;
      }
    };
    auto clamp_start = [&](int64_t si) -> int64_t {
      if (si < s || si > smax) {
        bad = true;
        si = si < s ? s : smax;
      }
      return si;
    };
    // rotation k of the row held in x (pivot value xk in every lane) against window row k
    auto rotate = [&](auto KK, T& x, T& xk) {
      constexpr int k = decltype(KK)::value;
      const T Rk = Rw[k];
      const T a = bw_bcast<0>(Rk);
      const T q = fma(xk, xk, a * a);
      const bool refl = q >= BwTiny<T>::value;
      const T inv = bw_rsqrt(q);
      const T rn = fma(xk, x, a * Rk);
      const T xn = fma(-xk, Rk, a * x);
      Rw[k] = refl ? inv * rn : Rk;
      const T xr = refl ? inv * xn : x;
      if constexpr (k + 1 < W) {
        xk = bw_bcast<1>(xr);
        if constexpr (W <= 12) {
          // lanes 0..11 move down one lane, lanes 12..15 (zeros and the rhs) stay
          x = bw_dpp<0x101, 0x7, false>(xr, xr);
        } else {
          const T dn = bw_down(xr);
          x = lane == RHS ? xr : (lane == RHS - 1 ? T(0) : dn);
        }
      }
    };
    // Rows are taken in pairs of chunk slots.  Two consecutive rows with the same start go
    // through the window together, the second one rotation behind the first (its rotation
    // k - 1 needs window row k - 1 after the first row's rotation k - 1): two independent
    // dependency chains in one instruction stream.
    static_for<0, C / 2>([&](auto PP) {
      constexpr int c = 2 * decltype(PP)::value;
      if (base + c >= M) return;
      shift_to(clamp_start(cst[c]));
      const bool hasB = base + c + 1 < M;
      const int64_t sb = hasB ? clamp_start(cst[c + 1]) : s;
      T xa = cx[c], ka = bw_bcast<0>(cx[c]);
      if (hasB && sb == s) {
        T xb = cx[c + 1], kb = bw_bcast<0>(cx[c + 1]);
        static_for<0, W + 1>([&](auto KK) {
          constexpr int k = decltype(KK)::value;
          if constexpr (k < W) rotate(std::integral_constant<int, k>{}, xa, ka);
          if constexpr (k >= 1) rotate(std::integral_constant<int, k - 1>{}, xb, kb);
        });
      } else {
        static_for<0, W>([&](auto KK) { rotate(KK, xa, ka); });
        if (hasB) {
          shift_to(sb);
          T xb = cx[c + 1], kb = bw_bcast<0>(cx[c + 1]);
          static_for<0, W>([&](auto KK) { rotate(KK, xb, kb); });
        }
      }
    });
#pragma unroll
    for (int c = 0; c < C; ++c) {
      cst[c] = nst[c];
      cx[c] = nx[c];
    }
    dq = ndq;
  }
  while (s < smax) {
    retire();
#pragma unroll
    for (int k = 0; k + 1 < W; ++k) Rw[k] = Rw[k + 1];
    Rw[W - 1] = lane == 0 ? sl * (T)dd[s + W] : T(0);
    ++s;
  }
  // the last window: rows s .. s + W - 1 (entries beyond column N - 1 are zero)
#pragma unroll
  for (int k = 0; k < W; ++k) {
    if (lane < W) R[(s + k) * W + lane] = Rw[k];
    if (lane == RHS) cc[s + k] = Rw[k];
    if (lane == 0) iv[s + k] = 1.0 / (double)Rw[k];
    if (S16) S16[(s + k) * 16 + lane] = (lane >= 1 && lane < W) ? Rw[k] : T(0);
  }
  if (bad) set_status(status, ST_BADINPUT);
}

// Exchange the odd 16-lane rows of v0 with the even rows of v1 (v_permlane16_swap).
__device__ __forceinline__ void bw_swap16(float& v0, float& v1) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, v0), __builtin_bit_cast(unsigned, v1),
                                                  false, false);
  v0 = __builtin_bit_cast(float, (unsigned)r[0]);
  v1 = __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ void bw_swap16(double& v0, double& v1) {
  const uint64_t a = __builtin_bit_cast(uint64_t, v0), b = __builtin_bit_cast(uint64_t, v1);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)a, (unsigned)b, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
  v0 = __builtin_bit_cast(double, ((uint64_t)(unsigned)hi[0] << 32) | (unsigned)lo[0]);
  v1 = __builtin_bit_cast(double, ((uint64_t)(unsigned)hi[1] << 32) | (unsigned)lo[1]);
}
// The odd row's value in both rows of each pair of 16-lane rows.
template <typename T>
__device__ __forceinline__ T bw_from_odd(T x) {
  T y = x;
  if constexpr (sizeof(T) == 4) {
    asm volatile("" : "+v"(y));
  } else {
    uint64_t u = __builtin_bit_cast(uint64_t, y);
    asm volatile("" : "+v"(u));
    y = __builtin_bit_cast(T, u);
  }
  bw_swap16(x, y);  // y: even rows take the odd rows' values
  return y;
}

// The same Givens QR with two problems per wave and two rows in flight per problem: a problem
// owns 32 lanes, rows taken in pairs of equal start go through the window together, the first
// (lanes 0-15, "A") two rotations ahead of the second (lanes 16-31, "B").  At step t, A
// rotates against window row t and B against window row t - 2 in the same instructions:
// register k holds window row k in A's lanes and window row k - 2 in B's lanes.  After each
// step v_permlane16_swap hands the row A just rotated to B (register t of A -> register t + 2
// of B) and the row B just rotated back to A (register t of B -> register t - 2 of A), so
// every row is current in A's lanes once a pair is done.  The two-step lag keeps the hand-over
// off the dependency chain of the rotations.  Rows whose starts differ go one at a time
// in A's lanes.  With every SIMD holding a wave, this takes about half the time of four
// problems per wave when the problems number fewer than four per SIMD.
template <typename T, int W>
__global__ void __launch_bounds__(256)
k_bgivens2_w(int P, int64_t M, int64_t N, const int32_t* __restrict__ row_start, const T* __restrict__ vals,
             const T* __restrict__ bvec, const double* __restrict__ d, const double* __restrict__ lam,
             T* __restrict__ Rb, T* __restrict__ cb, double* __restrict__ binv, T* __restrict__ R16,
             int* __restrict__ status) {
  static_assert(W >= 1 && W <= 15, "band width");
  constexpr int C = 8;    // rows per prefetch chunk (4 pairs)
  constexpr int NP = C / 2;
  constexpr int RHS = 15; // lane of the right-hand side (in each half)
  const int lane32 = threadIdx.x & 31;
  const int half = lane32 >> 4;
  const int lane = lane32 & 15;
  const int64_t prob = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5;
  if (prob >= P) return;
  const T sl = (T)sqrt(lam[prob]);
  const int32_t* rs = row_start + prob * M;
  const T* V = vals + prob * M * W;
  const T* bb = bvec + prob * M;
  const double* dd = d + prob * N;
  T* R = Rb + prob * N * W;
  T* cc = cb + prob * N;
  double* iv = binv + prob * N;
  T* S16 = R16 ? R16 + prob * N * 16 : nullptr;
  const int64_t smax = N - W;
  const bool isA = half == 0;

  T Rw[W + 2];  // A: register k = window row k (k < W);  B: register k = window row k - 2
#pragma unroll
  for (int k = 0; k < W + 2; ++k) Rw[k] = (isA && k < W && lane == 0) ? sl * (T)dd[k] : T(0);

  auto load_x = [&](int64_t i) -> T {  // row i in this lane's half
    if (i >= M) return T(0);
    if (lane < W) return V[i * W + lane];
    return lane == RHS ? bb[i] : T(0);
  };
  auto load_st = [&](int64_t i) -> int32_t { return i < M ? rs[i] : 0; };
  auto load_dq = [&](int64_t s0) -> T {
    const int64_t col = s0 + W + lane;
    return (lane < 15 && col < N) ? sl * (T)dd[col] : T(0);
  };

  T cx[NP], nx[NP];
  int32_t cst[C], nst[C];
#pragma unroll
  for (int p = 0; p < NP; ++p) cx[p] = load_x(2 * p + half);
#pragma unroll
  for (int c = 0; c < C; ++c) cst[c] = load_st(c);
  T dq = load_dq(0);
  int64_t s = 0;
  bool bad = false;

  auto retire = [&]() {  // window row 0 (R row s) is final; A's lanes hold it
    if (isA) {
      if (lane < W) R[s * W + lane] = Rw[0];
      if (lane == RHS) cc[s] = Rw[0];
      if (lane == 0) iv[s] = 1.0 / (double)Rw[0];
      if (S16) S16[s * 16 + lane] = (lane >= 1 && lane < W) ? Rw[0] : T(0);
    }
  };
  auto clamp_start = [&](int64_t si) -> int64_t {
    if (si < s || si > smax) {
      bad = true;
      si = si < s ? s : smax;
    }
    return si;
  };
  // rotation of the row held in x against register K (see the layout above)
  auto rotate = [&](auto KK, T& x, T& xk) {
    constexpr int k = decltype(KK)::value;
    const T Rk = Rw[k];
    const T a = bw_bcast<0>(Rk);
    const T q = fma(xk, xk, a * a);
    const bool refl = q >= BwTiny<T>::value;
    const T inv = bw_rsqrt(q);
    const T rn = fma(xk, x, a * Rk);
    const T xn = fma(-xk, Rk, a * x);
    Rw[k] = refl ? inv * rn : Rk;
    const T xr = refl ? inv * xn : x;
    xk = bw_bcast<1>(xr);
    if constexpr (W <= 12) {
      x = bw_dpp<0x101, 0x7, false>(xr, xr);
    } else {
      const T dn = bw_down(xr);
      x = lane == RHS ? xr : (lane == RHS - 1 ? T(0) : dn);
    }
  };

  for (int64_t base = 0; base < M; base += C) {
    int64_t s_end = s;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (base + c < M) {
        int64_t si = cst[c];
        si = si < s_end ? s_end : (si > smax ? smax : si);
        s_end = si;
      }
#pragma unroll
    for (int p = 0; p < NP; ++p) nx[p] = load_x(base + C + 2 * p + half);
#pragma unroll
    for (int c = 0; c < C; ++c) nst[c] = load_st(base + C + c);
    const T ndq = load_dq(s_end);
    int jsh = 0;
    auto shift_to = [&](int64_t si) {
      while (s < si) {
        retire();
#pragma unroll
        for (int k = 0; k + 1 < W; ++k) Rw[k] = Rw[k + 1];
        T e;
        if (jsh < 15) {
          e = dq;
        } else {
          e = (isA && lane == 0) ? sl * (T)dd[s + W] : T(0);
        }
        Rw[W - 1] = (isA && lane == 0) ? e : T(0);
        dq = bw_down(dq);
        ++jsh;
        ++s;
      }
    };
    static_for<0, NP>([&](auto PP) {
      constexpr int p = decltype(PP)::value;
      constexpr int c = 2 * p;
      if (base + c >= M) return;
      shift_to(clamp_start(cst[c]));
      const bool hasB = base + c + 1 < M;
      const int64_t sb = hasB ? clamp_start(cst[c + 1]) : s;
      T x = cx[p];
      T xk = bw_bcast<0>(x);
      if (hasB && sb == s) {
        static_for<0, W + 2>([&](auto TT) {
          constexpr int t = decltype(TT)::value;
          constexpr bool runA = t < W, runB = t >= 2;
          if constexpr (runA && runB) {
            rotate(std::integral_constant<int, t>{}, x, xk);
          } else if constexpr (runA) {
            if (isA) rotate(std::integral_constant<int, t>{}, x, xk);
          } else if constexpr (runB) {
            if (!isA) rotate(std::integral_constant<int, t>{}, x, xk);
          }
          if constexpr (t >= 2) bw_swap16(Rw[t], Rw[t - 2]);  // B's row t-2 back to A
          if constexpr (t < W) bw_swap16(Rw[t + 2], Rw[t]);   // A's row t on to B
        });
      } else {
        if (isA) static_for<0, W>([&](auto KK) { rotate(KK, x, xk); });
        if (hasB) {
          shift_to(sb);
          T y = bw_from_odd(cx[p]);  // B's row, into A's lanes
          T yk = bw_bcast<0>(y);
          if (isA) static_for<0, W>([&](auto KK) { rotate(KK, y, yk); });
        }
      }
    });
#pragma unroll
    for (int p = 0; p < NP; ++p) cx[p] = nx[p];
#pragma unroll
    for (int c = 0; c < C; ++c) cst[c] = nst[c];
    dq = ndq;
  }
  while (s < smax) {
    retire();
#pragma unroll
    for (int k = 0; k + 1 < W; ++k) Rw[k] = Rw[k + 1];
    Rw[W - 1] = (isA && lane == 0) ? sl * (T)dd[s + W] : T(0);
    ++s;
  }
  if (isA) {
#pragma unroll
    for (int k = 0; k < W; ++k) {
      if (lane < W) R[(s + k) * W + lane] = Rw[k];
      if (lane == RHS) cc[s + k] = Rw[k];
      if (lane == 0) iv[s + k] = 1.0 / (double)Rw[k];
      if (S16) S16[(s + k) * 16 + lane] = (lane >= 1 && lane < W) ? Rw[k] : T(0);
    }
  }
  if (bad && isA && lane == 0) set_status(status, ST_BADINPUT);
}

// Banded triangular sweep over every problem, one unknown per step.
//   BWD:  x = R^{-1} rhs, steps t = 0 .. N-1 on rows j = N-1-t;
//         x_j = (rhs_j - sum_{l=1}^{W-1} R[j][j+l] x_{j+l}) / R[j][j]
//   !BWD: y = R^{-T} rhs, steps on rows j = t;  y_j = (rhs_j - sum_l R[j-l][j] y_{j-l}) / R[j][j]
// rhs: c (T, RHS_T) or a float64 vector; out: set, or added to when ADD.  With CHECK, pivots
// that are tiny against the largest one flag ST_SINGULAR and non-finite results ST_NONFINITE.
// Lane ownership rotates with the step: lane c (mod 16) accumulates the pending sum of the
// unknowns of steps t = c (mod 16).  At step t (t mod 16 = c, a compile-time lane in a chunk of
// 16 steps) lane c's sum is complete; lane c forms the unknown from its own reciprocal pivot
// and right-hand side, the unknown is broadcast from lane c, lane c's sum restarts at zero
// and every other lane adds the unknown times its coupling entry (the lane l steps ahead,
// l = 1 .. W-1, holds R's entry at band offset l).  No value moves between lanes except the
// one broadcast per step.  Data for a chunk (per lane: 16 coupling entries, its reciprocal
// pivot, scaled right-hand side and output) are loaded three chunks ahead.
template <typename T, int W, bool BWD, bool ADD, bool RHS_T, bool CHECK>
__global__ void __launch_bounds__(256)
k_bsweep_w(int P, int64_t N, const T* __restrict__ R16, const double* __restrict__ binv, const T* __restrict__ rhsT,
           const double* __restrict__ rhsD, double* __restrict__ out, int* __restrict__ status) {
  static_assert(W >= 1 && W <= 15, "band width");
  constexpr int C = 16;  // steps per chunk (one per lane)
  constexpr int D = 3;   // chunks in flight
  const int lane = threadIdx.x & 15;
  const int64_t prob = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  if (prob >= P) return;
  if (N <= 0) return;
  const double* iv = binv + prob * N;
  const T* rt = RHS_T ? rhsT + prob * N : nullptr;
  const double* rd = RHS_T ? nullptr : rhsD + prob * N;
  double* o = out + prob * N;

  auto row_of = [&](int64_t t) -> int64_t { return BWD ? N - 1 - t : t; };
  // Couplings come from the sweep copy of the band (rows of 16 slots, slot l = band offset l
  // for 1 <= l < W, zero elsewhere, kBandPad rows of padding before the first and after the
  // last problem).  Lane `lane` at step t0 + c reads slot l = (lane - c) mod 16 of row j - l
  // (backward) or j (forward): a zero for the lanes that are not coupled to the step.  Rows
  // past either end of the problem fall in a neighbour or the padding and only feed unknowns
  // past the end, which are never stored.  The address is a wave-uniform base (the step part)
  // plus a per-lane 32-bit offset fixed for the whole sweep.
  const char* g16 = reinterpret_cast<const char*>(R16 - (int64_t)kBandPad * 16);
  uint32_t voff[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int l = (lane - c) & 15;
    const int64_t row = kBandPad + prob * N + (BWD ? (N - 1 - c - l) : c);
    voff[c] = (uint32_t)((row * 16 + l) * (int64_t)sizeof(T));
  }
  struct Chunk {
    T cr[C];  // cr[c]: coupling of step t0 + c's unknown into this lane's pending unknown
    double ivv, bvv, outv;
  };
  auto load_chunk = [&](int64_t t0, Chunk& k) {
    const char* sb = g16 + (BWD ? -t0 : t0) * 16 * (int64_t)sizeof(T);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      uint32_t vo = voff[c];
      asm("" : "+v"(vo));
      k.cr[c] = *reinterpret_cast<const T*>(sb + (uint64_t)vo);
    }
    // the step whose unknown this lane forms (clamped past the end: the value is not used)
    const int64_t tl = t0 + lane < N ? t0 + lane : N - 1;
    const int64_t j = row_of(tl);
    const double ivn = iv[j];
    const double bn = RHS_T ? (double)rt[j] : rd[j];
    k.ivv = ivn;
    k.bvv = bn * ivn;
    k.outv = ADD ? o[j] : 0.0;
  };

  Chunk ring[D];
#pragma unroll
  for (int b = 0; b < D; ++b) load_chunk((int64_t)b * C, ring[b]);
  double acc = 0.0;
  double amin = __builtin_inf(), amax = 0.0;  // extreme |1 / pivot| seen by this lane
  bool nonfinite = false;

  for (int64_t T0 = 0; T0 < N; T0 += (int64_t)C * D) {
    static_for<0, D>([&](auto BB) {
      constexpr int b = decltype(BB)::value;
      const int64_t t0 = T0 + (int64_t)b * C;
      if (t0 >= N) return;
      Chunk& k = ring[b];
      double xs = 0.0;  // lane c: the unknown of step t0 + c
      static_for<0, C>([&](auto CC) {
        constexpr int c = decltype(CC)::value;
        const double x = fma(-acc, k.ivv, k.bvv);  // meaningful in lane c
        if (lane == c) xs = x;
        const double xb = bw_bcast<c>(x);
        acc = lane == c ? 0.0 : acc;
        acc = fma((double)k.cr[c], xb, acc);
      });
      const int64_t t = t0 + lane;
      if (t < N) {
        if (CHECK) {
          const double a = fabs(k.ivv);
          if (!is_finite(xs)) nonfinite = true;
          if (a == a) {
            amin = fmin(amin, a);
            amax = fmax(amax, a);
          }
        }
        o[row_of(t)] = ADD ? k.outv + xs : xs;
      }
      load_chunk(t0 + (int64_t)C * D, k);  // refill this slot with the chunk D ahead
    });
  }
  if (CHECK && status) {
    // |pivot| = 1 / |1 / pivot|: flag a pivot at most N eps times the largest one
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
      amin = fmin(amin, __shfl_xor(amin, off, 16));
      amax = fmax(amax, __shfl_xor(amax, off, 16));
    }
    const double pmax = 1.0 / amin, pmin = 1.0 / amax;
    const bool bad = amax > 0.0 && is_finite(pmin) && pmin <= (double)N * Eps<T>::value * pmax;
    if (lane == 0 && bad) set_status(status, ST_SINGULAR);
    if (nonfinite) set_status(status, ST_NONFINITE);
  }
}

}  // namespace qrk

namespace qrk {

// r = b - J v (float64), one row per thread, the W products unrolled (all loads issued up
// front); with b == nullptr, r = J v.  Same arithmetic order as the run-time-width kernel.
template <typename T, int W>
__global__ void __launch_bounds__(256)
k_bapply_w(int P, int64_t M, int64_t N, const int32_t* __restrict__ row_start, const T* __restrict__ vals,
           const T* __restrict__ bvec, const double* __restrict__ v, double* __restrict__ r) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)P * M) return;
  const int64_t prob = t / M;
  int64_t si = row_start[t];
  si = si < 0 ? 0 : (si > N - W ? N - W : si);
  const T* row = vals + t * W;
  const double* vp = v + prob * N + si;
  T a[W];
  double x[W];
#pragma unroll
  for (int l = 0; l < W; ++l) {
    a[l] = row[l];
    x[l] = vp[l];
  }
  double acc = 0.0;
#pragma unroll
  for (int l = 0; l < W; ++l) acc += (double)a[l] * x[l];
  r[t] = bvec ? (double)bvec[t] - acc : acc;
}

}  // namespace qrk

namespace qrk {

// Host-side compile-time loop over I = A .. B-1.
template <int A, int B, typename F>
inline void bw_host_for(F&& f) {
  if constexpr (A < B) {
    f(std::integral_constant<int, A>{});
    bw_host_for<A + 1, B>(f);
  }
}

// Launchers for W = 1 .. 15 (one problem per 16 lanes, 16 problems per workgroup).
template <typename T>
hipError_t launch_bgivens_w(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                            const T* b, const double* d, const double* lam, T* Rb, T* cb, double* binv, T* R16,
                            int* status, hipStream_t st) {
  const dim3 grid((unsigned)(((int64_t)P * 16 + 255) / 256)), blk(256);
  hipError_t e = hipErrorInvalidValue;
  bw_host_for<1, 16>([&](auto WW) {
    constexpr int W = decltype(WW)::value;
    if (w != W) return;
    if (P < 4096) {
      // fewer than four problems per SIMD: two per wave, two rows in flight
      const dim3 grid2((unsigned)(((int64_t)P * 32 + 255) / 256));
      hipLaunchKernelGGL((k_bgivens2_w<T, W>), grid2, blk, 0, st, P, M, N, row_start, vals, b, d, lam, Rb, cb, binv,
                         R16, status);
    } else {
      hipLaunchKernelGGL((k_bgivens_w<T, W>), grid, blk, 0, st, P, M, N, row_start, vals, b, d, lam, Rb, cb, binv,
                         R16, status);
    }
    e = hipGetLastError();
  });
  return e;
}

template <typename T>
hipError_t launch_bapply_w(int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals, const T* b,
                           const double* v, double* r, hipStream_t st) {
  const int64_t threads = (int64_t)P * M;
  const dim3 grid((unsigned)((threads + 255) / 256)), blk(256);
  hipError_t e = hipErrorInvalidValue;
  bw_host_for<1, 16>([&](auto WW) {
    constexpr int W = decltype(WW)::value;
    if (w != W) return;
    hipLaunchKernelGGL((k_bapply_w<T, W>), grid, blk, 0, st, P, M, N, row_start, vals, b, v, r);
    e = hipGetLastError();
  });
  return e;
}

// kind 0: p = R^{-1} c (checked);  1: out += R^{-1} rhs;  2: y = R^{-T} rhs
template <typename T>
hipError_t launch_bsweep_w(int kind, int P, int64_t N, int w, const T* R16, const double* binv, const T* rhsT,
                           const double* rhsD, double* out, int* status, hipStream_t st) {
  if (!bsweep_w_fits(P, N, w, sizeof(T))) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(((int64_t)P * 16 + 255) / 256)), blk(256);
  hipError_t e = hipErrorInvalidValue;
  bw_host_for<1, 16>([&](auto WW) {
    constexpr int W = decltype(WW)::value;
    if (w != W) return;
    if (kind == 0)
      hipLaunchKernelGGL((k_bsweep_w<T, W, true, false, true, true>), grid, blk, 0, st, P, N, R16, binv, rhsT,
                         (const double*)nullptr, out, status);
    else if (kind == 1)
      hipLaunchKernelGGL((k_bsweep_w<T, W, true, true, false, false>), grid, blk, 0, st, P, N, R16, binv,
                         (const T*)nullptr, rhsD, out, (int*)nullptr);
    else
      hipLaunchKernelGGL((k_bsweep_w<T, W, false, false, false, false>), grid, blk, 0, st, P, N, R16, binv,
                         (const T*)nullptr, rhsD, out, (int*)nullptr);
    e = hipGetLastError();
  });
  return e;
}

}  // namespace qrk
