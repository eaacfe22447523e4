// Per-block Householder QR of the block-diagonal part and the in-place application of
// Q_i^T to the coupled columns (QRkit Sections 4.1 and 4.2; damping rows placed below
// each block as in the Backtrack LM of Section 5.2), for one block by one wave64.
//
// Lane j < n owns column j of [A_i; sqrt(lam) D_i]; every lane owns coupled columns lane
// and lane+64 of [B_i | b_i; 0 | 0] (b is column nB).  All rows of a block live in
// registers (ROWS >= m_i + n), so Q_i^T is applied without any cross-lane reduction: each
// Householder vector is broadcast once through LDS and each lane updates its own columns.
// B_i rows are read with consecutive lanes on consecutive columns (coalesced).
// R_i and the coupling rows S_i | c_i are written to global memory; the m_i reduced rows
// are handed to emit(row_in_block, column, value) (global memory or an LDS tile).
#pragma once

#include "qrk_device.hpp"

namespace qrk {

// A, B, bvec point at the block's first row (of A, of B_p with row stride ldb, of b), d at
// its first damping entry, Rb and Scb at its R_i (n x n) and S_i | c_i (n x (nB+1)).
// cam (non-null: camera columns, at the block's first row): B holds each row's ldb values, in
// the columns of camera cam[r] (cameras of ldb columns, nB = ncam * ldb; a camera outside
// [0, ncam) is none).
template <typename T, int ROWS, int SLOTS, typename Emit>
__device__ __forceinline__ void block_qr_wave(int n, int nB, int m, const T* __restrict__ A,
                                              const T* __restrict__ B, int64_t ldb, const T* __restrict__ bvec,
                                              const double* __restrict__ d, double sqrt_lam, T* __restrict__ Rb,
                                              T* __restrict__ Scb, T* __restrict__ v, T* __restrict__ tb,
                                              int lane, Emit&& emit, const int32_t* __restrict__ cam = nullptr) {
  const int L = nB + 1;
  const int rows = m + n;

  T a[ROWS];
  T c[SLOTS][ROWS];
  const T dl = (lane < n) ? (T)(sqrt_lam * d[lane < n ? lane : 0]) : T(0);
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    T x = T(0);
    if (lane < n) {
      if (r < m)
        x = A[r * n + lane];
      else if (r == m + lane)
        x = dl;
    }
    a[r] = x;
  }
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int col = s * 64 + lane;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      T x = T(0);
      if (r < m) {
        if (col < nB) {
          if (cam) {
            const int cr = cam[r];
            if ((uint32_t)cr < (uint32_t)(nB / ldb)) {
              const uint32_t k = (uint32_t)(col - cr * (int)ldb);
              if (k < (uint32_t)ldb) x = B[r * ldb + k];
            }
          } else {
            x = B[r * ldb + col];
          }
        } else if (col == nB) {
          x = bvec[r];
        }
      }
      c[s][r] = x;
    }
  }

  for (int k = 0; k < n; ++k) {
    // Each lane forms the reflector of its own column; lane k's is the one used.
    T alpha = T(0), sig0 = T(0), sig1 = T(0);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
      if (r == k) alpha = a[r];
      if (r > k && r < rows) {
        if (r & 1)
          sig1 += a[r] * a[r];
        else
          sig0 += a[r] * a[r];
      }
    }
    const T sigma = sig0 + sig1;
    T beta = alpha, tau = T(0), scale = T(0);
    if (sigma != T(0)) {
      const T nrm = sqrt(alpha * alpha + sigma);
      beta = alpha >= T(0) ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = T(1) / (alpha - beta);
    }
    if (lane == k) {
#pragma unroll
      for (int r = 0; r < ROWS; ++r)
        v[r] = (r == k) ? T(1) : ((r > k && r < rows) ? a[r] * scale : T(0));
      *tb = tau;
    }
    wave_lds_sync();
    T vr[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) vr[r] = v[r];
    const T tk = *tb;
    wave_lds_sync();
    if (tk != T(0)) {
      T w0 = T(0), w1 = T(0);
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        if (r & 1)
          w1 += vr[r] * a[r];
        else
          w0 += vr[r] * a[r];
      }
      const T w = (w0 + w1) * tk;
#pragma unroll
      for (int r = 0; r < ROWS; ++r) a[r] -= vr[r] * w;
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        T u0 = T(0), u1 = T(0);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
          if (r & 1)
            u1 += vr[r] * c[s][r];
          else
            u0 += vr[r] * c[s][r];
        }
        const T u = (u0 + u1) * tk;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) c[s][r] -= vr[r] * u;
      }
    }
    if (lane == k) {
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        if (r == k) a[r] = beta;
        if (r > k) a[r] = T(0);
      }
    }
  }

  // R_i: lane j < n holds column j.
  if (lane < n) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (r < n) Rb[r * n + lane] = (r <= lane) ? a[r] : T(0);
  }
  // Coupling rows (top n) and reduced rows (the other m).
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int col = s * 64 + lane;
    if (col < L) {
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        if (r < n)
          Scb[r * L + col] = c[s][r];
        else if (r < rows)
          emit(r - n, col, c[s][r]);
      }
    }
  }
}

}  // namespace qrk
