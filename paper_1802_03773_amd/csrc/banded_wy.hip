// Block-banded QR of banded J on the matrix cores (QRkit Section 4.4, Eq. blockBandedYTY):
// the banded factor as a sequence of small dense steps, each step's Householder vectors local
// to the rows it touches and applied in the compact WY form (Section 2), float32 with fp32 or
// BF16x3 matrix-core products.  Same outputs as the Givens kernels (band R, c, reciprocal
// pivots, the 16-slot sweep copy), so back-substitution, refinement, the adjoint and the LM
// driver use it unchanged.
//
// One wave per problem.  Columns go in blocks of 16 (w <= 15, so a row whose first nonzero is
// in block k ends in block k or k+1).  The wave keeps a running upper triangle of three column
// blocks in the matrix-core accumulator layout: block k, block k+1 and the right-hand side
// (column 32).  At the start of step k its block row 0 is the triangle carried from step k-1
// (block k's damping rows for k = 0), block row 1 the damping rows sqrt(lam) d of block k+1.
// The rows of J whose first nonzero lies in block k are merged into it, 32 at a time, by
// merge_tile: its two column panels are factored (Householder with compact WY, the column
// block of the right-hand side only updated).  Block row 0 is then R's rows 16k .. 16k+15 with
// their entries of c; block row 1, a triangle over block k+1's columns, moves up for step k+1.
// The merged rows' leftover right-hand side is the residual, which the banded step does not
// keep.
//
// A row start below its predecessor's or outside [0, N - w] is flagged as bad input, as in the
// Givens kernels (the factor of such a call is not meaningful); starts are clamped into
// [16k, N - w] when their row is reached, so that every row is merged exactly once.
#include "qrk_banded.hpp"
#include "qrk_device.hpp"
#include "tsqr_mfma.hpp"

namespace qrk {

template <bool BF>
__global__ void __launch_bounds__(256, 2)
k_bwy(int P, int64_t M, int64_t N, int w, const int32_t* __restrict__ row_start, const float* __restrict__ vals,
      const float* __restrict__ bvec, const double* __restrict__ d, const double* __restrict__ lam,
      float* __restrict__ Rb, float* __restrict__ cb, double* __restrict__ binv, float* __restrict__ R16,
      int* __restrict__ status) {
  constexpr int NCB = 3;       // block k, block k+1, right-hand side
  constexpr int NRB = 2;       // 32 rows of J per merge
  constexpr int KT = 16 * NRB;
  __shared__ float lds_all[4][kWaveLds];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t prob = (int64_t)blockIdx.x * 4 + wv;
  if (prob >= P) return;
  float* lds = lds_all[wv];
  const int g = lane >> 4;
  const int c = lane & 15;
  const float sl = (float)sqrt(lam[prob]);
  const int32_t* rs = row_start + prob * M;
  const float* V = vals + prob * M * w;
  const float* bb = bvec + prob * M;
  const double* dd = d + prob * N;
  float* R = Rb + prob * N * w;
  float* cc = cb + prob * N;
  double* iv = binv + prob * N;
  float* S16 = R16 ? R16 + prob * N * 16 : nullptr;
  const int64_t smax = N - w;

  f4 T[Tri<NCB>::count];
#pragma unroll
  for (int t = 0; t < Tri<NCB>::count; ++t) T[t] = f4{0.f, 0.f, 0.f, 0.f};
  // damping rows of block 0 (block row 0) and block 1 (block row 1): diagonal entries
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (4 * g + v == c) {
      T[Tri<NCB>::idx(0, 0)][v] = c < N ? sl * (float)dd[c] : 0.f;
      T[Tri<NCB>::idx(1, 1)][v] = 16 + c < N ? sl * (float)dd[16 + c] : 0.f;
    }
  }

  bool bad = false;
  int64_t i = 0;      // next row of J
  int32_t slast = 0;  // start of row i - 1 (as given)
  const int64_t nblk = (N + 15) / 16;
  for (int64_t k = 0; k < nblk; ++k) {
    const int64_t lo = 16 * k;
    // ---- merge the rows whose first nonzero lies in block k, KT at a time -------------------
    while (i < M) {
      // effective starts of rows i .. i+KT-1 (lanes 0 .. KT-1), clamped into [lo, N - w]; a
      // start below its predecessor's or outside [0, N - w] is flagged
      const bool have = lane < KT && i + lane < M;
      const int32_t s0 = have ? rs[i + lane] : 0;
      const int32_t sp = lane == 0 ? slast : __shfl_up(s0, 1, 64);
      if (have && (s0 < sp || s0 < 0 || (int64_t)s0 > smax)) bad = true;
      const int64_t st = s0 < lo ? lo : ((int64_t)s0 > smax ? smax : (int64_t)s0);
      const bool in = have && st < lo + 16;
      const uint64_t ball = __ballot(in);
      const int cnt = (int)__builtin_ctzll(~ball);  // the leading rows that belong to block k
      if (cnt == 0) break;
      slast = __shfl(s0, cnt - 1, 64);
      f4 X[NRB][NCB];
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rt = rb * 16 + 4 * g + v;  // row of the tile
          const int o = (int)(__shfl((int)(st - lo), rt, 64));
          const bool live = rt < cnt;
          const int64_t row = i + rt;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int l = 16 * q + c - o;
            X[rb][q][v] = (live && l >= 0 && l < w) ? V[row * w + l] : 0.f;
          }
          X[rb][2][v] = (live && c == 0) ? bb[row] : 0.f;
        }
      merge_tile<NCB, NRB, false, BF, 2, true>(T, X, 0, lds, lane);
      i += cnt;
      if (cnt < KT) break;
    }
    // ---- R's rows 16k .. 16k+15 from block row 0 ------------------------------------------
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ri = 4 * g + v;
      const int64_t r = lo + ri;
      if (r < N) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int l = 16 * q + c - ri;  // R[r][r + l]
          const float val = T[Tri<NCB>::idx(0, q)][v];
          if (l >= 0 && l < w) R[r * w + l] = val;
          if (S16 && l >= 0 && l < 16) S16[r * 16 + l] = (l >= 1 && l < w) ? val : 0.f;
          if (l == 0) iv[r] = 1.0 / (double)val;
        }
        if (c == 0) cc[r] = T[Tri<NCB>::idx(0, 2)][v];
      }
    }
    // ---- block row 1 moves up; block k+2's damping rows enter -------------------------------
    T[Tri<NCB>::idx(0, 0)] = T[Tri<NCB>::idx(1, 1)];
    T[Tri<NCB>::idx(0, 1)] = f4{0.f, 0.f, 0.f, 0.f};
    T[Tri<NCB>::idx(0, 2)] = T[Tri<NCB>::idx(1, 2)];
    T[Tri<NCB>::idx(1, 2)] = f4{0.f, 0.f, 0.f, 0.f};
    T[Tri<NCB>::idx(2, 2)] = f4{0.f, 0.f, 0.f, 0.f};
    const int64_t col = lo + 32 + c;
    const float dq = col < N ? sl * (float)dd[col] : 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) T[Tri<NCB>::idx(1, 1)][v] = (4 * g + v == c) ? dq : 0.f;
  }
  if (i < M) bad = true;  // rows left over (not reached by any block): bad starts
  if (__ballot(bad) != 0 && lane == 0) set_status(status, ST_BADINPUT);
}

template <typename T>
hipError_t launch_bwy(bool bf16x3, int P, int64_t M, int64_t N, int w, const int32_t* row_start, const T* vals,
                      const T* b, const double* d, const double* lam, T* Rb, T* cb, double* binv, T* R16,
                      int* status, hipStream_t st) {
  if constexpr (!std::is_same<T, float>::value) {
    return hipErrorInvalidValue;
  } else {
    if (w < 1 || w > 15) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((P + 3) / 4)), blk(256);
    if (bf16x3)
      hipLaunchKernelGGL((k_bwy<true>), grid, blk, 0, st, P, M, N, w, row_start, vals, b, d, lam, Rb, cb, binv,
                         R16, status);
    else
      hipLaunchKernelGGL((k_bwy<false>), grid, blk, 0, st, P, M, N, w, row_start, vals, b, d, lam, Rb, cb, binv,
                         R16, status);
    return hipGetLastError();
  }
}

template hipError_t launch_bwy<float>(bool, int, int64_t, int64_t, int, const int32_t*, const float*, const float*,
                                      const double*, const double*, float*, float*, double*, float*, int*,
                                      hipStream_t);
template hipError_t launch_bwy<double>(bool, int, int64_t, int64_t, int, const int32_t*, const double*,
                                       const double*, const double*, const double*, double*, double*, double*,
                                       double*, int*, hipStream_t);

}  // namespace qrk
