// Back-substitution through the structured R of a horizontal concatenation
// (QRkit Section 4.2: R = [[blkdiag(R_i), S], [0, R_B]]) and corrected
// semi-normal-equation refinement of the step (Bjorck 1987):
//     r = b - J p,  g = J^T r - lam D^2 p   (float64),
//     R^T y = g,  R delta = y,  p <- p + delta.
// The two triangular solves run through the structure:
//     R_i^T y_i = g_i;   R_B^T y_B = g_B - sum_i S_i^T y_i;
//     R_B delta_B = y_B; R_i delta_i = y_i - S_i delta_B.
// Sums over blocks are deterministic: per-wave partials in registers, workgroup partials
// combined in a fixed order, then a fixed-order reduction of the workgroup partials.
// Every kernel serves a batch of independent problems (ProbDesc); a single problem is the
// batch of one.
#include "qrk_batch.hpp"
#include "qrk_device.hpp"
#include "qrk_launch.hpp"

namespace qrk {

// ---------------------------------------------------------------------------------
// Dense triangle, one wave: forward (R_B^T y = g) and backward (R_B x = y) sweeps with
// R_B staged in LDS.  Lane i holds rows i and i + 64 of the right-hand side.
// ---------------------------------------------------------------------------------
// R_B (L x L, row-major) into LDS by NT threads: each thread issues all of its loads before
// its first store, so the copy costs one memory latency rather than one per element.
template <typename T, int NT>
__device__ __forceinline__ void stage_dense(const T* __restrict__ RB, int L, float* Rs, double* Rsd, int tid) {
  constexpr int PER = (kMaxDense * kMaxDense + NT - 1) / NT;
  const int LL = L * L;
  T buf[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + u * NT;
    buf[u] = e < LL ? RB[e] : T(0);
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + u * NT;
    if (e < LL) {
      if constexpr (sizeof(T) == 4)
        Rs[e] = (float)buf[u];
      else
        Rsd[e] = (double)buf[u];
    }
  }
}

template <typename T>
__device__ __forceinline__ double rs_at(const float* Rs, const double* Rsd, int e) {
  if constexpr (sizeof(T) == 4)
    return (double)Rs[e];
  else
    return Rsd[e];
}

__device__ __forceinline__ double read_lane_d(double x, int lane) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Reciprocals of the diagonal of R for rows lane and lane + 64 (1 past nB), computed by all
// lanes at once so the sweeps below multiply instead of dividing on their critical path.
template <typename T>
__device__ __forceinline__ void dense_diag_inv(const float* Rs, const double* Rsd, int L, int nB, int lane,
                                               double& dv0, double& dv1) {
  dv0 = lane < nB ? 1.0 / rs_at<T>(Rs, Rsd, lane * L + lane) : 1.0;
  dv1 = lane + 64 < nB ? 1.0 / rs_at<T>(Rs, Rsd, (lane + 64) * L + lane + 64) : 1.0;
}

// Forward: y = R^{-T} g (upper-triangular R, column sweep).  v0/v1 hold g for rows lane and
// lane + 64 on entry and y on exit; dv0/dv1 the reciprocal diagonal.  Step k broadcasts
// y_k = v_k / R_kk from lane k and takes R_kj y_k off every later row j; a row's value is
// final once its own step is past, so every lane scales by its reciprocal at the end.  The
// entries of R for eight steps are read from LDS in one batch (masked to the rows a step
// updates), so a step waits on no LDS access.
template <typename T>
__device__ __forceinline__ void wave_fwd_T(const float* Rs, const double* Rsd, int L, int nB, int lane,
                                           double dv0, double dv1, double& v0, double& v1) {
  for (int kb = 0; kb < nB; kb += 8) {
    double r0[8], r1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = kb + u < nB ? kb + u : nB - 1;
      const double a0 = rs_at<T>(Rs, Rsd, k * L + lane);
      const double a1 = rs_at<T>(Rs, Rsd, k * L + lane + 64);
      r0[u] = (lane > k && lane < nB) ? a0 : 0.0;
      r1[u] = (lane + 64 > k && lane + 64 < nB) ? a1 : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = kb + u;
      if (k < nB) {
        const double yk = read_lane_d(k < 64 ? v0 * dv0 : v1 * dv1, k & 63);
        v0 -= r0[u] * yk;
        v1 -= r1[u] * yk;
      }
    }
  }
  v0 *= dv0;
  v1 *= dv1;
}

// Backward: x = R^{-1} y, columns from the last; the same batching and final scaling.
template <typename T>
__device__ __forceinline__ void wave_bwd(const float* Rs, const double* Rsd, int L, int nB, int lane,
                                         double dv0, double dv1, double& v0, double& v1) {
  for (int kb = nB - 1; kb >= 0; kb -= 8) {
    double r0[8], r1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = kb - u >= 0 ? kb - u : 0;
      const double a0 = rs_at<T>(Rs, Rsd, lane * L + k);
      const double a1 = rs_at<T>(Rs, Rsd, (lane + 64) * L + k);
      r0[u] = lane < k ? a0 : 0.0;
      r1[u] = lane + 64 < k ? a1 : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = kb - u;
      if (k >= 0) {
        const double xk = read_lane_d(k < 64 ? v0 * dv0 : v1 * dv1, k & 63);
        v0 -= r0[u] * xk;
        v1 -= r1[u] * xk;
      }
    }
  }
  v0 *= dv0;
  v1 *= dv1;
}

// ---------------------------------------------------------------------------------
// Dense part of the back-substitution: R_B p_B = c_B, one workgroup (one working wave)
// per problem.  c_B is column L-1 of R_B | c_B, or cext (laid out like p) when that is given.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
k_backsub_dense(const ProbDesc* __restrict__ probs, int n, const T* __restrict__ RBall, double* __restrict__ p,
                int* __restrict__ status, const double* __restrict__ cext) {
  __shared__ float Rs[sizeof(T) == 4 ? kMaxDense * kMaxDense : 1];
  __shared__ double Rsd[sizeof(T) == 8 ? kMaxDense * kMaxDense : 1];
  const int pi = blockIdx.x;
  const ProbDesc& P = probs[pi];
  const int L = P.L, nB = P.nB;
  const int64_t off = P.noff + P.K * n;
  stage_dense<T, 256>(RBall + P.rboff, L, Rs, Rsd, threadIdx.x);
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  double v0 = lane < nB ? (cext ? cext[off + lane] : rs_at<T>(Rs, Rsd, lane * L + nB)) : 0.0;
  double v1 = lane + 64 < nB ? (cext ? cext[off + lane + 64] : rs_at<T>(Rs, Rsd, (lane + 64) * L + nB)) : 0.0;
  // largest pivot magnitude: each lane its own diagonal entries, then a wave maximum
  const double dg0 = lane < nB ? fabs(rs_at<T>(Rs, Rsd, lane * L + lane)) : 0.0;
  const double dg1 = lane + 64 < nB ? fabs(rs_at<T>(Rs, Rsd, (lane + 64) * L + lane + 64)) : 0.0;
  const double dmax = wave_allreduce_max(fmax(dg0, dg1));
  bool bad = false;
  for (int k = lane; k < nB; k += 64) {
    const double piv = rs_at<T>(Rs, Rsd, k * L + k);
    if (is_finite(piv) && !(fabs(piv) > (double)nB * Eps<T>::value * dmax)) bad = true;
  }
  double dv0, dv1;
  dense_diag_inv<T>(Rs, Rsd, L, nB, lane, dv0, dv1);
  wave_bwd<T>(Rs, Rsd, L, nB, lane, dv0, dv1, v0, v1);
  bool nonfinite = false;
  if (lane < nB) {
    p[off + lane] = v0;
    nonfinite |= !is_finite(v0);
  }
  if (lane + 64 < nB) {
    p[off + lane + 64] = v1;
    nonfinite |= !is_finite(v1);
  }
  if (bad) set_status(status + pi, ST_SINGULAR);
  if (nonfinite) set_status(status + pi, ST_NONFINITE);
}

template <typename T>
hipError_t launch_backsub_dense(const BatchView& bv, const T* RB, double* p, int* status, hipStream_t st,
                                const double* cext) {
  if (bv.max_L > kMaxDense) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_backsub_dense<T>), dim3(bv.P), dim3(256), 0, st, bv.probs, bv.n, RB, p, status, cext);
  return hipGetLastError();
}

// Raw buffer load of one element: the descriptor holds the wave-uniform row-block base, the
// row offset is the scalar offset and the lane's column offset the vector offset.  Word 3
// is the gfx9 raw-buffer format; the record count only bounds the range check, and every
// offset used stays inside the rows of the pack.
template <typename T>
__device__ __forceinline__ T buf_ld_row(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}

// ---------------------------------------------------------------------------------
// Blocks, pack-wise: x_i (= | +=) R_i^{-1} (base_i - S_i v) for the blocks of a pack (the
// packs and workgroup-to-problem map of refinement pass 1); v is the dense-part vector of
// the pack's problem.  The pack's coupling rows S|c are contiguous: they are streamed 16
// rows at a time through the wave's LDS tile (column-major, stride 17) and each row's dot
// with v is summed by four lanes; then lane k back-substitutes block k of the pack.
//   MODE 0 back-substitution: base_i = c_i (column nB of S|c, staged with weight -1),
//                             v = p_B, p_i set, pivot and finiteness status;
//   MODE 1 refinement:        base_i = y_i, v = delta_B, p_i incremented;
//   MODE 2 adjoint:           base_i = y_i, v = u_B, u_i set;
//   MODE 3 back-substitution for a given c (laid out like p, in ybase): base_i = c_i,
//                             v = p_B, p_i set, pivot and finiteness status.
// ---------------------------------------------------------------------------------
template <typename T, int N, int MODE>
__global__ void __launch_bounds__(256)
k_blocks_solve_n(const ProbDesc* __restrict__ probs, const int32_t* __restrict__ wg_prob,
                 const int64_t* __restrict__ pack_blk, const T* __restrict__ Rblk, const T* __restrict__ Sc,
                 const double* __restrict__ vbuf, const double* __restrict__ ybase, double* __restrict__ x,
                 int* __restrict__ status) {
  constexpr int CH = 16, LS = CH + 1;
  constexpr int MAXR = 64 * N;  // coupling rows of a pack (at most 64 blocks)
  __shared__ T tile_all[4][kMaxDense * LS];
  __shared__ double rhs_all[4][MAXR + CH];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  T* tile = tile_all[wv];
  double* rhs = rhs_all[wv];
  const int pi = wg_prob[blockIdx.x];
  const ProbDesc& P = probs[pi];
  const int nB = P.nB, L = P.L;
  const int64_t koff = P.koff, noff = P.noff, soff = P.soff;
  const double* v = MODE == 1 ? vbuf + (int64_t)pi * kMaxDense : vbuf + P.noff + P.K * N;
  // staged columns: nB (and the c column with weight -1 in mode 0)
  const int ncol = MODE == 0 ? L : nB;
  const int qi = lane & 15, qq = lane >> 4;
  double pq[kMaxDense / 4];
#pragma unroll
  for (int t = 0; t < kMaxDense / 4; ++t) {
    const int j = 4 * t + qq;
    pq[t] = j < nB ? v[j] : ((MODE == 0 && j == nB) ? -1.0 : 0.0);
  }
  const bool c0ok = lane < ncol, c1ok = lane + 64 < ncol;
  const uint32_t co0 = (uint32_t)(c0ok ? lane : 0) * (uint32_t)sizeof(T);
  const uint32_t co1 = (uint32_t)(c1ok ? lane + 64 : 0) * (uint32_t)sizeof(T);
  const int64_t lw = blockIdx.x - P.wg0;
  const int64_t pend = P.pack0 + P.npacks;
  for (int64_t pk = P.pack0 + lw * 4 + wv; pk < pend; pk += (int64_t)P.nwg * 4) {
    const int64_t b0 = pack_blk[pk];
    const int nb = (int)(pack_blk[pk + 1] - b0);
    const int rs = nb * N;
    // this lane's block (lanes < nb): R_i and the base values, loaded before the stream
    const int kb = lane < nb ? lane : nb - 1;
    const int64_t blk = b0 + kb;
    const int64_t lb = blk - koff;
    T Rb[N * N];
#pragma unroll
    for (int e = 0; e < N * N; ++e) Rb[e] = Rblk[blk * (N * N) + e];
    double base[N];
#pragma unroll
    for (int c = 0; c < N; ++c) base[c] = MODE == 0 ? 0.0 : (MODE == 3 ? ybase[noff + lb * N + c] : ybase[blk * N + c]);
    double xold[N];
#pragma unroll
    for (int c = 0; c < N; ++c) xold[c] = MODE == 1 ? x[noff + lb * N + c] : 0.0;
    const __amdgpu_buffer_rsrc_t rsS =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(Sc + soff + (b0 - koff) * N * L), 0, 0x7fffffff,
                                          0x00020000);
    for (int c0 = 0; c0 < rs; c0 += CH) {
      const int last = rs - 1 - c0;
      T v0[CH], v1[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int ri = i < last ? i : last;
        const uint32_t so = (uint32_t)((c0 + ri) * L) * (uint32_t)sizeof(T);
        const T x0 = buf_ld_row<T>(rsS, co0, so);
        const T x1 = buf_ld_row<T>(rsS, co1, so);
        v0[i] = c0ok ? x0 : T(0);
        v1[i] = c1ok ? x1 : T(0);
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        tile[lane * LS + i] = v0[i];
        tile[(lane + 64) * LS + i] = v1[i];
      }
      wave_lds_sync();
      double acc = 0.0;
      auto tier = [&](auto t_begin) {
        constexpr int tb = decltype(t_begin)::value;
#pragma unroll
        for (int t = tb; t < tb + 8; ++t) acc += (double)tile[(4 * t + qq) * LS + qi] * pq[t];
      };
      tier(std::integral_constant<int, 0>{});
      if (ncol > 32) tier(std::integral_constant<int, 8>{});
      if (ncol > 64) tier(std::integral_constant<int, 16>{});
      if (ncol > 96) tier(std::integral_constant<int, 24>{});
      acc += __shfl_xor(acc, 16, 64);
      acc += __shfl_xor(acc, 32, 64);
      if (qq == 0) rhs[c0 + qi] = -acc;  // -(S v) (mode 0: c - S p_B)
      wave_lds_sync();  // the next chunk overwrites the tile
    }
    if (lane < nb) {
      double rr[N], out[N];
#pragma unroll
      for (int c = 0; c < N; ++c) rr[c] = base[c] + rhs[lane * N + c];
#pragma unroll
      for (int i = N - 1; i >= 0; --i) {
        double sacc = rr[i];
#pragma unroll
        for (int j = i + 1; j < N; ++j) sacc -= (double)Rb[i * N + j] * out[j];
        out[i] = sacc / (double)Rb[i * N + i];
      }
      bool nonfinite = false;
      double* xo = x + noff + lb * N;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        xo[c] = MODE == 1 ? xold[c] + out[c] : out[c];
        nonfinite |= !is_finite(out[c]);
      }
      if ((MODE == 0 || MODE == 3) && status) {
        double dmax = 0.0;
#pragma unroll
        for (int c = 0; c < N; ++c) dmax = fmax(dmax, fabs((double)Rb[c * N + c]));
        bool bad = false;
#pragma unroll
        for (int c = 0; c < N; ++c) {
          const double piv = (double)Rb[c * N + c];
          if (is_finite(piv) && !(fabs(piv) > (double)N * Eps<T>::value * dmax)) bad = true;
        }
        if (bad) set_status(status + pi, ST_SINGULAR);
        if (nonfinite) set_status(status + pi, ST_NONFINITE);
      }
    }
    wave_lds_sync();  // the next pack overwrites rhs
  }
}

template <typename T, int MODE>
static hipError_t launch_blocks_solve(const BatchView& bv, const T* Rblk, const T* Sc, const double* vbuf,
                                      const double* ybase, double* x, int* status, hipStream_t st) {
  if (bv.max_L > kMaxDense) return hipErrorInvalidValue;
  switch (bv.n) {
#define QRK_BS(NN)                                                                                          \
  case NN:                                                                                                  \
    hipLaunchKernelGGL((k_blocks_solve_n<T, NN, MODE>), dim3(bv.nwg), dim3(256), 0, st, bv.probs, bv.wg_prob, \
                       bv.pack_blk, Rblk, Sc, vbuf, ybase, x, status);                                     \
    break;
    QRK_BS(1) QRK_BS(2) QRK_BS(3) QRK_BS(4) QRK_BS(5) QRK_BS(6) QRK_BS(7) QRK_BS(8)
#undef QRK_BS
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_backsub_blocks(const BatchView& bv, const T* Rblk, const T* Sc, double* p, int* status,
                                 hipStream_t st, const double* cext) {
  if (cext) return launch_blocks_solve<T, 3>(bv, Rblk, Sc, p, cext, p, status, st);
  return launch_blocks_solve<T, 0>(bv, Rblk, Sc, p, nullptr, p, status, st);
}

template <typename T>
hipError_t launch_refine_blocks(const BatchView& bv, const T* Rblk, const T* Sc, const double* y,
                                const double* delta_B, double* p, hipStream_t st) {
  return launch_blocks_solve<T, 1>(bv, Rblk, Sc, delta_B, y, p, nullptr, st);
}

template <typename T>
hipError_t launch_adjoint_blocks(const BatchView& bv, const T* Rblk, const T* Sc, const double* y, double* u,
                                 hipStream_t st) {
  return launch_blocks_solve<T, 2>(bv, Rblk, Sc, u, y, u, nullptr, st);
}

// ---------------------------------------------------------------------------------
// Refinement pass 1: one wave per pack of whole blocks (at most 64 rows).
//   r = b - A_i p_i - B p_B;  g_i = A_i^T r - lam d_i^2 p_i;  y_i = R_i^{-T} g_i;
//   per-workgroup partial of  B^T r - sum_i S_i^T y_i.
// The pack's rows of B are read once, coalesced, 16 rows at a time, and staged in the wave's
// LDS tile column-major with an odd column stride (17), so both products read it without
// bank conflicts: B p_B with four lanes per row (each summing every fourth column, then two
// shuffles), B^T r with one lane per column straight from the registers the chunk was
// loaded into.  Every sum runs in a fixed order, so the partials are deterministic.
// Workgroup w serves problem wg_prob[w] only; its packs are that problem's packs
// lw*4 + wave, lw*4 + wave + 4*nwg, ... (lw = w - wg0), its partial goes to part[w].
// CAM: the coupled columns are cameras of ldb columns (nB = ncam * ldb); B holds each row's ldb
// values and cam[row] its camera (outside [0, ncam): none), so a staged row is zero outside its
// camera's columns.
// ---------------------------------------------------------------------------------

template <typename T, int N, bool CAM>
__global__ void __launch_bounds__(256)
k_refine_pass1(const ProbDesc* __restrict__ probs, const int32_t* __restrict__ wg_prob,
               const int64_t* __restrict__ pack_blk, const int64_t* __restrict__ row_off,
               const T* __restrict__ A, const T* __restrict__ B, const int32_t* __restrict__ cam,
               const T* __restrict__ bvec,
               const double* __restrict__ d, const double* __restrict__ lamv, const T* __restrict__ Rblk,
               const T* __restrict__ Sc, const double* __restrict__ p, double* __restrict__ y,
               double* __restrict__ part) {
  constexpr int CH = 16;      // rows per staged chunk
  constexpr int LS = CH + 1;  // column stride of the staged tile
  static_assert(4 * kMaxDense * LS * sizeof(T) >= 4 * kMaxDense * sizeof(double), "reduction fits the tile");
  __shared__ T tile_all[4][kMaxDense * LS];
  __shared__ double rr_all[4][64 + CH];         // r per pack row (0 past the pack)
  __shared__ double prod_all[4][64 * N];        // A_row * r per pack row
  __shared__ double yv_all[4][64 * N + CH];     // y per coupling row (0 past the pack's blocks)
  __shared__ int rowblk_all[4][64];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  T* tile = tile_all[wv];
  double* rr = rr_all[wv];
  double* prod = prod_all[wv];
  double* yv = yv_all[wv];
  int* rowblk = rowblk_all[wv];
  const int pi = wg_prob[blockIdx.x];
  const ProbDesc& P = probs[pi];
  const int nB = P.nB, L = P.L;
  const int64_t koff = P.koff, noff = P.noff, moff = P.moff, soff = P.soff;
  const int ldb = nB > 0 ? (int)P.ldb : 0;
  const uint32_t ncam = CAM ? (uint32_t)(nB / ldb) : 0u;
  const double lam = lamv[pi];
  const double* pBv = p + noff + P.K * N;
  const int qi = lane & 15, qq = lane >> 4;  // row pass: row qi of the chunk, columns 4t + qq
  double pq[kMaxDense / 4];
#pragma unroll
  for (int t = 0; t < kMaxDense / 4; ++t) {
    const int j = 4 * t + qq;
    pq[t] = j < nB ? pBv[j] : 0.0;
  }
  const bool c0ok = lane < nB, c1ok = lane + 64 < nB;
  const uint32_t co0 = (uint32_t)(c0ok ? lane : 0) * (uint32_t)sizeof(T);
  const uint32_t co1 = (uint32_t)(c1ok ? lane + 64 : 0) * (uint32_t)sizeof(T);
  double t0 = 0.0, t1 = 0.0;  // partial B^T r - S^T y for columns lane, lane + 64
  const int64_t lw = blockIdx.x - P.wg0;
  const int64_t pend = P.pack0 + P.npacks;
  for (int64_t pk = P.pack0 + lw * 4 + wv; pk < pend; pk += (int64_t)P.nwg * 4) {
    const int64_t b0 = pack_blk[pk];
    const int nb = (int)(pack_blk[pk + 1] - b0);
    const int64_t pr0 = row_off[b0];
    const int prows = (int)(row_off[b0 + nb] - pr0);
    if (lane < nb) {
      const int lo = (int)(row_off[b0 + lane] - pr0), hi = (int)(row_off[b0 + lane + 1] - pr0);
      for (int r = lo; r < hi; ++r) rowblk[r] = lane;
    }
    wave_lds_sync();
    // with nB == 0 there may be no B at all: the (discarded) loads then read b[pr0]
    const T* Bbase = nB > 0 ? B + P.boff + (pr0 - moff) * ldb : bvec + pr0;
    const __amdgpu_buffer_rsrc_t rsB =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(Bbase), 0, 0x7fffffff, 0x00020000);
    // the pack's rows in chunks; W: the problem has coupled columns past 64 (the second column
    // slot of each lane holds some), else that slot is left out of the loads and products
    auto chunks = [&](auto Wc) {
      constexpr bool W = decltype(Wc)::value;
      for (int c0 = 0; c0 < prows; c0 += CH) {
        const int last = prows - 1 - c0;  // rows past the pack re-read its last row; their r is 0
        // this lane's row of the chunk for the r update (lanes 0..15): its A row and p_i
        const int myrow = c0 + (qi < last ? qi : last);
        const int64_t grow = pr0 + myrow;
        const int64_t lbr = b0 - koff + rowblk[myrow];
        T arow[N];
        double prow[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
          arow[c] = A[grow * N + c];
          prow[c] = p[noff + lbr * N + c];
        }
        const T bval = bvec[grow];
        // stage rows c0 .. c0 + 15; columns >= nB are zeros
        T v0[CH], v1[W ? CH : 1];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int ri = i < last ? i : last;
          const uint32_t so = (uint32_t)((c0 + ri) * ldb) * (uint32_t)sizeof(T);
          if constexpr (CAM) {
            const int cr = cam[pr0 + c0 + ri];
            const bool seen = (uint32_t)cr < ncam;
            const int cb = (seen ? cr : 0) * ldb;
            const uint32_t k0 = (uint32_t)(lane - cb), k1 = (uint32_t)(lane + 64 - cb);
            const bool on0 = seen && k0 < (uint32_t)ldb, on1 = seen && k1 < (uint32_t)ldb;
            const T x0 = buf_ld_row<T>(rsB, (on0 ? k0 : 0u) * (uint32_t)sizeof(T), so);
            v0[i] = on0 ? x0 : T(0);
            if constexpr (W) {
              const T x1 = buf_ld_row<T>(rsB, (on1 ? k1 : 0u) * (uint32_t)sizeof(T), so);
              v1[i] = on1 ? x1 : T(0);
            }
          } else {
            const T x0 = buf_ld_row<T>(rsB, co0, so);
            v0[i] = c0ok ? x0 : T(0);
            if constexpr (W) {
              const T x1 = buf_ld_row<T>(rsB, co1, so);
              v1[i] = c1ok ? x1 : T(0);
            }
          }
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          tile[lane * LS + i] = v0[i];
          if constexpr (W) tile[(lane + 64) * LS + i] = v1[i];
        }
        wave_lds_sync();
        // B p_B for row c0 + qi: lanes qi, qi + 16, qi + 32, qi + 48 split the columns
        // (32-column tiers; the columns past nB are zeros)
        double acc = 0.0;
        auto tier = [&](auto t_begin) {
          constexpr int tb = decltype(t_begin)::value;
#pragma unroll
          for (int t = tb; t < tb + 8; ++t) acc += (double)tile[(4 * t + qq) * LS + qi] * pq[t];
        };
        tier(std::integral_constant<int, 0>{});
        if (nB > 32) tier(std::integral_constant<int, 8>{});
        if constexpr (W) {
          tier(std::integral_constant<int, 16>{});
          if (nB > 96) tier(std::integral_constant<int, 24>{});
        }
        acc += __shfl_xor(acc, 16, 64);
        acc += __shfl_xor(acc, 32, 64);
        if (qq == 0) {
          double dot = 0.0;
#pragma unroll
          for (int c = 0; c < N; ++c) dot += (double)arow[c] * prow[c];
          const double rv = qi <= last ? (double)bval - dot - acc : 0.0;
          rr[c0 + qi] = rv;
          if (qi <= last) {
#pragma unroll
            for (int c = 0; c < N; ++c) prod[(c0 + qi) * N + c] = (double)arow[c] * rv;
          }
        }
        wave_lds_sync();
        // B^T r over the chunk's rows, from the registers the chunk was loaded into
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const double rv = rr[c0 + i];
          t0 += (double)v0[i] * rv;
          if constexpr (W) t1 += (double)v1[i] * rv;
        }
        wave_lds_sync();  // the next chunk overwrites the tile
      }
    };
    if (nB > 64)
      chunks(std::true_type{});
    else
      chunks(std::false_type{});
    // per block: g_i = A_i^T r - lam d_i^2 p_i, y_i = R_i^{-T} g_i
    if (lane < nb) {
      const int64_t blk = b0 + lane;
      const int64_t lb = blk - koff;
      double dd[N], pp[N];
      T Rb[N * N];
#pragma unroll
      for (int c = 0; c < N; ++c) {
        dd[c] = d[noff + lb * N + c];
        pp[c] = p[noff + lb * N + c];
      }
#pragma unroll
      for (int e = 0; e < N * N; ++e) Rb[e] = Rblk[blk * (N * N) + e];
      const int lo = (int)(row_off[blk] - pr0), hi = (int)(row_off[blk + 1] - pr0);
      double g[N];
#pragma unroll
      for (int c = 0; c < N; ++c) g[c] = 0.0;
      for (int r = lo; r < hi; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) g[c] += prod[r * N + c];
#pragma unroll
      for (int c = 0; c < N; ++c) g[c] -= lam * dd[c] * dd[c] * pp[c];
      // R_i^T y = g (R_i upper triangular, row-major)
      double yy[N];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double sacc = g[i];
#pragma unroll
        for (int j = 0; j < i; ++j) sacc -= (double)Rb[j * N + i] * yy[j];
        yy[i] = sacc / (double)Rb[i * N + i];
      }
#pragma unroll
      for (int c = 0; c < N; ++c) {
        y[blk * N + c] = yy[c];
        yv[lane * N + c] = yy[c];
      }
    }
    const int rs = nb * N;  // coupling rows of the pack
    if (lane < CH) yv[rs + lane] = 0.0;
    wave_lds_sync();
    // S^T y over the pack's coupling rows (contiguous), 16 rows at a time
    const __amdgpu_buffer_rsrc_t rsS =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(Sc + soff + (b0 - koff) * N * L), 0, 0x7fffffff,
                                          0x00020000);
    const uint32_t so0 = (uint32_t)(c0ok ? lane : 0) * (uint32_t)sizeof(T);
    const uint32_t so1 = (uint32_t)(c1ok ? lane + 64 : 0) * (uint32_t)sizeof(T);
    for (int s0 = 0; s0 < rs; s0 += CH) {
      const int last = rs - 1 - s0;
      T w0[CH], w1[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int ri = i < last ? i : last;
        const uint32_t so = (uint32_t)((s0 + ri) * L) * (uint32_t)sizeof(T);
        w0[i] = buf_ld_row<T>(rsS, so0, so);
        w1[i] = buf_ld_row<T>(rsS, so1, so);
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const double yc = yv[s0 + i];
        if (c0ok) t0 -= (double)w0[i] * yc;
        if (c1ok) t1 -= (double)w1[i] * yc;
      }
    }
    wave_lds_sync();
  }
  __syncthreads();  // every wave is done with its tile: the tiles hold the reduction now
  double* red = reinterpret_cast<double*>(&tile_all[0][0]);
  red[wv * kMaxDense + lane] = t0;
  red[wv * kMaxDense + lane + 64] = t1;
  __syncthreads();
  for (int j = threadIdx.x; j < nB; j += blockDim.x)
    part[(int64_t)blockIdx.x * kMaxDense + j] =
        ((red[j] + red[kMaxDense + j]) + red[2 * kMaxDense + j]) + red[3 * kMaxDense + j];
}

template <typename T>
hipError_t launch_refine_residual(const BatchView& bv, const T* A, const T* B, const int32_t* cam, const T* b,
                                  const double* d, const T* Rblk, const T* Sc, const double* p, double* y,
                                  double* part, hipStream_t st) {
  if (bv.max_L > kMaxDense) return hipErrorInvalidValue;
  switch (bv.n) {
#define QRK_P1(NN)                                                                                           \
  case NN:                                                                                                   \
    if (cam)                                                                                                 \
      hipLaunchKernelGGL((k_refine_pass1<T, NN, true>), dim3(bv.nwg), dim3(256), 0, st, bv.probs, bv.wg_prob, \
                         bv.pack_blk, bv.row_off, A, B, cam, b, d, bv.lam, Rblk, Sc, p, y, part);           \
    else                                                                                                     \
      hipLaunchKernelGGL((k_refine_pass1<T, NN, false>), dim3(bv.nwg), dim3(256), 0, st, bv.probs,           \
                         bv.wg_prob, bv.pack_blk, bv.row_off, A, B, cam, b, d, bv.lam, Rblk, Sc, p, y, part); \
    break;
    QRK_P1(1) QRK_P1(2) QRK_P1(3) QRK_P1(4) QRK_P1(5) QRK_P1(6) QRK_P1(7) QRK_P1(8)
#undef QRK_P1
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Refinement pass 2 (one workgroup per problem): g_B = sum of the problem's workgroup
// partials (fixed order) - lam d_B^2 p_B, then y_B = R_B^{-T} g_B and delta_B = R_B^{-1} y_B
// by one wave; p_B += delta_B.
// ADJ = false: refinement (delta_B -> delta[pi * kMaxDense ..]).
// ADJ = true : adjoint (rhs = g_B + sum of partials; the solution -> u_B in out, laid out
//              like p; p untouched).
// ---------------------------------------------------------------------------------
template <typename T, bool ADJ>
__global__ void __launch_bounds__(1024)
k_refine_dense(const ProbDesc* __restrict__ probs, int n, const double* __restrict__ part,
               const T* __restrict__ RBall, const double* __restrict__ dvec, const double* __restrict__ lamv,
               double* __restrict__ p, double* __restrict__ out, const double* __restrict__ gvec) {
  __shared__ float Rs[sizeof(T) == 4 ? kMaxDense * kMaxDense : 1];
  __shared__ double Rsd[sizeof(T) == 8 ? kMaxDense * kMaxDense : 1];
  __shared__ double acc[8][kMaxDense];
  const int pi = blockIdx.x;
  const ProbDesc& P = probs[pi];
  const int nB = P.nB, L = P.L;
  const int64_t off = P.noff + P.K * n;
  const double* pp = part + (int64_t)P.wg0 * kMaxDense;
  const int nparts = P.nwg;
  const int t = threadIdx.x;
  const int j = t & 127, q = t >> 7;
  // partials of group q: w = q, q + 8, ...; loaded 32 at a time so the loads overlap, then
  // added in order
  double s = 0.0;
  if (j < nB) {
    for (int w0 = q; w0 < nparts; w0 += 8 * 32) {
      double buf[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        const int w = w0 + 8 * u;
        buf[u] = w < nparts ? pp[(int64_t)w * kMaxDense + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 32; ++u) s += buf[u];
    }
  }
  acc[q][j] = s;
  stage_dense<T, 1024>(RBall + P.rboff, L, Rs, Rsd, t);
  __syncthreads();
  if (t >= 64) return;
  const int lane = t;
  const double lam = ADJ ? 0.0 : lamv[pi];
  double v0 = 0.0, v1 = 0.0;
  if (lane < nB) {
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) g += acc[k][lane];
    if (ADJ) {
      v0 = gvec[off + lane] + g;
    } else {
      const double dj = dvec[off + lane];
      v0 = g - lam * dj * dj * p[off + lane];
    }
  }
  if (lane + 64 < nB) {
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) g += acc[k][lane + 64];
    if (ADJ) {
      v1 = gvec[off + lane + 64] + g;
    } else {
      const double dj = dvec[off + lane + 64];
      v1 = g - lam * dj * dj * p[off + lane + 64];
    }
  }
  double dv0, dv1;
  dense_diag_inv<T>(Rs, Rsd, L, nB, lane, dv0, dv1);
  wave_fwd_T<T>(Rs, Rsd, L, nB, lane, dv0, dv1, v0, v1);
  wave_bwd<T>(Rs, Rsd, L, nB, lane, dv0, dv1, v0, v1);
  double* o = ADJ ? out + off : out + (int64_t)pi * kMaxDense;
  if (lane < nB) {
    o[lane] = v0;
    if (!ADJ) p[off + lane] += v0;
  }
  if (lane + 64 < nB) {
    o[lane + 64] = v1;
    if (!ADJ) p[off + lane + 64] += v1;
  }
}

template <typename T>
hipError_t launch_refine_dense(const BatchView& bv, const double* part, const T* RB, const double* dvec,
                               double* p, double* delta_B, hipStream_t st) {
  if (bv.max_L > kMaxDense) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_refine_dense<T, false>), dim3(bv.P), dim3(1024), 0, st, bv.probs, bv.n, part, RB, dvec,
                     bv.lam, p, delta_B, (const double*)nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_dense(const BatchView& bv, const double* part, const T* RB, const double* g, double* u,
                                hipStream_t st) {
  if (bv.max_L > kMaxDense) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_refine_dense<T, true>), dim3(bv.P), dim3(1024), 0, st, bv.probs, bv.n, part, RB,
                     (const double*)nullptr, bv.lam, (double*)nullptr, u, g);
  return hipGetLastError();
}

#define QRK_INST(T)                                                                                      \
  template hipError_t launch_backsub_dense<T>(const BatchView&, const T*, double*, int*, hipStream_t,      \
                                              const double*);                                            \
  template hipError_t launch_backsub_blocks<T>(const BatchView&, const T*, const T*, double*, int*,        \
                                               hipStream_t, const double*);                              \
  template hipError_t launch_refine_residual<T>(const BatchView&, const T*, const T*, const int32_t*,       \
                                                const T*, const double*, const T*, const T*, const double*, \
                                                double*, double*, hipStream_t);                          \
  template hipError_t launch_refine_dense<T>(const BatchView&, const double*, const T*, const double*,     \
                                             double*, double*, hipStream_t);                             \
  template hipError_t launch_refine_blocks<T>(const BatchView&, const T*, const T*, const double*,         \
                                              const double*, double*, hipStream_t);                      \
  template hipError_t launch_adjoint_blocks<T>(const BatchView&, const T*, const T*, const double*, double*, \
                                               hipStream_t);                                             \
  template hipError_t launch_adjoint_dense<T>(const BatchView&, const double*, const T*, const double*,     \
                                              double*, hipStream_t);
QRK_INST(float)
QRK_INST(double)
#undef QRK_INST

}  // namespace qrk
