// Per-block Householder QR with the block width n fixed at compile time (QRkit Sections 4.1
// and 4.2, damping rows of the Backtrack LM of Section 5.2 stacked under each block), for
// blocks with m_i >= n.  One wave64 per block.
//
// Register rows.  Rows 0 .. m_i-1 hold the block's data rows, rows RD .. RD+n-1 (RD = ROWS-n)
// its damping rows sqrt(lam) D_i (zero in the coupled columns), rows m_i .. RD-1 are padding.
// The padding rows are zero in the block's own columns, so every Householder vector is zero
// there: they take no part in the factorisation, and the result is that of [A_i; sqrt(lam) D_i]
// with its rows in their natural order.  Because m_i >= n, every pivot row k < n is a data row.
//
// Lanes.  Lane j < n owns column j of the block; every lane owns coupled columns lane and
// lane + 64 (column nB is b).  Reflector k is formed by lane k and reaches the other lanes by
// v_readlane into scalar registers; with z = (alpha - beta, a_{k+1}, ...) the unscaled vector
// and beta = -sign(alpha) ||a_{k..}||, the reflector maps a column c to
//     c - (z^T c) (-1 / beta) (1 / (alpha - beta)) z,
// which is LAPACK's I - tau v v^T with v = z / (alpha - beta), tau = (beta - alpha) / beta.
//
// Addressing.  The block index, its row offsets and every row pointer are wave-uniform
// (scalar registers); a lane adds only its fixed column offset, so loads and stores of a row
// need no vector address arithmetic.
#pragma once

#include "qrk_device.hpp"

namespace qrk {

template <typename T>
__device__ __forceinline__ T lane_value(T x, int k) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), k));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), k);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// A row of zeros that padding rows of the block's own columns are read from (64 bytes: the
// widest lane offset is (8 - 1) * sizeof(double)).
__device__ static const double kZeroRow[8] = {0, 0, 0, 0, 0, 0, 0, 0};

// Row pointers are pinned to scalar registers (an empty asm with an "s" operand), so an access
// is a scalar row base plus the lane's 32-bit column offset and the compiler does not fold the
// lane offset into a 64-bit vector address that every row then adds to.
#define QRK_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ const QRK_GLOBAL char* pin_uniform(const void* p) {
  const QRK_GLOBAL char* g = (const QRK_GLOBAL char*)p;
  asm("" : "+s"(g));
  return g;
}
__device__ __forceinline__ QRK_GLOBAL char* pin_uniform(void* p) {
  QRK_GLOBAL char* g = (QRK_GLOBAL char*)p;
  asm("" : "+s"(g));
  return g;
}

// element at byte offset off (a lane's column offset) of the row starting at base (uniform)
template <typename T>
__device__ __forceinline__ T ld_row(const T* base, uint32_t off) {
  return *reinterpret_cast<const QRK_GLOBAL T*>(pin_uniform(base) + off);
}
template <typename T>
__device__ __forceinline__ void st_row(T* base, uint32_t off, T v) {
  // the lane offset is re-pinned where the store is, so its zero extension is visible to the
  // store's address selection even when the store sits behind a branch
  asm("" : "+v"(off));
  *reinterpret_cast<QRK_GLOBAL T*>(pin_uniform(base) + off) = v;
}
// st_row for the reduced rows, the largest output: they are read once, by the dense part's
// leaves, and are stored streaming so they do not push A and B out of the last-level cache,
// from which the refinement pass that follows the solve reads them again
template <typename T>
__device__ __forceinline__ void st_row_stream(T* base, uint32_t off, T v) {
  asm("" : "+v"(off));
  __builtin_nontemporal_store(v, reinterpret_cast<QRK_GLOBAL T*>(pin_uniform(base) + off));
}

// Raw buffer access: the descriptor holds the (wave-uniform) base, the row offset goes in the
// scalar offset and the lane's column offset in the vector offset, so a row costs no vector
// address arithmetic whatever basic block it sits in.  Word 3 is the gfx9 raw-buffer format
// (32-bit data format, no swizzle, no stride); the record count only bounds the range check,
// and every offset used stays inside the rows the caller owns.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}

// A, B, bvec point at the block's first row (of A with row stride N, of B_p with row stride
// ldb, of b); d at its first damping entry; Rb at R_i (N x N), Scb at S_i | c_i (N x L),
// red at the block's first reduced row (row stride ldr).  Requires N <= m <= ROWS - N,
// nB + 1 <= 64 * SLOTS and (m - 1) * ldb * sizeof(T) < 2^31.  All scalar arguments are
// wave-uniform.
// qv: when non-null, the block's reflectors are stored (QKeep layout): qvd at the block's first
// data row (row stride N), qvp at its damping rows (N x N), qg its g_j (N).
// CAM: the coupled columns are cameras of ldb columns each (nB = ncam * ldb, nB > 0): B holds
// every row's ldb values, cam (at the block's first row) the camera of every row, and row r's
// values lie in columns cam[r] * ldb .. cam[r] * ldb + ldb - 1; a camera outside [0, ncam) is
// none (the row's coupled entries are zero).
template <typename T, int N, int ROWS, int SLOTS, bool CAM = false>
__device__ __forceinline__ void block_qr_wave_n(int nB, int m, int ldb, int ldr, const T* __restrict__ A,
                                                const T* __restrict__ B, const T* __restrict__ bvec,
                                                const double* __restrict__ d, double sqrt_lam, T* __restrict__ Rb,
                                                T* __restrict__ Scb, T* __restrict__ red, int lane,
                                                T* __restrict__ qvd = nullptr, T* __restrict__ qvp = nullptr,
                                                T* __restrict__ qg = nullptr,
                                                const int32_t* __restrict__ cam = nullptr) {
  static_assert(N >= 1 && N <= 8 && ROWS >= 2 * N, "block shape");
  constexpr int RD = ROWS - N;  // first damping row
  __builtin_assume(m >= N && m <= RD);
  const int L = nB + 1;
  const int mc = m - 1;         // last data row

  // block columns: data rows, padding rows read from the zero row, damping row RD + j of
  // column j
  T a[ROWS];
  {
    const uint32_t jo = (uint32_t)(lane < N ? lane : N - 1) * (uint32_t)sizeof(T);
    const T dl = (T)(sqrt_lam * d[lane < N ? lane : N - 1]);
    const T* zero = reinterpret_cast<const T*>(kZeroRow);
#pragma unroll
    for (int r = 0; r < RD; ++r) a[r] = ld_row(r < m ? A + r * N : zero, jo);
#pragma unroll
    for (int j = 0; j < N; ++j) a[RD + j] = lane == j ? dl : T(0);
  }
  // coupled columns: data rows (padding rows hold finite copies of row m-1, which the zero
  // Householder entries there keep out of every product), damping rows zero
  T c[SLOTS][ROWS];
  {
    // with nB == 0 no lane needs B: the loads then read b with unit stride
    const T* Bb = nB > 0 ? B : bvec;
    const int ldbe = nB > 0 ? ldb : 1;
    const __amdgpu_buffer_rsrc_t rsB = raw_rsrc(Bb);
    const uint32_t ncam = CAM ? (uint32_t)(nB / ldbe) : 0u;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int col = s * 64 + lane;
      const int cc = col < nB ? col : (nB > 0 ? nB - 1 : 0);
      const uint32_t co = (uint32_t)cc * (uint32_t)sizeof(T);
#pragma unroll
      for (int r = 0; r < RD; ++r) {
        const int rr = r < mc ? r : mc;
        if constexpr (CAM) {
          // the row's camera (wave-uniform): this lane's column within it, if any
          const int cr = cam[rr];
          const bool seen = (uint32_t)cr < ncam;
          const uint32_t k = (uint32_t)(cc - (seen ? cr : 0) * ldbe);
          const bool on = seen && col < nB && k < (uint32_t)ldbe;
          const T x = buf_ld<T>(rsB, (on ? k : 0u) * (uint32_t)sizeof(T), (uint32_t)(rr * ldbe) * (uint32_t)sizeof(T));
          c[s][r] = on ? x : T(0);
        } else {
          c[s][r] = buf_ld<T>(rsB, co, (uint32_t)(rr * ldbe) * (uint32_t)sizeof(T));
        }
      }
#pragma unroll
      for (int j = 0; j < N; ++j) c[s][RD + j] = T(0);
      // column nB is b: the lane holding it copies the (scalar-loaded) entries in
      if ((nB >> 6) == s && col == nB) {
#pragma unroll
        for (int r = 0; r < RD; ++r) c[s][r] = bvec[r < mc ? r : mc];
      }
    }
  }

  T zsave = T(0), gsave = T(0);  // lane k: z_k's pivot entry and g_k (for the stored Q)
#pragma unroll
  for (int k = 0; k < N; ++k) {
    // lane k's column: alpha = a_k, sigma = sum of squares below the pivot
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int r = k + 1; r < ROWS; ++r) {
      if ((r - k) & 1)
        s0 += a[r] * a[r];
      else
        s1 += a[r] * a[r];
    }
    const T sigma = s0 + s1;
    const T alpha = a[k];
    T beta = alpha, z0 = T(0), rbeta = T(0), rz = T(0);
    if constexpr (sizeof(T) == 4) {
      // hardware square root and reciprocals (1 ulp); a squared norm below the smallest
      // normal float would be flushed by them, so such a column takes the identity
      const T nrm2 = alpha * alpha + sigma;
      if (sigma != T(0) && nrm2 >= 0x1p-126f) {
        const T nrm = __builtin_amdgcn_sqrtf(nrm2);
        beta = alpha >= T(0) ? -nrm : nrm;
        z0 = alpha - beta;
        rbeta = -__builtin_amdgcn_rcpf(beta);
        rz = __builtin_amdgcn_rcpf(z0);
      }
    } else {
      if (sigma != T(0)) {
        const T nrm = sqrt(alpha * alpha + sigma);
        beta = alpha >= T(0) ? -nrm : nrm;
        z0 = alpha - beta;
        rbeta = T(-1) / beta;
        rz = T(1) / z0;
      }
    }
    // reflector of lane k to every lane
    const T zk = lane_value(z0, k);
    const T g = lane_value(rbeta, k) * lane_value(rz, k);  // 0: identity
    T zr[ROWS];
#pragma unroll
    for (int r = k + 1; r < ROWS; ++r) zr[r] = lane_value(a[r], k);

    auto apply = [&](T* col, bool skip) {
      T u0 = zk * col[k], u1 = T(0);
#pragma unroll
      for (int r = k + 1; r < ROWS; ++r) {
        if ((r - k) & 1)
          u1 += zr[r] * col[r];
        else
          u0 += zr[r] * col[r];
      }
      const T t = skip ? T(0) : -(u0 + u1) * g;  // col <- col - g (z^T col) z
      col[k] += t * zk;
#pragma unroll
      for (int r = k + 1; r < ROWS; ++r) col[r] += t * zr[r];
    };
    // columns right of k (lanes > k); the finished columns (lanes <= k) are left alone, so that
    // lane j keeps its reflector's entries below row j (R's entries there are not used)
    if (k + 1 < N) apply(a, lane <= k);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) apply(c[s], false);
    if (lane == k) {
      zsave = z0;
      gsave = g;
    }
    a[k] = lane == k ? beta : a[k];
  }
  // the reflectors: lane j < N writes z_j (data rows, damping rows) and g_j
  if (qvd != nullptr && lane < N) {
    const uint32_t jo = (uint32_t)lane * (uint32_t)sizeof(T);
    int ms = m;
    asm("" : "+s"(ms));
#pragma unroll
    for (int r = 0; r < RD; ++r)
      if (r < ms) st_row(qvd + r * N, jo, r > lane ? a[r] : (r == lane ? zsave : T(0)));
#pragma unroll
    for (int t = 0; t < N; ++t) st_row(qvp + t * N, jo, a[RD + t]);
    qg[lane] = gsave;
  }

  // R_i: lane j < N holds column j (rows above the diagonal and the diagonal)
  if (lane < N) {
#pragma unroll
    for (int r = 0; r < N; ++r) Rb[r * N + lane] = r <= lane ? a[r] : T(0);
  }
  // coupling rows S_i | c_i (rows 0 .. N-1), reduced rows: data rows N .. m-1, then the
  // damping rows
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int col = s * 64 + lane;
    if (col < L) {
      const uint32_t co = (uint32_t)col * (uint32_t)sizeof(T);
#pragma unroll
      for (int r = 0; r < N; ++r) st_row(Scb + r * L, co, c[s][r]);
      // the row count is re-pinned so these tests are not shared with the loads' (which
      // would keep one lane mask per row alive across the whole factorisation)
      int ms = m;
      asm("" : "+s"(ms));
#pragma unroll
      for (int r = N; r < RD; ++r)
        if (r < ms) st_row_stream(red + (int64_t)(r - N) * ldr, co, c[s][r]);
#pragma unroll
      for (int j = 0; j < N; ++j) st_row_stream(red + (int64_t)(m - N + j) * ldr, co, c[s][RD + j]);
    }
  }
}

}  // namespace qrk
