// Tall-skinny QR of the reduced dense rows on the gfx950 matrix cores (float32).
//
// What is computed (QRkit Section 4.2): the triangle R' of qr(Q_1^perp^T A_2), i.e. of
// all reduced rows of the block-angular step stacked with the damping rows
// sqrt(lam) D_B, with the right-hand side carried as the last column.
//
// Organisation (communication-avoiding tall-skinny QR, for a batch of problems with the
// same number of 16-column blocks at once):
//   * every wave is a leaf of one problem: it streams a contiguous range of that problem's
//     rows, a tile of 16*NRB rows at a time, into its own running upper triangle R (a flat
//     tree inside the wave);
//   * the leaf triangles of each problem are then merged pairwise, QR([R_left; R_right]),
//     in the same launch: the second wave of a pair to finish performs the merge (arrival
//     counted with a device-scope atomic), so no wave ever waits for another, and the trees
//     of different problems proceed independently;
//   * each problem's root is written out row-major (L x L).
//
// Merging a tile X into R uses blocked Householder with the compact WY form (paper
// Section 2, compressed WY: Q = I - V T V^T; the paper writes I + Y T Y^T, the sign of
// T differs), panels of 16 columns:
//   panel   for each column j: reflector [1; w_j] acting on R's row j and the tile (the
//           zeros of R below its diagonal are never touched), applied to the rest of the
//           panel; the Gram entries w_k^T w_j come out of the same reductions and
//           T[0:j, j] = -tau_j T[0:j, 0:j] (W[:, 0:j]^T w_j), T_jj = tau_j, is built
//           alongside;
//   update  Z = R[panel rows, trail] + W^T X_trail;  Z' = T^T Z;
//           R[panel rows, trail] -= Z';  X_trail -= W Z'        (MFMA f32 16x16x4).
//
// Register layout: a 16x16 block M is one float4 per lane in the matrix-core
// accumulator layout: lane l, component v holds M[4*(l>>4) + v][l & 15].  With that
// layout the tile blocks are directly the operands of W^T X and T is directly the A
// operand of T^T Z; only W and T are re-laid out through LDS, once per panel.
#pragma once

#include <type_traits>

#include "qrk_batch.hpp"
#include "qrk_device.hpp"

namespace qrk {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float f_of(unsigned u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ unsigned u_of(float x) { return __builtin_bit_cast(unsigned, x); }

// A copy of x that the compiler cannot identify with x (an empty asm on a register;
// no memory is touched).  The permlane swaps need two distinct operands.
__device__ __forceinline__ unsigned opaque_copy(unsigned x) {
  unsigned y = x;
  asm volatile("" : "+v"(y));
  return y;
}

// Sum over the four 16-lane rows of the wave (lanes l, l^16, l^32, l^48), in every lane.
// permlane16_swap exchanges the odd rows of its first operand with the even rows of
// the second, permlane32_swap the upper half of the first with the lower half of the
// second; with both operands equal to x, the two results add up to x[l] + x[l^16]
// (resp. x[l^32]).  IEEE addition is commutative, so all lanes get the same bits.
__device__ __forceinline__ float sum_rows4(float x) {
  auto a = __builtin_amdgcn_permlane16_swap(u_of(x), opaque_copy(u_of(x)), false, false);
  x = f_of(a[0]) + f_of(a[1]);
  auto b = __builtin_amdgcn_permlane32_swap(u_of(x), opaque_copy(u_of(x)), false, false);
  return f_of(b[0]) + f_of(b[1]);
}

// Broadcast lane J of every 16-lane row to the whole row.
template <int J>
__device__ __forceinline__ float row_bcast(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x150 + J,
                                                            0xF, 0xF, false));
}

// Fused forms of acc += row_bcast<J>(x) * y: the broadcast is the DPP modifier of the FMA
// itself (v_fmac_f32 with row_newbcast on its first source), one instruction instead of a DPP
// move and an FMA.  Each group starts with s_nop 1: a DPP source must not have been written by
// the VALU in the two preceding cycles, and the compiler does not track that hazard across an
// asm statement.  Inside a group no instruction reads, through DPP, a register that an earlier
// instruction of the group wrote.
// Gram terms of one 4-row block: pr0 += b(x0) x0 + b(x2) x2, pr1 += b(x1) x1 + b(x3) x3.
template <int J>
__device__ __forceinline__ void gram4_bcast(float& pr0, float& pr1, const f4& x) {
  asm(
      "s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %2, %2 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %1, %3, %3 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %0, %4, %4 row_newbcast:%6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %1, %5, %5 row_newbcast:%6 row_mask:0xf bank_mask:0xf"
      : "+v"(pr0), "+v"(pr1)
      : "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "n"(J));
}
// x_v += b(x_v) * f for the four components of one 4-row block.
template <int J>
__device__ __forceinline__ void axpy4_bcast(f4& x, float f) {
  float x0 = x[0], x1 = x[1], x2 = x[2], x3 = x[3];
  asm(
      "s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %0, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %1, %1, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %2, %2, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %3, %3, %4 row_newbcast:%5 row_mask:0xf bank_mask:0xf"
      : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3)
      : "v"(f), "n"(J));
  x = f4{x0, x1, x2, x3};
}

__device__ __forceinline__ float read_lane(float x, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
}

// Lane (g, c) receives lane (G, c)'s x: row G of the wave copied to all four rows (a
// cross-lane fetch through the LDS crossbar, no LDS storage; every lane must be active).
template <int G>
__device__ __forceinline__ float rows_from(float x, int c) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute((G * 16 + c) * 4, __builtin_bit_cast(int, x)));
}

// Householder factorisation of one 16-column panel [Rd; X[0..RBN-1]] (paper Section 2: one
// reflector per column, the compact-WY factor T built alongside).  Rd is the 16x16 diagonal
// block of the triangle, X the panel's tile blocks, both in the accumulator layout; lane
// (g, c) owns column c.  Step j:
//   G_c   = x_j^T x_c over the tile rows (one pass, all columns; G_j = sigma_j = ||x_j||^2)
//   beta  = -sign(alpha) sqrt(alpha^2 + sigma), alpha = R[j][j]; tau = (beta - alpha) / beta;
//           the reflector is [1; s_j x_j] with s_j = 1 / (alpha - beta) (the tile column stays
//           unscaled in place)
//   pd_c  = R[j][c] + s_j G_c   (= [e_j; w_j]^T [R[:, c]; x_c])
//   R[j][c] -= tau pd_c, x_c -= x_j s_j tau pd_c   (c > j);  R[j][j] = beta
//   T[0:j, j] = -tau T[0:j, 0:j] (W[:, 0:j]^T w_j), T[j][j] = tau, with w_k^T w_j = s_k s_j G_k.
// sigma below the smallest normal float counts as zero (identity reflector).  A leaf that
// starts from a zero triangle reflects the roundoff left in the columns beyond the rank of its
// first tiles; that residue shrinks by about eps per tile height and can reach the subnormal
// range, where the hardware square root returns 0 and the scale would be infinite.  Selects,
// not branches, for the reflector itself: the panel stays one straight-line block the scheduler
// can interleave with the matrix-core updates around it.
// On return lane (g, c) holds row c of T in trow and s_c in sc.
// FUSE selects the fused broadcast-FMA groups from a panel's second column on (faster for the
// two-block tiles of the banded kernel; the dense-part leaves and tree measured a little slower
// with them and keep the compiler's DPP moves).
template <int RBN, bool FUSE = false>
__device__ __forceinline__ void panel_factor(f4& Rd, f4 (&X)[RBN], float (&trow)[16], float& sc, int lane) {
  const int g = lane >> 4;
  const int c = lane & 15;
  sc = 0.f;
  static_for<0, 16>([&](auto JJ) {
    constexpr int j = decltype(JJ)::value;
    // R's row j in every row of the wave; the steps before j leave that row unchanged
    const float rrow = rows_from<(j >> 2)>(Rd[j & 3], c);
    // Column 0 of the panel reads tile values that the matrix cores may have just written (the
    // previous panel's trailing update); that read goes through compiler-generated code, which
    // keeps the matrix-core result hazard.  From column 1 on every tile value was last written
    // by column j-1's update on the VALU, which the fused groups' s_nop covers.
    float pr0 = 0.f, pr1 = 0.f;
    if constexpr (j == 0 || !FUSE) {
#pragma unroll
      for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (v & 1)
            pr1 += row_bcast<j>(X[rb][v]) * X[rb][v];
          else
            pr0 += row_bcast<j>(X[rb][v]) * X[rb][v];
        }
    } else {
#pragma unroll
      for (int rb = 0; rb < RBN; ++rb) gram4_bcast<j>(pr0, pr1, X[rb]);
    }
    const float gram = sum_rows4(pr0 + pr1);  // x_j^T x_c
    const float sigma = row_bcast<j>(gram);
    const float alpha = read_lane(Rd[j & 3], (j >> 2) * 16 + j);
    const bool refl = sigma >= 0x1p-126f;
    const float nrm = __builtin_amdgcn_sqrtf(alpha * alpha + sigma);
    const float bneg = alpha >= 0.f ? -nrm : nrm;
    const float beta = refl ? bneg : alpha;
    const float tau = refl ? (bneg - alpha) * __builtin_amdgcn_rcpf(bneg) : 0.f;
    const float scale = refl ? __builtin_amdgcn_rcpf(alpha - bneg) : 0.f;
    const float pd = gram * scale + rrow;  // R[j][c] + w_j^T x_c
    const float s = tau * pd;
    const float nf = (c > j) ? -scale * s : 0.f;
    if constexpr (j == 0 || !FUSE) {
#pragma unroll
      for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) X[rb][v] += row_bcast<j>(X[rb][v]) * nf;
    } else {
#pragma unroll
      for (int rb = 0; rb < RBN; ++rb) axpy4_bcast<j>(X[rb], nf);
    }
    if (g == (j >> 2)) Rd[j & 3] = (c > j) ? Rd[j & 3] - s : (c == j ? beta : Rd[j & 3]);
    const float gk = sc * pd;  // at lane k < j: s_k s_j x_j^T x_k = w_k^T w_j
    float t = 0.f;
    static_for<0, j>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      t += trow[k] * row_bcast<k>(gk);
    });
    trow[j] = (c < j) ? -tau * t : (c == j ? tau : 0.f);
    if (c == j) sc = scale;
  });
}

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// bf16 operands of the 16x16x32 matrix-core product: lane l supplies A[l%16][8(l/16) + e] and
// B[8(l/16) + e][l%16], e = 0..7.  Any fixed assignment of a lane's eight K slots to tile rows
// (or panel columns) gives the same sum as long as A and B use the same one.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma_bf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// BF16x3 split of eight floats: hi = bf16(x), lo = bf16(x - hi) (round to nearest even).
struct BfPair {
  bf8 hi, lo;
};
__device__ __forceinline__ BfPair bf_split(const float (&x)[8]) {
  BfPair r;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    r.hi[e] = h;
    r.lo[e] = (__bf16)(x[e] - (float)h);
  }
  return r;
}

constexpr int kWaveLds = 256 + 256 + 256 * 8;  // T staging, scales, W staging (up to 8 blocks)

// The kept panels of a merge of two triangles (per-wave LDS in the merge tree, and the stored Q
// of a merge node), in the node_panel_off layout of qrk_batch.hpp.
template <int NCB>
struct TreeKeep {
  static constexpr int off(int p) { return (int)node_panel_off(p); }
  static constexpr int total = off(NCB);
};

template <int NCB>
struct Tri {
  static constexpr int count = NCB * (NCB + 1) / 2;
  static constexpr int idx(int p, int q) { return p * NCB - (p * (p - 1)) / 2 + (q - p); }
};

// A running triangle whose block rows from RL on live in the wave's LDS (block t at
// rl + (t - first) * 256, lane-major like a stored triangle) while its first RL block rows stay
// in registers; RL = NCB keeps all of it in registers.  A panel reads and writes only its own
// block row, so the LDS rows cost one load and one store per block and panel.
template <int NCB, int RL>
struct TriSplit {
  static constexpr int first = Tri<NCB>::idx(RL, RL);  // first block kept in LDS (count if none)
  static constexpr int lds_blocks = Tri<NCB>::count - first;
};

template <int NCB, int RL, int P, int Q>
__device__ __forceinline__ f4 tri_get(const f4 (&R)[Tri<NCB>::count], const float* rl, int lane) {
  constexpr int t = Tri<NCB>::idx(P, Q);
  if constexpr (P < RL)
    return R[t];
  else
    return *reinterpret_cast<const f4*>(rl + (t - TriSplit<NCB, RL>::first) * 256 + lane * 4);
}

template <int NCB, int RL, int P, int Q>
__device__ __forceinline__ void tri_put(f4 (&R)[Tri<NCB>::count], float* rl, int lane, const f4& v) {
  constexpr int t = Tri<NCB>::idx(P, Q);
  if constexpr (P < RL)
    R[t] = v;
  else
    *reinterpret_cast<f4*>(rl + (t - TriSplit<NCB, RL>::first) * 256 + lane * 4) = v;
}

// Merge the tile X (NRB block rows) into the running triangle R.
//   TRI = false: a dense tile of 16*NRB rows; panels before pstart are skipped (their
//                tile columns are known to be zero).
//   TRI = true : the tile is an upper-triangular NCB x NCB block triangle (NRB == NCB);
//                in panel P only block rows 0..P are nonzero, which is used at compile
//                time.
// The Householder vectors are kept unscaled: the tile column x_j stays in place and the
// reflector's tile part is w_j = s_j x_j with s_j = 1/(alpha_j - beta_j); the scales are
// applied once per row of the small Z products instead of once per tile element.
// Only the first NPANEL panels are factored; their reflectors are still applied to every
// column block (the later blocks then hold columns that are carried, not factored).
// KEEPQ: the panels' compact-WY factors (T, the scales and the raw reflector blocks,
// qrk_batch.hpp) are stored at qkeep for a later Q^T: panel P at P * tile_panel_floats for a
// dense tile, at TreeKeep<NCB>::off(P) for a triangle.
// RL < NCB: R's block rows from RL on are in LDS at rl (TriSplit).
template <int NCB, int NRB, bool TRI, bool BF = false, int NPANEL = NCB, bool FUSE = false, bool KEEPQ = false,
          int RL = NCB>
__device__ __forceinline__ void merge_tile(f4 (&R)[Tri<NCB>::count], f4 (&X)[NRB][NCB], int pstart,
                                           float* __restrict__ lds, int lane, float* __restrict__ qkeep = nullptr,
                                           float* __restrict__ rl = nullptr) {
  const int g = lane >> 4;
  const int c = lane & 15;
  float* Tl = lds;            // [16][16]
  float* Sl = lds + 256;      // [16] column scales
  float* Wl = lds + 512;      // [NRB][16][16]

  static_for<0, NCB>([&](auto PP) {
    constexpr int P = decltype(PP)::value;
    constexpr int rp = Tri<NCB>::idx(P, P);
    constexpr int RBN = TRI ? (P + 1 < NRB ? P + 1 : NRB) : NRB;  // active block rows
    if (!TRI && P < pstart) return;
    if constexpr (P >= NPANEL) return;

    // ---- panel factorisation of [R[P][P]; X[:, P]] (and T alongside) -------------------
    float trow[16];  // lane (g, c) builds row c of T
    float sc;        // scale of this lane's column
    {
      f4 Xp[RBN];
#pragma unroll
      for (int rb = 0; rb < RBN; ++rb) Xp[rb] = X[rb][P];
      if constexpr (RL == NCB) {
        panel_factor<RBN, FUSE>(R[rp], Xp, trow, sc, lane);
      } else {
        f4 Rd = tri_get<NCB, RL, P, P>(R, rl, lane);
        panel_factor<RBN, FUSE>(Rd, Xp, trow, sc, lane);
        tri_put<NCB, RL, P, P>(R, rl, lane, Rd);
      }
#pragma unroll
      for (int rb = 0; rb < RBN; ++rb) X[rb][P] = Xp[rb];
    }

    // ---- re-lay out T (rows -> accumulator layout), scales and W^T through LDS ------------
    if (g == 0) {
#pragma unroll
      for (int k = 0; k < 16; k += 4)
        *reinterpret_cast<f4*>(Tl + c * 16 + k) = f4{trow[k], trow[k + 1], trow[k + 2], trow[k + 3]};
      Sl[c] = sc;
    }
#pragma unroll
    for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) Wl[rb * 256 + (4 * g + v) * 16 + c] = X[rb][P][v];
    wave_lds_sync();
    if constexpr (KEEPQ) {
      // T, the scales and W of this panel, from the registers they are staged from: lane (0, c)
      // holds row c of T (trow) and scale c, lane (g, c) the entries 4g .. 4g+3 of W's column c
      // in each block
      float* qp = qkeep + (TRI ? (int64_t)TreeKeep<NCB>::off(P) : P * tile_panel_floats(NRB));
      if (g == 0) {
#pragma unroll
        for (int k = 0; k < 16; k += 4)
          *reinterpret_cast<f4*>(qp + c * 16 + k) = f4{trow[k], trow[k + 1], trow[k + 2], trow[k + 3]};
        qp[256 + c] = sc;
      }
#pragma unroll
      for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) qp[320 + rb * 256 + (4 * g + v) * 16 + c] = X[rb][P][v];
    }
    f4 Td;
#pragma unroll
    for (int v = 0; v < 4; ++v) Td[v] = Tl[(4 * g + v) * 16 + c];
    const f4 srow = *reinterpret_cast<const f4*>(Sl + 4 * g);  // scales of rows 4g .. 4g+3
    float Wt[RBN][4];  // -x[rb*16 + c][4g + v]  (raw tile columns, transposed)
#pragma unroll
    for (int rb = 0; rb < RBN; ++rb) {
      const f4 w4 = *reinterpret_cast<const f4*>(Wl + rb * 256 + c * 16 + 4 * g);
#pragma unroll
      for (int v = 0; v < 4; ++v) Wt[rb][v] = -w4[v];
    }
    wave_lds_sync();

    // ---- trailing update on the matrix cores ----------------------------------------------
    //   Z = R_rows + diag(s) X_P^T X_q;  Z' = T^T Z;  R_rows -= Z';  X_q -= X_P diag(s) Z'
    // BF: X_P^T X_q and X_P (s Z') as three bf16 products each (hi hi' + hi lo' + lo hi'),
    // fp32 accumulation.  For X_P^T X_q, chunk h covers block rows 2h and 2h+1: lane (g, c)
    // gives K slots 8g + v and 8g + 4 + v the tile rows 16(2h) + 4g + v and 16(2h+1) + 4g + v of
    // column c (the panel's for A, column block q's for B).  For X_P (s Z') the K slots 8g + v
    // are panel columns 4g + v and the slots 8g + 4 .. 8g + 7 are zero.
    constexpr int NCH = (RBN + 1) / 2;
    BfPair Pbf[BF ? NCH : 1];
    BfPair Wbf[BF ? RBN : 1];
    if constexpr (BF) {
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        float t[8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          t[v] = X[2 * h][P][v];
          t[4 + v] = (2 * h + 1 < RBN) ? X[2 * h + 1 < RBN ? 2 * h + 1 : 0][P][v] : 0.f;
        }
        Pbf[h] = bf_split(t);
      }
#pragma unroll
      for (int rb = 0; rb < RBN; ++rb) {
        float t[8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          t[v] = Wt[rb][v];
          t[4 + v] = 0.f;
        }
        Wbf[rb] = bf_split(t);
      }
    }
    static_for<P + 1, NCB>([&](auto QQ) {
      constexpr int q = decltype(QQ)::value;
      constexpr int rq = Tri<NCB>::idx(P, q);
      f4 Y0 = {0.f, 0.f, 0.f, 0.f}, Y1 = {0.f, 0.f, 0.f, 0.f};
      if constexpr (BF) {
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
          float t[8];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            t[v] = X[2 * h][q][v];
            t[4 + v] = (2 * h + 1 < RBN) ? X[2 * h + 1 < RBN ? 2 * h + 1 : 0][q][v] : 0.f;
          }
          const BfPair qb = bf_split(t);
          Y0 = mfma_bf(Pbf[h].hi, qb.hi, Y0);
          Y1 = mfma_bf(Pbf[h].hi, qb.lo, Y1);
          Y1 = mfma_bf(Pbf[h].lo, qb.hi, Y1);
        }
      } else {
#pragma unroll
        for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if ((rb * 4 + v) & 1)
              Y1 = mfma4(X[rb][P][v], X[rb][q][v], Y1);
            else
              Y0 = mfma4(X[rb][P][v], X[rb][q][v], Y0);
          }
      }
      f4 Rq;
      if constexpr (RL == NCB)
        Rq = R[rq];
      else
        Rq = tri_get<NCB, RL, P, q>(R, rl, lane);
      const f4 Z = Rq + srow * (Y0 + Y1);
      f4 Zp = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) Zp = mfma4(Td[v], Z[v], Zp);
      if constexpr (RL == NCB)
        R[rq] -= Zp;
      else
        tri_put<NCB, RL, P, q>(R, rl, lane, Rq - Zp);
      const f4 Zs = srow * Zp;
      if constexpr (BF) {
        float t[8];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          t[v] = Zs[v];
          t[4 + v] = 0.f;
        }
        const BfPair zb = bf_split(t);
#pragma unroll
        for (int rb = 0; rb < RBN; ++rb) {
          X[rb][q] = mfma_bf(Wbf[rb].hi, zb.hi, X[rb][q]);
          X[rb][q] = mfma_bf(Wbf[rb].hi, zb.lo, X[rb][q]);
          X[rb][q] = mfma_bf(Wbf[rb].lo, zb.hi, X[rb][q]);
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int rb = 0; rb < RBN; ++rb) X[rb][q] = mfma4(Wt[rb][v], Zs[v], X[rb][q]);
      }
    });
  });
}

// A stored triangle is its NCB(NCB+1)/2 blocks, 1 KiB each, lane-contiguous.
// RL < NCB: the blocks from TriSplit<NCB, RL>::first on are read from / written to the LDS rows.
template <int NCB, int RL = NCB>
__device__ __forceinline__ void store_tri(float* __restrict__ dst, const f4 (&R)[Tri<NCB>::count],
                                          int lane, const float* __restrict__ rl = nullptr) {
  constexpr int first = TriSplit<NCB, RL>::first;
#pragma unroll
  for (int t = 0; t < Tri<NCB>::count; ++t)
    *reinterpret_cast<f4*>(dst + t * 256 + lane * 4) =
        t < first ? R[t] : *reinterpret_cast<const f4*>(rl + (t - first) * 256 + lane * 4);
}

template <int NCB, int RL = NCB>
__device__ __forceinline__ void load_tri(const float* __restrict__ src, f4 (&R)[Tri<NCB>::count],
                                         int lane, float* __restrict__ rl = nullptr) {
  constexpr int first = TriSplit<NCB, RL>::first;
#pragma unroll
  for (int t = 0; t < Tri<NCB>::count; ++t) {
    const f4 v = __builtin_nontemporal_load(reinterpret_cast<const f4*>(src + t * 256 + lane * 4));
    if (t < first)
      R[t] = v;
    else
      *reinterpret_cast<f4*>(rl + (t - first) * 256 + lane * 4) = v;
  }
}

// R <- triangle of QR([R; stored triangle at src]).
template <int NCB, bool BF = false, bool KEEPQ = false, int RL = NCB>
__device__ __forceinline__ void merge_stored_tri(f4 (&R)[Tri<NCB>::count], const float* __restrict__ src,
                                                 float* lds, int lane, float* __restrict__ qkeep = nullptr,
                                                 float* __restrict__ rl = nullptr) {
  f4 X[NCB][NCB];
  static_for<0, NCB>([&](auto RB) {
    constexpr int rb = decltype(RB)::value;
    static_for<0, NCB>([&](auto QQ) {
      constexpr int q = decltype(QQ)::value;
      if constexpr (q >= rb)
        X[rb][q] = __builtin_nontemporal_load(
            reinterpret_cast<const f4*>(src + Tri<NCB>::idx(rb, q) * 256 + lane * 4));
      else
        X[rb][q] = f4{0.f, 0.f, 0.f, 0.f};
    });
  });
  merge_tile<NCB, NCB, true, BF, NCB, false, KEEPQ, RL>(R, X, 0, lds, lane, qkeep, rl);
}

// One leaf of the dense part, by one wave: leaf li of problem p streams rows
// [li * rows_per_leaf, ...) of the problem's reduced rows into its triangle (leaf 0 starts from
// diag(sqrt(lam_p) d_B)); the leaves of each problem are then merged pairwise (the problem's own
// slots and arrival counters: the second wave of a pair to finish merges) and the root is
// written row-major to the problem's R_B | c_B.
// KEEP (the stored Q): the panels of the leaf's tiles go to qs.qt (at the problem's qt0, qtiles
// tiles per leaf) and those of its merges to qs.qn (at qn0, one TreeKeep per merge node, numbered
// level by level from the leaves up as the separate merge tree numbers its nodes).  A separate
// instantiation, so that the kernels without it are compiled as if it did not exist.
// RL < NCB: the running triangle's block rows from RL on are kept in the wave's LDS at rl
// (TriSplit) instead of registers.
template <int NCB, int NRB, bool BF, bool KEEP = false, int RL = NCB>
__device__ __forceinline__ void tsqr_leaf(int pi, int leaf, const ProbDesc* __restrict__ probs, int n,
                                          const float* __restrict__ Red, const double* __restrict__ d,
                                          const double* __restrict__ lamv, float* __restrict__ slots,
                                          int* __restrict__ counters, float* __restrict__ RBall, float* lds,
                                          int lane, const QStore qs = QStore(), float* __restrict__ rl = nullptr) {
  static_assert(!KEEP || RL == NCB, "the stored Q's leaves keep the triangle in registers");
  const ProbDesc& P = probs[pi];
  const float* Xg = Red + P.redoff;
  const int64_t ldx = P.ldr;
  const int64_t nrows = P.M;
  const int L = P.L;
  const int nleaves = P.leaves;
  const int64_t rows_per_leaf = P.rows_per_leaf;
  const int g = lane >> 4;
  const int c = lane & 15;
  constexpr int NT = Tri<NCB>::count;
  constexpr int SLOT = NT * 256;
  constexpr int KT = 16 * NRB;

  f4 R[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) R[t] = f4{0.f, 0.f, 0.f, 0.f};
  if (leaf == 0) {
    const double* dB = d + P.noff + P.K * n;
    const double sqrt_lam = sqrt(lamv[pi]);
    static_for<0, NCB>([&](auto PP) {
      constexpr int Q = decltype(PP)::value;
      const int col = 16 * Q + c;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (4 * g + v == c && col < L - 1) R[Tri<NCB>::idx(Q, Q)][v] = (float)(sqrt_lam * dB[col]);
    });
  }
  if constexpr (RL < NCB) {  // the rows kept in LDS start from the values just set
#pragma unroll
    for (int t = TriSplit<NCB, RL>::first; t < Tri<NCB>::count; ++t)
      *reinterpret_cast<f4*>(rl + (t - TriSplit<NCB, RL>::first) * 256 + lane * 4) = R[t];
  }

  // ---- leaf: stream this wave's rows -------------------------------------------------------
  const int64_t r0 = (int64_t)leaf * rows_per_leaf;
  const int64_t r1 = r0 + rows_per_leaf < nrows ? r0 + rows_per_leaf : nrows;
  for (int64_t t = r0; t < r1; t += KT) {
    f4 X[NRB][NCB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int q = 0; q < NCB; ++q) {
        const int col = 16 * q + c;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = t + rb * 16 + 4 * g + v;
          // read once: streaming, so the reduced rows do not displace A and B in the last-level
          // cache, where the next block QR and refinement pass find them
          X[rb][q][v] = (row < r1 && col < L) ? __builtin_nontemporal_load(Xg + row * ldx + col) : 0.f;
        }
      }
    if constexpr (KEEP) {
      const int64_t tile = (t - r0) / KT;
      float* qk = qs.qt + qs.qo[pi].qt0 + ((int64_t)leaf * qs.qo[pi].qtiles + tile) * (NCB * tile_panel_floats(NRB));
      merge_tile<NCB, NRB, false, BF, NCB, false, true>(R, X, 0, lds, lane, qk);
    } else {
      merge_tile<NCB, NRB, false, BF, NCB, false, false, RL>(R, X, 0, lds, lane, nullptr, rl);
    }
  }

  // ---- pairwise merges up the problem's tree, in the same launch ----------------------------
  float* pslots = slots + P.slot0;
  if (P.tree_sep && nleaves > 1) {  // the merges are a separate, pipelined launch
    store_tri<NCB, RL>(pslots + (int64_t)leaf * SLOT, R, lane, rl);
    return;
  }
  int* pctr = counters + P.ctr0;
  int nl = nleaves;
  int slot = leaf;
  int64_t base = 0;   // first slot of the current level
  int64_t cbase = 0;  // first counter of the current level
  int64_t mbase = 0;  // merges of the levels below (the stored Q's node numbering)
  while (nl > 1) {
    const int sib = slot ^ 1;
    const int parent = slot >> 1;
    const int nn = (nl + 1) >> 1;
    if (sib >= nl) {  // no sibling at this level: carry the triangle up unchanged
      base += nl;
      cbase += nn;
      if constexpr (KEEP) mbase += nl >> 1;
      slot = parent;
      nl = nn;
      continue;
    }
    store_tri<NCB, RL>(pslots + (base + slot) * SLOT, R, lane, rl);
    __threadfence();
    int old = 0;
    if (lane == 0) old = atomicAdd(&pctr[cbase + parent], 1);
    old = __builtin_amdgcn_readfirstlane(old);
    if (old == 0) return;  // the sibling is still running; it will merge
    __threadfence();
    const int left = slot & ~1;
    load_tri<NCB, RL>(pslots + (base + left) * SLOT, R, lane, rl);
    if constexpr (KEEP)
      merge_stored_tri<NCB, BF, true>(R, pslots + (base + left + 1) * SLOT, lds, lane,
                                      qs.qn + qs.qo[pi].qn0 + (mbase + parent) * TreeKeep<NCB>::total);
    else
      merge_stored_tri<NCB, BF, false, RL>(R, pslots + (base + left + 1) * SLOT, lds, lane, nullptr, rl);
    base += nl;
    cbase += nn;
    if constexpr (KEEP) mbase += nl >> 1;
    slot = parent;
    nl = nn;
  }

  // ---- root: row-major L x L ----------------------------------------------------------------
  float* Rout = RBall + P.rboff;
  static_for<0, NCB>([&](auto PP) {
    constexpr int Q = decltype(PP)::value;
    static_for<0, NCB>([&](auto QQ) {
      constexpr int q = decltype(QQ)::value;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * Q + 4 * g + v;
        const int col = 16 * q + c;
        float val = 0.f;
        if constexpr (q >= Q) val = (col >= row) ? tri_get<NCB, RL, Q, q>(R, rl, lane)[v] : 0.f;
        if (row < L && col < L) Rout[(int64_t)row * L + col] = val;
      }
    });
  });
}

// Block rows of the running triangle the plain leaf keeps in registers (the rest in LDS): all
// up to 5 column blocks; at 6 the first (15 blocks in LDS free the registers of its 128-row
// tiles: 64-row tiles with three rows in registers measured 9% slower on the scale workload); at
// 7 none and at 8 the first (28 blocks in LDS either way).
constexpr int leaf_lds_rows(int ncb) { return ncb <= 5 ? ncb : (ncb == 6 ? 1 : (ncb == 7 ? 0 : 1)); }

// One launch per column-block count NCB: wave w is global leaf leaf_begin + w.  The launch
// that stores Q is a kernel of its own with one more argument; the one without it keeps the
// argument list it had before Q could be stored.
template <int NCB, int NRB, bool BF>
__global__ void __launch_bounds__(256)
k_tsqr_mfma(int leaf_begin, int nleaves_cls, const int32_t* __restrict__ leaf_prob,
            const int32_t* __restrict__ leaf_idx, const ProbDesc* __restrict__ probs, int n,
            const float* __restrict__ Red, const double* __restrict__ d, const double* __restrict__ lamv,
            float* __restrict__ slots, int* __restrict__ counters, float* __restrict__ RBall) {
  __shared__ float lds_all[4][kWaveLds];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int wl = blockIdx.x * 4 + wv;
  if (wl >= nleaves_cls) return;
  if constexpr (leaf_lds_rows(NCB) < NCB) {
    // 6..8 column blocks: the triangle's later block rows in LDS (15 KiB per wave at 6, 28 KiB
    // at 7 and 8: 152 KiB per workgroup with the staging), which frees the registers the tile
    // needs
    constexpr int RL = leaf_lds_rows(NCB);
    __shared__ float rl_all[4][TriSplit<NCB, RL>::lds_blocks * 256];
    tsqr_leaf<NCB, NRB, BF, false, RL>(leaf_prob[leaf_begin + wl], leaf_idx[leaf_begin + wl], probs, n, Red, d,
                                       lamv, slots, counters, RBall, lds_all[wv], lane, QStore(), rl_all[wv]);
  } else {
    tsqr_leaf<NCB, NRB, BF>(leaf_prob[leaf_begin + wl], leaf_idx[leaf_begin + wl], probs, n, Red, d, lamv, slots,
                            counters, RBall, lds_all[wv], lane);
  }
}
template <int NCB, int NRB, bool BF>
__global__ void __launch_bounds__(256)
k_tsqr_mfma_keep(int leaf_begin, int nleaves_cls, const int32_t* __restrict__ leaf_prob,
                 const int32_t* __restrict__ leaf_idx, const ProbDesc* __restrict__ probs, int n,
                 const float* __restrict__ Red, const double* __restrict__ d, const double* __restrict__ lamv,
                 float* __restrict__ slots, int* __restrict__ counters, float* __restrict__ RBall, const QStore qs) {
  __shared__ float lds_all[4][kWaveLds];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int wl = blockIdx.x * 4 + wv;
  if (wl >= nleaves_cls) return;
  tsqr_leaf<NCB, NRB, BF, true>(leaf_prob[leaf_begin + wl], leaf_idx[leaf_begin + wl], probs, n, Red, d, lamv, slots,
                                counters, RBall, lds_all[wv], lane, qs);
}

// Leaf tile blocks of 16 rows for each column-block count (leaf_tile_rows, qrk_batch.hpp).
template <int NCB>
struct LeafTile {
  static constexpr int nrb = leaf_tile_rows(NCB) / 16;
  static constexpr int nrb_keep = leaf_tile_rows_keep(NCB) / 16;
};

// The leaves of every problem with at most kQueueNCB column blocks in one persistent launch:
// each wave takes the next item of the leaf list (widest problems first) from a device-scope
// counter until the list is exhausted, and runs that leaf with the body instantiated for its
// problem's column-block count.  A wave that finds its merge partner still running goes on to
// the next item.  Every leaf body needs the whole register file (one wave per SIMD), so one
// launch over all widths costs no occupancy against one launch per width, and the narrow
// problems' leaves fill the SIMDs that the wide ones leave idle at the end.  kQueueNCB (the
// widest count in the queue) is in qrk_batch.hpp.

// The queue kernel calls each width's body as a function of its own, so that every body keeps
// the register allocation it has in a kernel by itself (inlined side by side, the six bodies
// exceed the register file and spill).
template <int NCB, bool BF>
__device__ __noinline__ void tsqr_leaf_call(int pi, int leaf, const ProbDesc* __restrict__ probs, int n,
                                            const float* __restrict__ Red, const double* __restrict__ d,
                                            const double* __restrict__ lamv, float* __restrict__ slots,
                                            int* __restrict__ counters, float* __restrict__ RBall, float* lds,
                                            int lane, float* rl) {
  tsqr_leaf<NCB, LeafTile<NCB>::nrb, BF, false, leaf_lds_rows(NCB)>(pi, leaf, probs, n, Red, d, lamv, slots,
                                                                     counters, RBall, lds, lane, QStore(), rl);
}
template <int NCB, bool BF>
__device__ __noinline__ void tsqr_leaf_call_keep(int pi, int leaf, const ProbDesc* __restrict__ probs, int n,
                                                 const float* __restrict__ Red, const double* __restrict__ d,
                                                 const double* __restrict__ lamv, float* __restrict__ slots,
                                                 int* __restrict__ counters, float* __restrict__ RBall, float* lds,
                                                 int lane, const QStore qs) {
  tsqr_leaf<NCB, LeafTile<NCB>::nrb_keep, BF, true>(pi, leaf, probs, n, Red, d, lamv, slots, counters, RBall, lds, lane,
                                               qs);
}

// The queue's work loop; KEEP: the stored-Q bodies.
template <bool BF, bool KEEP>
__device__ __forceinline__ void tsqr_queue_loop(int nitems, const int32_t* __restrict__ leaf_prob,
                                                const int32_t* __restrict__ leaf_idx,
                                                const ProbDesc* __restrict__ probs, int n,
                                                const float* __restrict__ Red, const double* __restrict__ d,
                                                const double* __restrict__ lamv, float* __restrict__ slots,
                                                int* __restrict__ counters, int* __restrict__ qhead,
                                                float* __restrict__ RBall, const QStore& qs) {
  __shared__ float lds_all[4][kWaveLds];
  const int lane = threadIdx.x & 63;
  float* lds = lds_all[threadIdx.x >> 6];
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(qhead, 1);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= nitems) return;
    const int pi = leaf_prob[item];
    const int leaf = leaf_idx[item];
    switch ((probs[pi].L + 15) >> 4) {
#define QRK_QLEAF(C)                                                                                          \
  case C:                                                                                                     \
    if constexpr (KEEP) {                                                                                     \
      tsqr_leaf_call_keep<C, BF>(pi, leaf, probs, n, Red, d, lamv, slots, counters, RBall, lds, lane, qs);    \
    } else if constexpr (leaf_lds_rows(C) < C) {                                                              \
      __shared__ float rl_all[4][TriSplit<C, leaf_lds_rows(C)>::lds_blocks * 256];                            \
      tsqr_leaf_call<C, BF>(pi, leaf, probs, n, Red, d, lamv, slots, counters, RBall, lds, lane,              \
                            rl_all[threadIdx.x >> 6]);                                                        \
    } else {                                                                                                  \
      tsqr_leaf_call<C, BF>(pi, leaf, probs, n, Red, d, lamv, slots, counters, RBall, lds, lane, nullptr);    \
    }                                                                                                         \
    break;
      QRK_QLEAF(1) QRK_QLEAF(2) QRK_QLEAF(3) QRK_QLEAF(4) QRK_QLEAF(5) QRK_QLEAF(6)
#undef QRK_QLEAF
      default:
        break;
    }
  }
}

template <bool BF>
__global__ void __launch_bounds__(256)
k_tsqr_queue(int nitems, const int32_t* __restrict__ leaf_prob, const int32_t* __restrict__ leaf_idx,
             const ProbDesc* __restrict__ probs, int n, const float* __restrict__ Red, const double* __restrict__ d,
             const double* __restrict__ lamv, float* __restrict__ slots, int* __restrict__ counters,
             int* __restrict__ qhead, float* __restrict__ RBall) {
  tsqr_queue_loop<BF, false>(nitems, leaf_prob, leaf_idx, probs, n, Red, d, lamv, slots, counters, qhead, RBall,
                             QStore());
}
template <bool BF>
__global__ void __launch_bounds__(256)
k_tsqr_queue_keep(int nitems, const int32_t* __restrict__ leaf_prob, const int32_t* __restrict__ leaf_idx,
                  const ProbDesc* __restrict__ probs, int n, const float* __restrict__ Red,
                  const double* __restrict__ d, const double* __restrict__ lamv, float* __restrict__ slots,
                  int* __restrict__ counters, int* __restrict__ qhead, float* __restrict__ RBall, const QStore qs) {
  tsqr_queue_loop<BF, true>(nitems, leaf_prob, leaf_idx, probs, n, Red, d, lamv, slots, counters, qhead, RBall, qs);
}

template <int NCB, int NRB>
hipError_t launch_tsqr_mfma_ncb(bool bf16x3, int leaf_begin, int nleaves_cls, const int32_t* leaf_prob,
                                const int32_t* leaf_idx, const ProbDesc* probs, int n, const float* Red, const double* d,
                                const double* lam, float* slots, int* counters, float* RB, const QStore& qs,
                                hipStream_t st) {
  // the plain leaves stream tiles of leaf_tile_rows rows, the leaves that store Q those of
  // leaf_tile_rows_keep (the stored Q's tile count per leaf)
  static_assert(16 * NRB == leaf_tile_rows(NCB), "leaf tile height");
  constexpr int NRBK = LeafTile<NCB>::nrb_keep;  // the leaves that store Q
  const int grid = (nleaves_cls + 3) / 4;
  if (qs.qt != nullptr) {
    if (bf16x3)
      hipLaunchKernelGGL((k_tsqr_mfma_keep<NCB, NRBK, true>), dim3(grid), dim3(256), 0, st, leaf_begin, nleaves_cls,
                         leaf_prob, leaf_idx, probs, n, Red, d, lam, slots, counters, RB, qs);
    else
      hipLaunchKernelGGL((k_tsqr_mfma_keep<NCB, NRBK, false>), dim3(grid), dim3(256), 0, st, leaf_begin, nleaves_cls,
                         leaf_prob, leaf_idx, probs, n, Red, d, lam, slots, counters, RB, qs);
  } else {
    if (bf16x3)
      hipLaunchKernelGGL((k_tsqr_mfma<NCB, NRB, true>), dim3(grid), dim3(256), 0, st, leaf_begin, nleaves_cls,
                         leaf_prob, leaf_idx, probs, n, Red, d, lam, slots, counters, RB);
    else
      hipLaunchKernelGGL((k_tsqr_mfma<NCB, NRB, false>), dim3(grid), dim3(256), 0, st, leaf_begin, nleaves_cls,
                         leaf_prob, leaf_idx, probs, n, Red, d, lam, slots, counters, RB);
  }
  return hipGetLastError();
}

}  // namespace qrk
