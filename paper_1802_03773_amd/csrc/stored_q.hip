// Q^T b with the stored Q of a float32 block-angular factor (QRkit Section 2: Q kept as an
// object that applies its Householder reflectors rather than as a matrix; Sections 5.1 and 5.2:
// Q^T applied to a new right-hand side).  The reflectors are applied in the order the
// factorisation produced them:
//   1. blocks: the reflectors of block i applied to [b_i; 0] (its data rows, then its n damping
//      rows): the first n entries are c_i, the others the right-hand side of the block's reduced
//      rows (data rows n .. m_i-1, then the damping rows, as the factorisation stores them);
//   2. dense part, one wave per leaf: the compact-WY panels of every tile the leaf merged,
//      applied to the leaf's running right-hand side u (one entry per triangle row; the leaf's
//      triangle starts as the damping rows sqrt(lam) D_B for leaf 0 and as zero rows otherwise,
//      whose right-hand side is zero) and to the tile's reduced right-hand side;
//   3. merges: each node's panels applied to [u_left; u_right] along the same pairwise tree as
//      the factorisation (the second leaf of a pair to finish merges), the root's u holding c_B.
// c_i and c_B are written laid out like p.  Everything after stage 1 runs in float32, as the
// factorisation did; stage 1 accumulates in float64.
#include "qrk_batch.hpp"
#include "qrk_device.hpp"
#include "qrk_launch.hpp"
#include "tsqr_mfma.hpp"
#include "tsqr_tree.hpp"

namespace qrk {

// ---- stage 1: per-block reflectors (one wave per block, lane r holds row r) -----------------
// H_j = I - g_j z_j z_j^T over the block's rows: z_j at the data rows in qvd (row-major like A),
// at the damping rows in qvp ([block][damping row][j]), g_j in qg.  Requires n <= m_i and
// m_i + n <= 64.
template <int N>
__global__ void __launch_bounds__(256)
k_qt_blocks(int64_t K, const ProbDesc* __restrict__ probs, const int32_t* __restrict__ blk_prob,
            const int64_t* __restrict__ row_off, const float* __restrict__ b, const float* __restrict__ qvd,
            const float* __restrict__ qvp, const float* __restrict__ qg, double* __restrict__ c,
            float* __restrict__ xr) {
  const int lane = threadIdx.x & 63;
  const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blk >= K) return;
  const int pi = blk_prob ? blk_prob[blk] : 0;
  const ProbDesc& P = probs[pi];
  const int64_t r0 = row_off[blk];
  const int m = (int)(row_off[blk + 1] - r0);
  const bool data = lane < m;
  const bool damp = lane >= m && lane < m + N;
  double v = data ? (double)b[r0 + lane] : 0.0;
  float z[N];
#pragma unroll
  for (int j = 0; j < N; ++j)
    z[j] = data ? qvd[(r0 + lane) * N + j] : (damp ? qvp[(blk * N + (lane - m)) * N + j] : 0.f);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double s = wave_allreduce_sum((double)z[j] * v);
    v -= (double)qg[blk * N + j] * s * (double)z[j];
  }
  if (lane < N)
    c[P.noff + (blk - P.koff) * N + lane] = v;
  else if (lane < m + N)
    xr[r0 + lane - N] = (float)v;  // reduced row lane - N of the block
}

// ---- stages 2 and 3: compact-WY panels ----------------------------------------------------
// One kept panel applied to a right-hand side (Q_p^T = I - V T^T V^T, V = [I; W diag(s)]):
//   z = u + diag(s) W^T x;  z' = T^T z;  u -= z';  x -= W diag(s) z'
// u: lane k of every 16-lane row holds entry k of the panel's 16 triangle rows; x: this lane's
// rows of the tile (row q * 64 + lane); w: those rows' raw reflector entries (zero past the
// tile); tc: column k of T (k = lane % 16), sk: scale k; sm: the wave's LDS.
constexpr int kSmFloats = 64 * 17 + 16;

template <int RPL>
__device__ __forceinline__ void qt_panel(const float (&w)[RPL][16], float (&x)[RPL], float& u, const float (&tc)[16],
                                         float sk, float* sm, int lane) {
  const int k = lane & 15;
  const int part = lane >> 4;
  // W^T x: this lane's row products, then the column sums through LDS (lane (part, k) adds
  // rows 16 part .. 16 part + 15 of column k) and across the four 16-lane rows
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    float pj = 0.f;
#pragma unroll
    for (int q = 0; q < RPL; ++q) pj += w[q][j] * x[q];
    sm[lane * 17 + j] = pj;
  }
  wave_lds_sync();
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += sm[(part * 16 + i) * 17 + k];
  s = sum_rows4(s);
  const float z = u + sk * s;
  // z'_k = sum_i T[i][k] z_i (T upper triangular), z_i from lane i of the row
  float zp = 0.f;
  static_for<0, 16>([&](auto II) {
    constexpr int i = decltype(II)::value;
    zp += tc[i] * row_bcast<i>(z);
  });
  u -= zp;
  if (lane < 16) sm[64 * 17 + lane] = sk * zp;
  wave_lds_sync();
  float y[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) y[j] = sm[64 * 17 + j];
#pragma unroll
  for (int q = 0; q < RPL; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) x[q] -= w[q][j] * y[j];
  wave_lds_sync();  // the next panel overwrites sm
}

// The data of NP kept panels that one application reads, loaded into registers before the
// first panel's exchange so that the loads of all panels are in flight together.  TS(p): the
// panel's T and scales; its reflector blocks follow at + 320, row r at + 320 + 16 r, rows at or
// past `rows` (of this lane's RPL rows) read as zero.
template <int NP, int RPL>
struct PanelSet {
  float w[NP][RPL][16];
  float tc[NP][16];
  float sk[NP];
  template <typename TSof>
  __device__ __forceinline__ void load(TSof TS, int rows_lim_step, int lane) {
    const int k = lane & 15;
    static_for<0, NP>([&](auto PP) {
      constexpr int p = decltype(PP)::value;
      const float* ts = TS(p);
      const int rows = rows_lim_step < 0 ? 64 * RPL : rows_lim_step * (p + 1);
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int row = q * 64 + lane;
        const bool in = row < rows;
        const f4* wr = reinterpret_cast<const f4*>(ts + 320 + (in ? row : 0) * 16);  // in bounds
#pragma unroll
        for (int j4 = 0; j4 < 4; ++j4) {
          const f4 l = wr[j4];
          const f4 v = in ? l : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int e = 0; e < 4; ++e) w[p][q][4 * j4 + e] = v[e];
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) tc[p][i] = ts[i * 16 + k];
      sk[p] = ts[256 + k];
    });
  }
};

// One wave per leaf of the problems with NCB column blocks (the factorisation's leaf list):
// stage 2 over the leaf's tiles, then stage 3 up the problem's tree.  xr: the reduced
// right-hand side by global row; uslots: 128 floats per tree slot from the problem's qc0 (QOff);
// counters from ctr0, cleared beforehand.
template <int NCB>
__global__ void __launch_bounds__(256)
k_qt_leaves(int leaf_begin, int nleaves_cls, const int32_t* __restrict__ leaf_prob,
            const int32_t* __restrict__ leaf_idx, const ProbDesc* __restrict__ probs, int n,
            const QStore qs, const float* __restrict__ xr, float* __restrict__ uslots, int* __restrict__ counters,
            double* __restrict__ c) {
  constexpr int KT = leaf_tile_rows_keep(NCB);
  constexpr int RPL = KT / 64;                // tile rows per lane
  constexpr int RPM = (16 * NCB + 63) / 64;   // triangle rows per lane in a merge
  constexpr int64_t TPF = tile_panel_floats(KT / 16);
  __shared__ float sm_all[4][kSmFloats];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int wl = blockIdx.x * 4 + wv;
  if (wl >= nleaves_cls) return;
  float* sm = sm_all[wv];
  const int pi = leaf_prob[leaf_begin + wl];
  const int leaf = leaf_idx[leaf_begin + wl];
  const ProbDesc& P = probs[pi];
  const QOff& Q = qs.qo[pi];
  const int k = lane & 15;
  const float* xp = xr + P.moff;
  float u[NCB];
#pragma unroll
  for (int p = 0; p < NCB; ++p) u[p] = 0.f;

  // ---- stage 2: the leaf's tiles (their reflector blocks are zero past the leaf's rows) ----
  const int64_t r0 = (int64_t)leaf * P.rows_per_leaf;
  const int64_t r1 = r0 + P.rows_per_leaf < P.M ? r0 + P.rows_per_leaf : P.M;
  int64_t tile = 0;
  for (int64_t t = r0; t < r1; t += KT, ++tile) {
    float x[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int64_t row = t + q * 64 + lane;
      x[q] = row < r1 ? xp[row] : 0.f;
    }
    const float* qp = qs.qt + Q.qt0 + ((int64_t)leaf * Q.qtiles + tile) * (NCB * TPF);
    PanelSet<NCB, RPL> ps;
    ps.load([&](int p) { return qp + p * TPF; }, -1, lane);
    static_for<0, NCB>([&](auto PP) {
      constexpr int p = decltype(PP)::value;
      qt_panel<RPL>(ps.w[p], x, u[p], ps.tc[p], ps.sk[p], sm, lane);
    });
  }

  // ---- stage 3: merges up the problem's tree (the factorisation's pairing and node order) ----
  float* us = uslots + Q.qc0;
  int* pctr = counters + P.ctr0;
  int nl = P.leaves;
  int slot = leaf;
  int64_t base = 0, cbase = 0, mbase = 0;
  while (nl > 1) {
    const int sib = slot ^ 1;
    const int parent = slot >> 1;
    const int nn = (nl + 1) >> 1;
    if (sib < nl) {
      // the node's panels (written by the factorisation): their loads overlap the arrival
      // (panel p of a node reflects rows 0 .. 16 (p + 1) - 1 of the right triangle)
      const float* nq = qs.qn + Q.qn0 + (mbase + parent) * node_panel_off(NCB);
      PanelSet<NCB, RPM> ps;
      ps.load([&](int p) { return nq + node_panel_off(p); }, 16, lane);
      // publish u with device-coherent stores, wait for them, then arrive (as the separate merge
      // tree of the factorisation publishes its blocks): no cache-wide fence
      const auto rs_u = __builtin_amdgcn_make_buffer_rsrc(us + (base + slot) * 128, 0, 512, 0x00020000);
      if (lane < 16) {
#pragma unroll
        for (int p = 0; p < NCB; ++p)
          __builtin_amdgcn_raw_buffer_store_b32(u_of(u[p]), rs_u, (16 * p + lane) * 4, 0, kCoherent);
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      int old = 0;
      if (lane == 0)
        old = __hip_atomic_fetch_add(&pctr[cbase + parent], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      old = __builtin_amdgcn_readfirstlane(old);
      if (old == 0) return;  // the sibling is still running; it will merge
      asm volatile("" ::: "memory");  // the sibling's vector is read after its arrival was seen
      const int left = slot & ~1;
      const auto rs_l = __builtin_amdgcn_make_buffer_rsrc(us + (base + left) * 128, 0, 512, 0x00020000);
      const auto rs_r = __builtin_amdgcn_make_buffer_rsrc(us + (base + left + 1) * 128, 0, 512, 0x00020000);
#pragma unroll
      for (int p = 0; p < NCB; ++p) u[p] = f_of(__builtin_amdgcn_raw_buffer_load_b32(rs_l, (16 * p + k) * 4, 0, kCoherent));
      float x[RPM];
#pragma unroll
      for (int q = 0; q < RPM; ++q) {
        const int row = q * 64 + lane;
        const float l = f_of(__builtin_amdgcn_raw_buffer_load_b32(rs_r, (row < 16 * NCB ? row : 0) * 4, 0, kCoherent));
        x[q] = row < 16 * NCB ? l : 0.f;
      }
      static_for<0, NCB>([&](auto PP) {
        constexpr int p = decltype(PP)::value;
        qt_panel<RPM>(ps.w[p], x, u[p], ps.tc[p], ps.sk[p], sm, lane);
      });
    }
    base += nl;
    cbase += nn;
    mbase += nl >> 1;
    slot = parent;
    nl = nn;
  }

  // ---- root: c_B ----
  if (lane < 16) {
#pragma unroll
    for (int p = 0; p < NCB; ++p) {
      const int col = 16 * p + lane;
      if (col < P.nB) c[P.noff + P.K * n + col] = (double)u[p];
    }
  }
}

hipError_t launch_apply_qt(const BatchView& bv, const int* cls_begin, const int* cls_count,
                           const int32_t* leaf_prob, const int32_t* leaf_idx, const float* b, const QKeep& qk,
                           const QStore& qs, float* xr, float* uslots, int* counters, int64_t nctr, double* c,
                           hipStream_t st) {
  if (!qk.vd || !qk.vp || !qk.g || bv.max_L > kMaxDense || bv.max_rows > 64) return hipErrorInvalidValue;
  hipError_t e = launch_zero_ints(counters, nctr, st);
  if (e != hipSuccess) return e;
  const int32_t* bp = bv.P == 1 ? nullptr : bv.blk_prob;
  const dim3 blk(256);
  if (bv.Ktot > 0) {
    const dim3 grd((unsigned)((bv.Ktot + 3) / 4));
    const float* vd = static_cast<const float*>(qk.vd);
    const float* vp = static_cast<const float*>(qk.vp);
    const float* g = static_cast<const float*>(qk.g);
    switch (bv.n) {
#define QRK_QB(NN)                                                                                        \
  case NN:                                                                                                \
    hipLaunchKernelGGL((k_qt_blocks<NN>), grd, blk, 0, st, bv.Ktot, bv.probs, bp, bv.row_off, b, vd, vp, g, \
                       c, xr);                                                                            \
    break;
      QRK_QB(1) QRK_QB(2) QRK_QB(3) QRK_QB(4) QRK_QB(5) QRK_QB(6) QRK_QB(7) QRK_QB(8)
#undef QRK_QB
      default:
        return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int cl = 8; cl >= 1; --cl) {
    const int nlv = cls_count[cl];
    if (nlv == 0) continue;
    const dim3 grd((unsigned)((nlv + 3) / 4));
    switch (cl) {
#define QRK_QL(C)                                                                                            \
  case C:                                                                                                    \
    hipLaunchKernelGGL((k_qt_leaves<C>), grd, blk, 0, st, cls_begin[cl], nlv, leaf_prob, leaf_idx, bv.probs, \
                       bv.n, qs, xr, uslots, counters, c);                                                   \
    break;
      QRK_QL(1) QRK_QL(2) QRK_QL(3) QRK_QL(4) QRK_QL(5) QRK_QL(6) QRK_QL(7) QRK_QL(8)
#undef QRK_QL
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace qrk
