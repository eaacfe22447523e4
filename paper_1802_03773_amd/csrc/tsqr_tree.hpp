// Dense-part merge tree as a launch of its own, pipelined over column blocks (float32).
//
// What is computed (QRkit Section 4.2): the triangle of QR([R_left; R_right]) at every inner
// node of the tall-skinny QR's reduction tree, the root being R_B | c_B.
//
// Organisation.  The leaves (k_tsqr_mfma with the problem's tree_sep set) store their
// triangles and exit.  Here one wave per merge node works left-looking over column blocks of
// 16.  Column block q is published in two parts, each with a flag of its own: the blocks above
// the diagonal (block rows 0..q-1), which are final once the node's panels 0..q-1 have been
// applied, and then the diagonal block, final once panel q is factored.  For column block q a
// node waits until both children have published the part above the diagonal, loads it and
// applies the reflectors of its own panels 0..q-1 to it (compact WY, kept in LDS; panel p
// touches block rows 0..p only), publishes that part, then waits for the children's diagonal
// blocks, factors panel q, keeps that panel's reflectors (T, column scales, raw tile columns W)
// for the later column blocks and publishes its diagonal block.  The applications thus overlap
// the children's factorisation of the same column block, and a parent starts on column block
// 0 while its children are still on later ones, so the root trails the leaves by about
// (tree depth + column blocks) panel times rather than (tree depth) whole merges.
//
// Memory ordering.  A node's published blocks are written and read with device-coherent
// accesses (through the L2 to memory and back); the producer waits for its block stores to
// complete before storing the flag, the consumer polls the flag with device-scope loads and
// only then issues the block's loads.
//
// Forward progress.  Nodes are numbered level by level from the leaves up, and the children
// of a node are leaves or nodes with smaller numbers.  Wave w of the launch runs node w and
// workgroups are dispatched in order, so a wave only waits for waves that were dispatched
// before it or belong to its own workgroup.  Every wait is bounded: a flag not seen within the
// bound sets the problem's ST_STALL status bit, and the wave still publishes every column
// block so that no other wave waits on it.
//
// The panel factorisation and the compact-WY application are those of merge_tile (same
// reflector sign, scales, T recurrence and layouts), split so that a panel's reflectors can be
// applied to column blocks that arrive later.
#pragma once

#include "tsqr_mfma.hpp"

namespace qrk {


// Factor the panel [Rd; X[0..RBN-1]]: Rd is the 16x16 diagonal block of the R part, X the
// tile blocks of this column block (accumulator layout).  On return Rd holds the new diagonal
// block and R's row j entries, X the raw reflector columns, and T, the scales and W are kept
// in LDS at `keep`.
template <int RBN>
__device__ __forceinline__ void tree_panel_factor(f4& Rd, f4* X, float* __restrict__ keep, int lane) {
  const int g = lane >> 4;
  const int c = lane & 15;
  float trow[16];  // lane (g, c) builds row c of T
  float sc;        // scale of this lane's column
  {
    f4 Xp[RBN];
#pragma unroll
    for (int rb = 0; rb < RBN; ++rb) Xp[rb] = X[rb];
    panel_factor<RBN>(Rd, Xp, trow, sc, lane);
#pragma unroll
    for (int rb = 0; rb < RBN; ++rb) X[rb] = Xp[rb];
  }
  float* Tl = keep;
  float* Sl = keep + 256;
  float* Wl = keep + 320;
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < 16; k += 4)
      *reinterpret_cast<f4*>(Tl + c * 16 + k) = f4{trow[k], trow[k + 1], trow[k + 2], trow[k + 3]};
    Sl[c] = sc;
  }
#pragma unroll
  for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) Wl[rb * 256 + (4 * g + v) * 16 + c] = X[rb][v];
  wave_lds_sync();
}

// Apply a kept panel (RBN tile blocks) to one column block: Rp is the column block's R-part
// block in the panel's block row, X its tile blocks 0..RBN-1.
//   Z = Rp + diag(s) X_P^T X;  Z' = T^T Z;  Rp -= Z';  X -= X_P diag(s) Z'
template <int RBN>
__device__ __forceinline__ void tree_panel_apply(const float* __restrict__ keep, f4& Rp, f4* X, int lane) {
  const int g = lane >> 4;
  const int c = lane & 15;
  const float* Tl = keep;
  const float* Sl = keep + 256;
  const float* Wl = keep + 320;
  f4 Td;
#pragma unroll
  for (int v = 0; v < 4; ++v) Td[v] = Tl[(4 * g + v) * 16 + c];
  const f4 srow = *reinterpret_cast<const f4*>(Sl + 4 * g);
  float Pa[RBN][4];  // x[rb*16 + 4g + v][c]       (panel columns, accumulator layout)
  float Wt[RBN][4];  // -x[rb*16 + c][4g + v]      (transposed)
#pragma unroll
  for (int rb = 0; rb < RBN; ++rb) {
    const f4 w4 = *reinterpret_cast<const f4*>(Wl + rb * 256 + c * 16 + 4 * g);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Pa[rb][v] = Wl[rb * 256 + (4 * g + v) * 16 + c];
      Wt[rb][v] = -w4[v];
    }
  }
  f4 Y0 = {0.f, 0.f, 0.f, 0.f}, Y1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if ((rb * 4 + v) & 1)
        Y1 = mfma4(Pa[rb][v], X[rb][v], Y1);
      else
        Y0 = mfma4(Pa[rb][v], X[rb][v], Y0);
    }
  const f4 Z = Rp + srow * (Y0 + Y1);
  f4 Zp = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int v = 0; v < 4; ++v) Zp = mfma4(Td[v], Z[v], Zp);
  Rp -= Zp;
  const f4 Zs = srow * Zp;
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int rb = 0; rb < RBN; ++rb) X[rb] = mfma4(Wt[rb][v], Zs[v], X[rb]);
}

// Published node outputs move through device-coherent accesses (the sc1 cache policy, which is
// what a relaxed device-scope atomic access compiles to): stores write through and loads read
// past the per-XCD L2, so a consumer never sees a stale L2 copy, and a producer's release is
// just the wait for its own stores to complete before the flag store -- no L2-wide write-back
// or invalidation, which at one per column block and node (on every XCD) had cost more than
// the arithmetic.  Each lane moves its four values of a 16x16 block as one 16-byte access.
constexpr int kCoherent = 16;  // buffer cache-policy bits: sc1
__device__ __forceinline__ void tree_store_block(float* dst, const f4& v, int lane) {
  const auto rs = __builtin_amdgcn_make_buffer_rsrc(dst, 0, 1024, 0x00020000);
  __builtin_amdgcn_raw_buffer_store_b128(v, rs, lane * 16, 0, kCoherent);
}
__device__ __forceinline__ f4 tree_load_block(const float* src, int lane) {
  const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(src), 0, 1024, 0x00020000);
  return __builtin_amdgcn_raw_buffer_load_b128(rs, lane * 16, 0, kCoherent);
}

// Wait (bounded) until both *fa and *fb are set (a null flag counts as set); false on
// timeout.  Lane 0 polls with relaxed device-scope loads (no cache invalidation per poll),
// both flags in the same round trip.
__device__ __forceinline__ bool tree_wait2(const int* fa, const int* fb, int lane) {
  for (int it = 0; it < (1 << 20); ++it) {
    int ready = 1;
    if (lane == 0) {
      const int va = fa ? __hip_atomic_load(fa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 1;
      const int vb = fb ? __hip_atomic_load(fb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 1;
      ready = (va != 0) && (vb != 0);
    }
    if (__builtin_amdgcn_readfirstlane(ready) != 0) return true;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

// One wave per inner node of the (single) problem's tree.  node_l / node_r: child references,
// r >= 0 an inner node, r < 0 leaf -1 - r.  Leaf triangles are at slots 0 .. leaves-1 of the
// problem, node outputs at slots leaves + node; flags[(node * NCB + q) * 2] marks column block
// q of a node's output as published above the diagonal, flags[(node * NCB + q) * 2 + 1] its
// diagonal block.  The root (the last node) writes R_B | c_B row-major.  KEEP (the stored Q):
// node w's kept panels are written to qs.qn + qn0 + w * TreeKeep<NCB>::total at its end.
// Waves (nodes) per workgroup: four, or three at 8 column blocks, whose kept panels (46 KiB per
// wave) fit the 160 KiB of LDS only three at a time.
constexpr int tree_waves(int ncb) { return ncb <= 7 ? 4 : 3; }

template <int NCB, bool KEEP>
__device__ __forceinline__ void tsqr_tree_node(const ProbDesc* probs, const int32_t* node_l, const int32_t* node_r,
                                               int nnodes, float* slots, int* flags, float* RBall, int* status,
                                               const QStore& qs) {
  constexpr int WPG = tree_waves(NCB);
  __shared__ float keep_all[WPG][TreeKeep<NCB>::total];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int node = blockIdx.x * WPG + wv;
  if (node >= nnodes) return;
  const ProbDesc& P = probs[0];
  const int L = P.L;
  const int nleaves = P.leaves;
  constexpr int SLOT = Tri<NCB>::count * 256;
  float* pslots = slots + P.slot0;
  int* pflags = flags + P.ctr0;
  const int lref = node_l[node], rref = node_r[node];
  const float* lsrc = pslots + (int64_t)(lref >= 0 ? nleaves + lref : -1 - lref) * SLOT;
  const float* rsrc = pslots + (int64_t)(rref >= 0 ? nleaves + rref : -1 - rref) * SLOT;
  float* out = pslots + (int64_t)(nleaves + node) * SLOT;
  const bool root = node == nnodes - 1;
  float* keep = keep_all[wv];
  const int g = lane >> 4;
  const int c = lane & 15;
  bool stalled = false;
  f4 a[NCB];  // column block q: R part (left child), block rows 0..q
  f4 x[NCB];  // column block q: tile (right child), block rows 0..q
  // block (p, q) of the left (a) or right (x) child's triangle: published node outputs are read
  // past the L2, leaf triangles come from the previous launch (plain loads)
  auto load_blocks = [&](int p, int q, f4& av, f4& xv) {
    const float* ls = lsrc + Tri<NCB>::idx(p, q) * 256;
    const float* rs = rsrc + Tri<NCB>::idx(p, q) * 256;
    av = lref >= 0 ? tree_load_block(ls, lane) : __builtin_nontemporal_load(reinterpret_cast<const f4*>(ls + lane * 4));
    xv = rref >= 0 ? tree_load_block(rs, lane) : __builtin_nontemporal_load(reinterpret_cast<const f4*>(rs + lane * 4));
  };
  // flag k (0: above the diagonal, 1: diagonal block) of column block q, once the stores before
  // it have completed
  auto publish = [&](int q, int k) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (lane == 0)
      __hip_atomic_store(pflags + ((int64_t)node * NCB + q) * 2 + k, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto wait_children = [&](int q, int k) {
    if (!stalled && (lref >= 0 || rref >= 0))
      stalled = !tree_wait2(lref >= 0 ? pflags + ((int64_t)lref * NCB + q) * 2 + k : nullptr,
                            rref >= 0 ? pflags + ((int64_t)rref * NCB + q) * 2 + k : nullptr, lane);
    asm volatile("" ::: "memory");  // the block's loads stay after the flags were seen
  };
  static_for<0, NCB>([&](auto QQ) {
    constexpr int q = decltype(QQ)::value;
    if constexpr (q > 0) {
      // above the diagonal: panels 0..q-1 applied, then published
      wait_children(q, 0);
#pragma unroll
      for (int p = 0; p < q; ++p) load_blocks(p, q, a[p], x[p]);
      static_for<0, q>([&](auto PP) {
        constexpr int p = decltype(PP)::value;
        tree_panel_apply<p + 1>(keep + TreeKeep<NCB>::off(p), a[p], x, lane);
      });
      if (!root) {
#pragma unroll
        for (int p = 0; p < q; ++p) tree_store_block(out + Tri<NCB>::idx(p, q) * 256, a[p], lane);
        publish(q, 0);
      }
    }
    // the diagonal block: panel q factored, then published
    wait_children(q, 1);
    load_blocks(q, q, a[q], x[q]);
    tree_panel_factor<q + 1>(a[q], x, keep + TreeKeep<NCB>::off(q), lane);
    if (root) {
      // column block q of R_B | c_B, row-major L x L (zeros below the diagonal)
      float* Rout = RBall + P.rboff;
      static_for<0, NCB>([&](auto PR) {
        constexpr int p = decltype(PR)::value;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * p + 4 * g + v;
          const int col = 16 * q + c;
          float val = 0.f;
          if constexpr (p < q) val = a[p][v];
          if constexpr (p == q) val = (col >= row) ? a[p][v] : 0.f;
          if (row < L && col < L) Rout[(int64_t)row * L + col] = val;
        }
      });
    } else {
      tree_store_block(out + Tri<NCB>::idx(q, q) * 256, a[q], lane);
      publish(q, 1);
    }
  });
  if constexpr (KEEP) {
    // the stored Q: this node's kept panels, as they are in LDS (TreeKeep layout)
    float* dst = qs.qn + qs.qo[0].qn0 + (int64_t)node * TreeKeep<NCB>::total;
    for (int e = lane * 4; e < TreeKeep<NCB>::total; e += 256)
      *reinterpret_cast<f4*>(dst + e) = *reinterpret_cast<const f4*>(keep + e);
  }
  if (stalled) set_status(status, ST_STALL);
}

// The launch that stores Q is a kernel of its own with one more argument.
template <int NCB>
__global__ void __launch_bounds__(256)
k_tsqr_tree(const ProbDesc* __restrict__ probs, const int32_t* __restrict__ node_l,
            const int32_t* __restrict__ node_r, int nnodes, float* __restrict__ slots, int* __restrict__ flags,
            float* __restrict__ RBall, int* __restrict__ status) {
  tsqr_tree_node<NCB, false>(probs, node_l, node_r, nnodes, slots, flags, RBall, status, QStore());
}
template <int NCB>
__global__ void __launch_bounds__(256)
k_tsqr_tree_keep(const ProbDesc* __restrict__ probs, const int32_t* __restrict__ node_l,
                 const int32_t* __restrict__ node_r, int nnodes, float* __restrict__ slots, int* __restrict__ flags,
                 float* __restrict__ RBall, int* __restrict__ status, const QStore qs) {
  tsqr_tree_node<NCB, true>(probs, node_l, node_r, nnodes, slots, flags, RBall, status, qs);
}

}  // namespace qrk
