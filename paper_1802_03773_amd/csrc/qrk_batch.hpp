// Layout of a batch of independent block-angular problems inside one handle.
//
// All problems share the block width n.  Problem p owns K_p consecutive blocks of the
// global block list, M_p consecutive rows of A and b, and N_p = K_p n + nB_p consecutive
// unknowns of d and p; its coupled columns B_p are a row-major M_p x ldb_p array starting
// at element boff of B.  The handle's workspace (S|c, reduced rows, R_B|c_B, merge-tree
// slots and counters, refinement partials) is carved per problem the same way.  A single
// problem is the batch of one with every offset zero.
#pragma once

#include <stdint.h>

namespace qrk {

constexpr int kMaxDense = 128;  // nB + 1 <= 128
// Dense parts of at most this many 16-column blocks run their leaves in one persistent launch
// (a device work queue of leaves, widest problems first); wider ones have a launch per width.
constexpr int kQueueNCB = 6;

// Dense-part leaves stream tiles of this many rows: 128 up to 4 column blocks and at 6 (there with
// the running triangle's block rows 1..5 in LDS), 64 at 5, 7 and 8 (a taller tile does not fit
// the register file there, at 5 not even with the triangle in LDS).  The leaves that store Q keep
// the triangle in registers and use leaf_tile_rows_keep (the stored tile panels are laid out by
// it).
constexpr int leaf_tile_rows(int ncb) { return ncb <= 4 || ncb == 6 ? 128 : 64; }
constexpr int leaf_tile_rows_keep(int ncb) { return ncb <= 4 ? 128 : 64; }

// Stored Q of the float32 dense part: per 16-column panel, T (16 x 16, row-major), the column
// scales (16, padded to 64) and the raw reflector blocks W (16 x 16 each, row-major, block row
// rb at float 320 + 256 rb).  A tile merged into a leaf keeps nrb = leaf_tile_rows_keep / 16 blocks
// per panel (tile_panel_floats each, panel p at p * tile_panel_floats); a merge of two
// triangles keeps p + 1 blocks for panel p (the rows of the right triangle it touches), panel p
// at node_panel_off(p), a node of ncb column blocks taking node_panel_off(ncb).
constexpr int64_t tile_panel_floats(int nrb) { return 320 + 256 * (int64_t)nrb; }
constexpr int64_t node_panel_off(int p) { return (int64_t)p * (256 + 64) + 256 * ((int64_t)p * (p + 1) / 2); }

struct ProbDesc {
  int64_t koff, K;        // first global block, blocks
  int64_t moff, M;        // first global row, rows
  int64_t noff;           // first unknown (index into d and p)
  int64_t boff, ldb;      // B_p at element boff of B, row stride ldb
  int64_t soff;           // S_p|c_p (K x n x L, row stride L) at element soff
  int64_t redoff, ldr;    // reduced rows (M x ldr) at element redoff
  int64_t rboff;          // R_B|c_B (L x L, row-major) at element rboff
  int64_t slot0, ctr0;    // merge tree: first slot float, first arrival counter
  int64_t rows_per_leaf;  // dense-part QR: rows per leaf
  int64_t pack0, npacks;  // packs of whole blocks (global index of the first)
  int32_t nB, L;          // coupled columns, L = nB + 1
  int32_t leaves;         // dense-part QR leaves
  int32_t wg0, nwg;       // refinement workgroups [wg0, wg0 + nwg)
  int32_t tree_sep;       // 1: the leaves only store their triangles; a separate launch merges them
  int32_t pad;
};

// Work the first per-block QR launch of a factor call does before its blocks: workgroup 0
// clears z0[0..n0) and z1[0..n1) (status words, merge-tree arrival counters), and when
// lam_out is set every block uses lam_val for lambda and thread 0 of workgroup 0 stores it
// to *lam_out for the later kernels (which run after the launch completes).
struct BqrPrologue {
  int* z0 = nullptr;
  int64_t n0 = 0;
  int* z1 = nullptr;
  int64_t n1 = 0;
  double* lam_out = nullptr;
  double lam_val = 0.0;
};

// Stored Q of a problem's dense part (in an array of its own, so that the kernels without the
// stored Q see the batch layout alone): first float of its leaves' tile panels and tiles per
// leaf, first float of its merge nodes' panels, first float of the application's merge vectors.
struct QOff {
  int64_t qt0, qtiles, qn0, qc0;
};
// Where the dense-part kernels store Q (all null: not stored).
struct QStore {
  float* qt = nullptr;       // tile panels
  float* qn = nullptr;       // merge-node panels
  const QOff* qo = nullptr;  // [P]
};

// Where a factor call keeps the per-block reflectors (the stored Q of qrk_set_keep_q; null
// pointers: not kept).  Block i's reflector j is H_j = I - g_j z_j z_j^T over the block's data
// rows and damping rows: vd [M x n] holds z_j at the data rows (row-major like A; z_j is zero
// above row j), vp [K x n x n] its entries at the damping rows ([block][damping row][j]), and
// g [K x n] the g_j.
struct QKeep {
  void* vd = nullptr;
  void* vp = nullptr;
  void* g = nullptr;
};

// Device view of a handle's batch, passed to the launchers.
struct BatchView {
  int P = 1;                           // problems
  int n = 1;                           // block width
  int64_t Ktot = 0;                    // blocks over all problems
  int max_L = 1;                       // max_p nB_p + 1
  int max_rows = 0;                    // max_i m_i + n
  const ProbDesc* probs = nullptr;     // [P]
  const int32_t* blk_prob = nullptr;   // [Ktot] problem of each block
  const int64_t* row_off = nullptr;    // [Ktot + 1] global row offsets
  const int64_t* pack_blk = nullptr;   // [npacks + 1] global block index of each pack start
  const int32_t* wg_prob = nullptr;    // [nwg] problem of each refinement workgroup
  int nwg = 1;
  const double* lam = nullptr;         // [P] damping, read on the device
  int grid_blocks = 1;                 // block-QR launch
};

}  // namespace qrk
