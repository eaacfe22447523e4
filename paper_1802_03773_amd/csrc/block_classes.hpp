// Grouping of the blocks of a batch into the classes the per-block QR kernels are
// instantiated for.  Classes 0 .. 5: blocks with m_i >= n, register rows 16 / 32 / 64 (m_i + n
// rows must fit) times column slots 1 / 2 (the L_p = nB_p + 1 coupled columns of the block's
// problem must fit 64 per slot).  Classes 6 and 7: blocks with m_i < n (at most 15 rows with
// their damping rows), column slots 1 / 2, factored by the kernel with run-time n.
// Host-only, no HIP types, so the grouping can be checked on its own.
#pragma once

#include <stdint.h>

#include <vector>

namespace qrk {

constexpr int kBlockClasses = 8;

// rows of class c: 16 << (c / 2) (16 for the m_i < n classes); column slots: 1 + c % 2
inline int block_class_rows(int c) { return c < 6 ? 16 << (c >> 1) : 16; }
inline int block_class_slots(int c) { return 1 + (c & 1); }
inline bool block_class_short(int c) { return c >= 6; }

struct BlockClasses {
  int64_t begin[kBlockClasses] = {0};
  int64_t count[kBlockClasses] = {0};
  // Block ids grouped by class (class c at [begin[c], begin[c] + count[c])).  Left empty
  // when every block is in one class: that class then covers blocks 0 .. K-1 in order and
  // no list is needed.
  std::vector<int32_t> list;
};

// row_off[0..K] block row offsets; L_of_block(i) the coupled width L of block i's problem.
// Returns false if a block fits no class (m_i + n > 64, L > 128 or n outside 1 .. 8).
template <typename LOf>
inline bool group_block_classes(const int64_t* row_off, int64_t K, int n, LOf L_of_block, BlockClasses& out) {
  out = BlockClasses{};
  if (n < 1 || n > 8) return false;
  std::vector<uint8_t> cls((size_t)K);
  for (int64_t i = 0; i < K; ++i) {
    const int64_t r = row_off[i + 1] - row_off[i] + n;
    const int L = L_of_block(i);
    if (r > 64 || L > 128 || r < 0) return false;
    const int rc = row_off[i + 1] - row_off[i] < n ? 3 : (r <= 16 ? 0 : (r <= 32 ? 1 : 2));
    const int c = rc * 2 + (L <= 64 ? 0 : 1);
    cls[(size_t)i] = (uint8_t)c;
    out.count[c] += 1;
  }
  int used = 0;
  for (int c = 0; c < kBlockClasses; ++c) used += out.count[c] > 0;
  if (used <= 1) return true;
  int64_t fill[kBlockClasses];
  int64_t at = 0;
  for (int c = 0; c < kBlockClasses; ++c) {
    out.begin[c] = at;
    fill[c] = at;
    at += out.count[c];
  }
  out.list.resize((size_t)K);
  for (int64_t i = 0; i < K; ++i) out.list[(size_t)fill[cls[(size_t)i]]++] = (int32_t)i;
  return true;
}

}  // namespace qrk
