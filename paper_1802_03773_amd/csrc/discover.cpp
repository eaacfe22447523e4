// Structure discovery by row and column permutations (QRkit Section 4.3): the host-side
// preprocessing that brings a sparse J given by its row patterns to the layouts of the
// structured solvers, J' = P_r J P_c.
//   block-angular: with the coupled (dense) columns given, rows sharing a non-dense column
//     belong to one block, transitively (union-find over rows, each non-dense column linking
//     the rows that touch it); a block's columns are the non-dense columns of its rows.
//   banded: rows in order of their first column (stable), starts clamped to N - w.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "qrkit.h"

namespace {

struct Dsu {
  std::vector<int64_t> p;
  explicit Dsu(int64_t n) : p((size_t)n) { std::iota(p.begin(), p.end(), 0); }
  int64_t find(int64_t x) {
    while (p[(size_t)x] != x) {
      p[(size_t)x] = p[(size_t)p[(size_t)x]];
      x = p[(size_t)x];
    }
    return x;
  }
  void unite(int64_t a, int64_t b) {
    a = find(a);
    b = find(b);
    if (a != b) p[(size_t)std::max(a, b)] = std::min(a, b);
  }
};

bool valid_csr(int64_t M, int64_t N, const int64_t* row_ptr, const int32_t* col_idx) {
  if (M < 0 || N < 1 || N > 0x7fffffff || !row_ptr || row_ptr[0] != 0) return false;
  for (int64_t i = 0; i < M; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return false;
  if (row_ptr[M] > 0 && !col_idx) return false;
  for (int64_t e = 0; e < row_ptr[M]; ++e)
    if (col_idx[e] < 0 || col_idx[e] >= N) return false;
  return true;
}

}  // namespace

extern "C" {

qrk_status qrk_discover_blockangular(int64_t M, int64_t N, const int64_t* row_ptr, const int32_t* col_idx,
                                     int32_t nB, const int32_t* dense_cols, int64_t* row_perm, int32_t* col_perm,
                                     int32_t* ncol, int64_t* row_off, int32_t* K_out) {
  if (!valid_csr(M, N, row_ptr, col_idx) || nB < 0 || nB > QRK_MAX_DENSE_COLS || nB >= N ||
      (nB > 0 && !dense_cols) || !row_perm || !col_perm || !ncol || !row_off || !K_out)
    return QRK_EINVAL;
  std::vector<char> dense((size_t)N, 0);
  for (int32_t k = 0; k < nB; ++k) {
    if (dense_cols[k] < 0 || dense_cols[k] >= N || dense[(size_t)dense_cols[k]]) return QRK_EINVAL;
    dense[(size_t)dense_cols[k]] = 1;
  }
  // rows linked through each non-dense column: the first row that touches a column is its anchor
  Dsu dsu(M);
  std::vector<int64_t> anchor((size_t)N, -1);
  std::vector<char> has_local((size_t)M, 0);
  for (int64_t i = 0; i < M; ++i)
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int32_t c = col_idx[e];
      if (dense[(size_t)c]) continue;
      has_local[(size_t)i] = 1;
      if (anchor[(size_t)c] < 0)
        anchor[(size_t)c] = i;
      else
        dsu.unite(i, anchor[(size_t)c]);
    }
  // blocks in order of their smallest column: a column's block is its anchor's root; columns no
  // row touches are blocks of their own (no rows)
  std::vector<int64_t> root_block((size_t)M, -1);
  std::vector<std::vector<int32_t>> bcols;
  std::vector<int64_t> col_block((size_t)N, -1);
  for (int64_t c = 0; c < N; ++c) {
    if (dense[(size_t)c]) continue;
    int64_t b;
    if (anchor[(size_t)c] < 0) {
      b = (int64_t)bcols.size();
      bcols.emplace_back();
    } else {
      const int64_t r = dsu.find(anchor[(size_t)c]);
      if (root_block[(size_t)r] < 0) {
        root_block[(size_t)r] = (int64_t)bcols.size();
        bcols.emplace_back();
      }
      b = root_block[(size_t)r];
    }
    bcols[(size_t)b].push_back((int32_t)c);
    col_block[(size_t)c] = b;
  }
  const int64_t K = (int64_t)bcols.size();
  if (K < 1 || K > 0x7fffffff) return QRK_EINVAL;
  std::vector<std::vector<int64_t>> brows((size_t)K);
  std::vector<int64_t> orphans;
  for (int64_t i = 0; i < M; ++i) {
    if (has_local[(size_t)i])
      brows[(size_t)root_block[(size_t)dsu.find(i)]].push_back(i);
    else
      orphans.push_back(i);
  }
  // rows with only dense columns: the first blocks with room
  size_t next = 0;
  for (int64_t i : orphans) {
    while (next < (size_t)K && (int64_t)brows[next].size() >= QRK_MAX_BLOCK_ROWS) ++next;
    if (next == (size_t)K) return QRK_EINVAL;
    brows[next].push_back(i);
  }
  int64_t pos = 0, cpos = 0;
  row_off[0] = 0;
  for (int64_t b = 0; b < K; ++b) {
    if ((int64_t)bcols[(size_t)b].size() > QRK_MAX_BLOCK_COLS || (int64_t)brows[(size_t)b].size() > QRK_MAX_BLOCK_ROWS)
      return QRK_EINVAL;
    std::sort(brows[(size_t)b].begin(), brows[(size_t)b].end());
    for (int64_t i : brows[(size_t)b]) row_perm[pos++] = i;
    row_off[b + 1] = pos;
    for (int32_t c : bcols[(size_t)b]) col_perm[cpos++] = c;
    ncol[b] = (int32_t)bcols[(size_t)b].size();
  }
  for (int32_t k = 0; k < nB; ++k) col_perm[cpos++] = dense_cols[k];
  *K_out = (int32_t)K;
  return QRK_OK;
}

qrk_status qrk_discover_banded(int64_t M, int64_t N, const int64_t* row_ptr, const int32_t* col_idx,
                               int64_t* row_perm, int32_t* row_start, int32_t* w_out) {
  if (!valid_csr(M, N, row_ptr, col_idx) || !row_perm || !row_start || !w_out) return QRK_EINVAL;
  std::vector<int32_t> first((size_t)M), last((size_t)M);
  int64_t w = 1;
  for (int64_t i = 0; i < M; ++i) {
    if (row_ptr[i + 1] == row_ptr[i]) return QRK_EINVAL;  // an empty row has no place in a band
    int32_t lo = col_idx[row_ptr[i]], hi = lo;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      lo = std::min(lo, col_idx[e]);
      hi = std::max(hi, col_idx[e]);
    }
    first[(size_t)i] = lo;
    last[(size_t)i] = hi;
    w = std::max<int64_t>(w, (int64_t)hi - lo + 1);
  }
  if (w > QRK_MAX_BAND || w > N) return QRK_EINVAL;
  std::vector<int64_t> order((size_t)M);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return first[(size_t)a] < first[(size_t)b]; });
  for (int64_t k = 0; k < M; ++k) {
    row_perm[k] = order[(size_t)k];
    row_start[k] = (int32_t)std::min<int64_t>(first[(size_t)order[(size_t)k]], N - w);
  }
  *w_out = (int32_t)w;
  return QRK_OK;
}

}  // extern "C"
