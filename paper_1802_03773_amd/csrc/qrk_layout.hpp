// Host-side layout rules of the block-angular workspace.
#pragma once

#include <cstdint>

namespace qrk {

// Row stride (elements) of the reduced rows for L columns of es-byte elements: a multiple of 128
// bytes when that costs at most 1/16 more than the smallest multiple of 4, so that no two blocks'
// rows share a cache line and the per-block QR writes whole lines; else a multiple of 4.
inline int64_t reduced_row_stride(int64_t L, int64_t es) {
  const int64_t line = 128 / es;
  const int64_t s4 = ((L + 3) / 4) * 4;
  const int64_t sl = ((L + line - 1) / line) * line;
  return sl * 16 <= s4 * 17 ? sl : s4;
}

}  // namespace qrk
