// Launch-shape choices of the block-angular autotuner, kept per device architecture and batch
// shape bucket in the process and, when a cache file is set (qrk_tune_cache_file or the
// QRK_TUNE_CACHE environment variable), in a JSON file that later processes read back.
// Host-only.
#pragma once

#include <stdint.h>

#include <string>

namespace qrk {

struct TuneChoice {
  double leaf_scale = 1.0;    // multiplies the default rows per dense-part leaf
  int leaf_queue = 1;         // batches of several widths: one persistent leaf launch (1) or one per width (0)
  double refine_scale = 1.0;  // multiplies the default refinement workgroup count
  double ms = 0.0;            // the measured factor + one-sweep solve time of the choice
};

// "arch/dtype/mode/P/n/rows/L/widths" with P and the row count bucketed by powers of two.
std::string tune_key(const char* arch, int dtype, int mode, int P, int n, int64_t rows, int max_L, int widths);
bool tune_lookup(const std::string& key, TuneChoice* out);
// Remembers the choice in the process and rewrites the cache file (when one is set); returns
// false if the file could not be written.
bool tune_store(const std::string& key, const TuneChoice& c);
// Sets (path != nullptr) or clears the cache file and loads its entries; false if a file that
// exists could not be parsed.
bool tune_set_file(const char* path);

}  // namespace qrk
