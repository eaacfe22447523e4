// The autotuner's cache: an in-process map and an optional JSON file of the form
//   {"version": 1, "entries": {
//     "<key>": {"leaf_scale": 2, "leaf_queue": 1, "refine_scale": 1, "ms": 25.1},
//     ...}}
// written by this file and read back by it (the reader accepts exactly this layout).
#include "tune_cache.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

namespace qrk {

namespace {

std::mutex g_mu;
std::map<std::string, TuneChoice> g_map;
std::string g_path;
bool g_env_checked = false;

int64_t pow2_bucket(int64_t x) {
  int64_t b = 1;
  while (b < x) b <<= 1;
  return b;
}

// Reads the entries of a file written by save(); false on a malformed file.
bool load(const std::string& path, std::map<std::string, TuneChoice>& out) {
  std::ifstream f(path);
  if (!f) return true;  // no file yet: nothing remembered
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t at = s.find("\"entries\"");
  if (at == std::string::npos) return false;
  at = s.find('{', at);
  if (at == std::string::npos) return false;
  ++at;
  for (;;) {
    const size_t k0 = s.find('"', at);
    const size_t close = s.find('}', at);
    if (k0 == std::string::npos || (close != std::string::npos && close < k0)) break;  // end of entries
    const size_t k1 = s.find('"', k0 + 1);
    const size_t b0 = s.find('{', k1);
    const size_t b1 = s.find('}', b0);
    if (k1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) return false;
    const std::string key = s.substr(k0 + 1, k1 - k0 - 1);
    const std::string body = s.substr(b0 + 1, b1 - b0 - 1);
    TuneChoice c;
    auto field = [&](const char* name, double* v) {
      const size_t p = body.find(std::string("\"") + name + "\"");
      if (p == std::string::npos) return false;
      const size_t colon = body.find(':', p);
      if (colon == std::string::npos) return false;
      *v = std::strtod(body.c_str() + colon + 1, nullptr);
      return std::isfinite(*v);
    };
    double q = 1.0;
    if (!field("leaf_scale", &c.leaf_scale) || !field("leaf_queue", &q) || !field("refine_scale", &c.refine_scale))
      return false;
    field("ms", &c.ms);
    c.leaf_queue = q != 0.0 ? 1 : 0;
    out[key] = c;
    at = b1 + 1;
  }
  return true;
}

bool save(const std::string& path, const std::map<std::string, TuneChoice>& m) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "{\"version\": 1, \"entries\": {";
    bool first = true;
    char buf[256];
    for (const auto& kv : m) {
      std::snprintf(buf, sizeof(buf), "{\"leaf_scale\": %.17g, \"leaf_queue\": %d, \"refine_scale\": %.17g, \"ms\": %.6g}",
                    kv.second.leaf_scale, kv.second.leaf_queue, kv.second.refine_scale, kv.second.ms);
      f << (first ? "\n  \"" : ",\n  \"") << kv.first << "\": " << buf;
      first = false;
    }
    f << "\n}}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

void check_env_locked() {
  if (g_env_checked) return;
  g_env_checked = true;
  const char* env = std::getenv("QRK_TUNE_CACHE");
  if (g_path.empty() && env && *env) {
    g_path = env;
    (void)load(g_path, g_map);
  }
}

}  // namespace

std::string tune_key(const char* arch, int dtype, int mode, int P, int n, int64_t rows, int max_L, int widths) {
  char buf[160];
  std::snprintf(buf, sizeof(buf), "%s/%s/%s/P%lld/n%d/rows%lld/L%d/w%d", arch, dtype == 0 ? "f32" : "f64",
                mode == 0 ? "plain" : "bf16x3", (long long)(P <= 8 ? P : pow2_bucket(P)), n,
                (long long)pow2_bucket(rows > 0 ? rows : 1), max_L, widths);
  return buf;
}

bool tune_lookup(const std::string& key, TuneChoice* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  check_env_locked();
  auto it = g_map.find(key);
  if (it == g_map.end()) return false;
  *out = it->second;
  return true;
}

bool tune_store(const std::string& key, const TuneChoice& c) {
  std::lock_guard<std::mutex> lk(g_mu);
  check_env_locked();
  g_map[key] = c;
  return g_path.empty() || save(g_path, g_map);
}

bool tune_set_file(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_env_checked = true;
  g_path = path ? path : "";
  return g_path.empty() || load(g_path, g_map);
}

}  // namespace qrk
