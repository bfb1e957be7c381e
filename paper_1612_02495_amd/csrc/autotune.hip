// Autotuner: times the real phase kernels over candidate (engine, tile width,
// steps per cycle) configurations and keeps the fastest per (kind, dtype, n).
// The paper picks, for every problem size, the best of all power-of-two block
// sizes from 32 to 1024 (Sec. 5); this does the same search on the swept
// kernels of this library, plus the engine and the phase height.
//
// Results live in an in-process table and, when SWEPT_AUTOTUNE_CACHE names a
// file, in a small JSON document there (read on lookup, rewritten atomically
// on update).
#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "swept.h"

namespace swept {

namespace {

using Key = std::tuple<int, int, int64_t>;
std::mutex g_mu;
std::map<Key, TuneEntry> g_table;

const char* cache_path() {
  const char* p = std::getenv("SWEPT_AUTOTUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// Minimal reader for the cache documents this file writes: a list of flat
// objects with numeric fields.
bool find_number(const std::string& obj, const char* key, double* out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t at = obj.find(k);
  if (at == std::string::npos) return false;
  at = obj.find(':', at + k.size());
  if (at == std::string::npos) return false;
  const char* s = obj.c_str() + at + 1;
  char* end = nullptr;
  errno = 0;
  const double v = std::strtod(s, &end);
  if (end == s || errno != 0) return false;
  *out = v;
  return true;
}

std::map<Key, TuneEntry> read_cache_file(const char* path) {
  std::map<Key, TuneEntry> out;
  FILE* f = std::fopen(path, "rb");
  if (!f) return out;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  size_t pos = text.find("\"entries\"");
  if (pos == std::string::npos) return out;
  while (true) {
    const size_t a = text.find('{', pos);
    if (a == std::string::npos) break;
    const size_t b = text.find('}', a);
    if (b == std::string::npos) break;
    const std::string obj = text.substr(a, b - a + 1);
    pos = b + 1;
    double kind, dtype, n, w, spc, eng, ns = 0.0;
    if (!find_number(obj, "kind", &kind) || !find_number(obj, "dtype", &dtype) || !find_number(obj, "n", &n) ||
        !find_number(obj, "tile_width", &w) || !find_number(obj, "steps_per_cycle", &spc) ||
        !find_number(obj, "engine", &eng))
      continue;
    find_number(obj, "ns_per_cell_update", &ns);
    TuneEntry e;
    e.tile_width = (int)w;
    e.steps_per_cycle = (int)spc;
    e.engine = (int)eng;
    e.ns_per_cell_update = ns;
    out[Key((int)kind, (int)dtype, (int64_t)n)] = e;
  }
  return out;
}

bool write_cache_file(const char* path, const std::map<Key, TuneEntry>& table) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  std::fprintf(f, "{\"swept_autotune\": 1, \"entries\": [\n");
  size_t i = 0;
  for (const auto& kv : table) {
    const TuneEntry& e = kv.second;
    std::fprintf(f,
                 "  {\"kind\": %d, \"dtype\": %d, \"n\": %lld, \"tile_width\": %d, \"steps_per_cycle\": %d, "
                 "\"engine\": %d, \"ns_per_cell_update\": %.9g}%s\n",
                 std::get<0>(kv.first), std::get<1>(kv.first), (long long)std::get<2>(kv.first), e.tile_width,
                 e.steps_per_cycle, e.engine, e.ns_per_cell_update, ++i < table.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

bool tune_lookup(int kind, int dtype, int64_t n, TuneEntry* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  const Key key(kind, dtype, n);
  auto it = g_table.find(key);
  if (it != g_table.end()) {
    *out = it->second;
    return true;
  }
  if (const char* p = cache_path()) {
    auto file = read_cache_file(p);
    auto jt = file.find(key);
    if (jt != file.end()) {
      g_table[key] = jt->second;
      *out = jt->second;
      return true;
    }
  }
  return false;
}

bool tune_store(int kind, int dtype, int64_t n, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_mu);
  const Key key(kind, dtype, n);
  g_table[key] = e;
  if (const char* p = cache_path()) {
    auto file = read_cache_file(p);
    file[key] = e;
    return write_cache_file(p, file);
  }
  return true;
}

void tune_forget_all() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
}

}  // namespace swept
