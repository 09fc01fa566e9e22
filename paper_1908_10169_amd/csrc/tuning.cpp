// Tuned kernel settings: a process-wide table loaded from the JSON file the
// project's tuner (paper_1908_10169_amd/tune.py) writes.  An entry holds,
// for one update precision and one block-width class of the initial
// partition, the settings that measured fastest: workers per CU of the
// factor sweep, matrix-core update tiles, the staging path of narrow
// blocks, the apply path and the accumulation order.  Entries for handles
// that require run-to-run reproducible results (reproducible = 1) always
// keep the ordered accumulation; entries for handles that do not may drop
// it where that measured faster.
#include <dlfcn.h>

#include <cctype>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace bilu {
namespace {

std::mutex g_tune_mu;
std::vector<TunedEntry> g_tune;

// The value of "key": <number> inside one JSON object's text, or fallback.
double field(const std::string& obj, const char* key, double fallback) {
  const std::string pat = std::string("\"") + key + "\"";
  size_t p = obj.find(pat);
  if (p == std::string::npos) return fallback;
  p = obj.find(':', p + pat.size());
  if (p == std::string::npos) return fallback;
  ++p;
  while (p < obj.size() && std::isspace((unsigned char)obj[p])) ++p;
  char* end = nullptr;
  const double v = std::strtod(obj.c_str() + p, &end);
  return end == obj.c_str() + p ? fallback : v;
}

}  // namespace

// The table shipped beside the library for this device's architecture
// (tuning/<gfx...>.json next to libbilu.so), loaded once per process on the
// first lookup unless a table was loaded explicitly.
bool g_tune_tried = false;
void load_default_table() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return;
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  Dl_info info;
  if (!dladdr(reinterpret_cast<void*>(&load_default_table), &info) || !info.dli_fname) return;
  std::string dir(info.dli_fname);
  const size_t slash = dir.rfind('/');
  dir = slash == std::string::npos ? std::string(".") : dir.substr(0, slash);
  const std::string path = dir + "/tuning/" + arch + ".json";
  FILE* fp = std::fopen(path.c_str(), "rb");
  if (!fp) return;
  std::fclose(fp);
  (void)bilu_load_tuning(path.c_str());
}

bool tuned_entry(int precision, int width_class, int reproducible, TunedEntry* out) {
  bool first = false;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    first = !g_tune_tried;
    g_tune_tried = true;
  }
  if (first) load_default_table();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const TunedEntry& e : g_tune)
    if (e.precision == precision && e.width_class == width_class &&
        e.reproducible == reproducible) {
      *out = e;
      return true;
    }
  return false;
}

}  // namespace bilu

using namespace bilu;

extern "C" bilu_status bilu_load_tuning(const char* path) {
  try {
    std::vector<TunedEntry> table;
    if (path && *path) {
      FILE* fp = std::fopen(path, "rb");
      if (!fp) return BILU_ERR_INVALID;
      std::string text;
      char buf[4096];
      size_t got;
      while ((got = std::fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, got);
      std::fclose(fp);
      const size_t arr = text.find("\"entries\"");
      if (arr == std::string::npos) return BILU_ERR_INVALID;
      size_t p = text.find('[', arr);
      if (p == std::string::npos) return BILU_ERR_INVALID;
      // the objects of the entries array (flat: no nested objects)
      while (true) {
        const size_t a = text.find_first_of("{]", p);
        if (a == std::string::npos) return BILU_ERR_INVALID;
        if (text[a] == ']') break;
        const size_t b = text.find('}', a);
        if (b == std::string::npos) return BILU_ERR_INVALID;
        const std::string obj = text.substr(a, b - a + 1);
        TunedEntry e;
        e.precision = (int)field(obj, "precision", -1);
        e.width_class = (int)field(obj, "width_class", -1);
        e.workers_per_cu = (int)field(obj, "workers_per_cu", 0);
        e.update_mfma = (int)field(obj, "update_mfma", 0);
        e.factor_path = (int)field(obj, "factor_path", 0);
        e.apply_path = (int)field(obj, "apply_path", 0);
        e.deterministic = (int)field(obj, "deterministic", 1);
        e.reproducible = (int)field(obj, "reproducible", 1);
        if (e.precision < 0 || e.precision > 2 || e.width_class < 0 || e.width_class > 1 ||
            e.workers_per_cu < 0 || e.workers_per_cu > 8 || e.update_mfma < 0 ||
            e.update_mfma > 1 || e.factor_path < 0 || e.factor_path > 2 || e.apply_path < 0 ||
            e.apply_path > 2 || e.deterministic < 0 || e.deterministic > 1 ||
            e.reproducible < 0 || e.reproducible > 1 || (e.reproducible && !e.deterministic))
          return BILU_ERR_INVALID;
        table.push_back(e);
        p = b + 1;
      }
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.swap(table);
    g_tune_tried = true;  // an explicit table replaces the shipped one
    return BILU_OK;
  } catch (...) {
    return BILU_ERR_INTERNAL;
  }
}

extern "C" int64_t bilu_tuning_entries(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return (int64_t)g_tune.size();
}
