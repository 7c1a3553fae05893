// Persistent cache of the autotuners' choices. The file is a JSON object with
// one entry per line,
//   "<key>": [a, b, ms],
// where the key names the tuned kernel or build, the device and the node set
// (its size, stencil count and whatever else changes the choice) and a, b
// are the choice (lanes per node and flags of a gather kernel, or the mode
// and workgroups per CU of the build).
#include "tune_cache.hpp"

#include <hip/hip_runtime.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <utility>

namespace labfm {
namespace {

using Table = std::map<std::string, std::pair<std::pair<int, int>, double>>;

// Parses the entries of a cache file; lines that do not hold an entry are
// skipped.
Table read_table(const std::string& path) {
  Table t;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return t;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const char* p = std::strchr(line, '"');
    if (!p) continue;
    const char* q = std::strchr(p + 1, '"');
    if (!q) continue;
    std::string key(p + 1, q);
    const char* r = std::strchr(q + 1, '[');
    if (!r) continue;
    char* end = nullptr;
    const long a = std::strtol(r + 1, &end, 10);
    if (end == r + 1 || *end != ',') continue;
    const char* s2 = end + 1;
    const long b = std::strtol(s2, &end, 10);
    if (end == s2 || *end != ',') continue;
    const char* s3 = end + 1;
    const double ms = std::strtod(s3, &end);
    if (end == s3) continue;
    t[key] = {{static_cast<int>(a), static_cast<int>(b)}, ms};
  }
  std::fclose(f);
  return t;
}

}  // namespace

std::string tune_cache_path(const char* given) {
  if (given && *given) return given;
  const char* env = std::getenv("LABFM_TUNE_CACHE");
  return env ? std::string(env) : std::string();
}

std::string tune_device_key() {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  return std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

bool tune_cache_lookup(const std::string& path, std::vector<TuneEntry>& want) {
  if (path.empty()) return false;
  const Table t = read_table(path);
  for (auto& e : want) {
    auto it = t.find(e.key);
    if (it == t.end()) return false;
    e.a = it->second.first.first;
    e.b = it->second.first.second;
    e.ms = it->second.second;
  }
  return true;
}

bool tune_cache_store(const std::string& path, const std::vector<TuneEntry>& entries,
                      std::string& err) {
  Table t = read_table(path);
  for (const auto& e : entries) t[e.key] = {{e.a, e.b}, e.ms};
  const std::string tmp = path + ".tmp." + std::to_string(static_cast<long>(getpid()));
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) {
    err = "cannot write " + tmp + ": " + std::strerror(errno);
    return false;
  }
  std::fputs("{\n", f);
  size_t k = 0;
  for (const auto& kv : t) {
    std::fprintf(f, " \"%s\": [%d, %d, %.6g]%s\n", kv.first.c_str(), kv.second.first.first,
                 kv.second.first.second, kv.second.second, ++k < t.size() ? "," : "");
  }
  std::fputs("}\n", f);
  const bool ok = std::fflush(f) == 0;
  std::fclose(f);
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
    err = "cannot replace " + path + ": " + std::strerror(errno);
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace labfm
