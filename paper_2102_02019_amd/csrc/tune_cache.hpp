// Persistent cache of the autotuners' choices (labfm_tune, labfm_tune_build).
#pragma once

#include <string>
#include <vector>

namespace labfm {

// One tuned choice: two integers (a launch shape, or a build distribution)
// and the duration it was measured at.
struct TuneEntry {
  std::string key;
  int a = 0, b = 0;
  double ms = 0.0;
};

// The cache file of a tuner call: `given` when not NULL or empty, else the
// LABFM_TUNE_CACHE environment variable, else "" (no cache).
std::string tune_cache_path(const char* given);

// Identity of the current device in cache keys: its architecture and
// compute-unit count (e.g. "gfx950:sramecc+:xnack-/256cu").
std::string tune_device_key();

// Looks up every key of `want` (filling a, b, ms); true only when all are
// present. A missing or unreadable file is a miss.
bool tune_cache_lookup(const std::string& path, std::vector<TuneEntry>& want);

// Adds or replaces the entries in the file (written to a temporary file in
// the same directory, then renamed over it). Returns false with a message in
// `err` when the file cannot be written.
bool tune_cache_store(const std::string& path, const std::vector<TuneEntry>& entries,
                      std::string& err);

}  // namespace labfm
