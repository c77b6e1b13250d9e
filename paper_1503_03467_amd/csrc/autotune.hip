// Build-kernel autotuner: the choice between the kernel variants of a build
// step (dense patch solves on the vector units or the matrix cores, the band
// patch solves of the finest level in registers or in LDS, the Galerkin
// product per coarse row or on strips) is made by timing every candidate on
// the level at hand and kept per (device, precision, level shape) in a
// process-wide table, optionally backed by a text file that later processes
// read: one line per decision, "<key> <choice> <time of candidate 0 in us>
// <time of candidate 1 in us>" (-1 for a candidate that does not apply).
#include "autotune.hpp"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

namespace gbl {

namespace {

std::mutex g_tune_mu;
std::map<std::string, std::map<std::string, int>> g_tables;   // path ("" = this process only) -> key -> choice

std::map<std::string, int>& table_for(const std::string& path) {
  auto it = g_tables.find(path);
  if (it != g_tables.end()) return it->second;
  std::map<std::string, int>& t = g_tables[path];
  if (!path.empty()) {
    if (FILE* f = std::fopen(path.c_str(), "r")) {
      char line[512];
      while (std::fgets(line, sizeof line, f)) {
        std::istringstream is(line);
        std::string key;
        int choice = -1;
        if (is >> key >> choice && choice >= 0) t[key] = choice;
      }
      std::fclose(f);
    }
  }
  return t;
}

}  // namespace

std::string tune_device_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string name = prop.gcnArchName;
  const size_t colon = name.find(':');
  return colon == std::string::npos ? name : name.substr(0, colon);
}

int tune_lookup(const std::string& path, const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const auto& t = table_for(path);
  const auto it = t.find(key);
  return it == t.end() ? -1 : it->second;
}

void tune_store(const std::string& path, const std::string& key, int choice, const double* us, int n) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto& t = table_for(path);
  if (t.count(key)) return;
  t[key] = choice;
  if (path.empty()) return;
  if (FILE* f = std::fopen(path.c_str(), "a")) {
    std::fprintf(f, "%s %d", key.c_str(), choice);
    for (int i = 0; i < n; ++i) std::fprintf(f, " %.2f", us[i]);
    std::fprintf(f, "\n");
    std::fclose(f);
  }
}

}  // namespace gbl
