// Build-kernel autotuner: decision table (see autotune.hip).
#pragma once

#include <string>

namespace gbl {

// gfx name of the current device ("gfx950"), part of every key
std::string tune_device_name();
// the recorded choice for key, or -1
int tune_lookup(const std::string& path, const std::string& key);
// record a choice (first one wins) and, with a path, append it to the file
void tune_store(const std::string& path, const std::string& key, int choice, const double* us, int n);

}  // namespace gbl
