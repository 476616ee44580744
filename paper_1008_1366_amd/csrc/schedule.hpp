// schedule.hpp -- process-wide cache of autotuned schedules (schedule.hip).
#pragma once
#include <stdint.h>

#include <string>

namespace impconv {

// Architecture name of the current device ("gfx950"), "unknown" on failure.
std::string device_arch();
// Recorded choice for (arch, variant, dtype, N); false if none.
bool sched_lookup(const std::string& arch, const char* variant, int dt, int64_t N, int64_t* choice, double* ms);
// Records (or replaces) the choice and its measured time in milliseconds.
void sched_store(const std::string& arch, const char* variant, int dt, int64_t N, int64_t choice, double ms);

}  // namespace impconv
