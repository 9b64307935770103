// Measured choice of launch parameters (autotuning), cached per device.
#pragma once
#include <functional>
#include <string>
#include <vector>

#include "internal.hpp"

namespace afsbem {

// Returns the candidate with the shortest measured time for (kernel, n,
// variant) on the current device.  On the first request run(c) enqueues the
// complete operation for candidate c on st; each candidate is run once to warm
// up and then timed over `reps` runs with HIP events.  Returns `fallback`
// without measuring when tuning is switched off or st is being captured.
int autotune(const char *kernel, int64_t n, int variant, const std::vector<int> &cands, hipStream_t st,
             const std::function<void(int)> &run, int fallback, int reps = 3);

void autotune_set_enabled(bool on);
std::string autotune_report();

}  // namespace afsbem
