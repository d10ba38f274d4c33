// Optional HIP-event timing of kernel launches (fit_profile_start/stop).
#pragma once

#include "fit_internal.h"

namespace fit {

// Returns a token (>= 0) if profiling is on, after recording a start event
// on stream s; pass it to prof_end after the launch.
int prof_begin(hipStream_t s);
void prof_end(int token, hipStream_t s, const char* name);

}  // namespace fit
