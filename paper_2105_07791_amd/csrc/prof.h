// Optional per-kernel timing with HIP events recorded on the launching
// stream.  Off by default; when on, launchers bracket selected kernels and
// record the algorithmic work (flops or bytes) of each launch.
#pragma once

#include "common.h"

namespace hssx {

bool prof_on();
void prof_enable(bool on);
// returns an event recorded on st (or null when profiling is off)
hipEvent_t prof_begin(hipStream_t st);
void prof_end(const char *kernel, hipStream_t st, hipEvent_t begin, double work);
// totals over the recorded launches of `kernel` (synchronises their events)
void prof_query(const char *kernel, double *ms, long *launches, double *work);

}  // namespace hssx
