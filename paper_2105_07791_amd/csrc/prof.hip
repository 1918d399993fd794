#include "prof.h"

#include <mutex>

namespace hssx {

namespace {
struct Rec {
  std::string name;
  hipEvent_t a, b;
  double work;
};
std::mutex g_mu;
std::vector<Rec> g_recs;
bool g_on = false;
}  // namespace

bool prof_on() { return g_on; }

void prof_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto &r : g_recs) {
    (void)hipEventSynchronize(r.b);
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_recs.clear();
  g_on = on;
}

hipEvent_t prof_begin(hipStream_t st) {
  if (!g_on) return nullptr;
  // launches recorded into a graph are not timed one by one (an event
  // captured into a graph has no elapsed time of its own)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return nullptr;
  hipEvent_t e;
  HSSX_HIP(hipEventCreate(&e));
  HSSX_HIP(hipEventRecord(e, st));
  return e;
}

void prof_end(const char *kernel, hipStream_t st, hipEvent_t begin, double work) {
  if (!g_on || !begin) return;
  hipEvent_t e;
  HSSX_HIP(hipEventCreate(&e));
  HSSX_HIP(hipEventRecord(e, st));
  std::lock_guard<std::mutex> lk(g_mu);
  g_recs.push_back(Rec{kernel, begin, e, work});
}

void prof_query(const char *kernel, double *ms, long *launches, double *work) {
  std::lock_guard<std::mutex> lk(g_mu);
  double t = 0, w = 0;
  long n = 0;
  for (auto &r : g_recs) {
    if (r.name != kernel) continue;
    HSSX_HIP(hipEventSynchronize(r.b));
    float x = 0;
    HSSX_HIP(hipEventElapsedTime(&x, r.a, r.b));
    t += x;
    w += r.work;
    ++n;
  }
  if (ms) *ms = t;
  if (launches) *launches = n;
  if (work) *work = w;
}

}  // namespace hssx
