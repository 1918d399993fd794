// Device workspace of the allocation-free apply (hssx_apply_noalloc): one
// file-scope array per device, held until the process ends.  Host code uses
// only the address hipGetSymbolAddress returns for the current device, never
// the array's name.
#include <map>
#include <mutex>

#include "engine.h"

namespace hssx {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, char *> g_ptr;   // device -> address of that device's copy

}  // namespace

char *noalloc_workspace(size_t *bytes) {
  int dev = 0;
  HSSX_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_ptr.find(dev);
  if (it == g_ptr.end()) {
    char *ptr = nullptr;
    HSSX_HIP(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
    HSSX_CHECK(ptr != nullptr, HSSX_EHIP, "no device address for the apply workspace");
    it = g_ptr.emplace(dev, ptr).first;
  }
  *bytes = kScratchBytes;
  return it->second;
}

}  // namespace hssx
