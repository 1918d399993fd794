// Device allocation of the library and the caller-allocator contexts.
#include "engine.h"

namespace hssx {

namespace {
thread_local hssx_ctx_ *g_scope = nullptr;
thread_local void *g_scope_stream = nullptr;
}  // namespace

AllocScope::AllocScope(hssx_ctx_ *ctx, void *stream) : prev(g_scope), prev_stream(g_scope_stream) {
  g_scope = ctx;
  g_scope_stream = stream;
}
AllocScope::~AllocScope() {
  g_scope = prev;
  g_scope_stream = prev_stream;
}
hssx_ctx_ *alloc_scope() { return g_scope; }

void *dev_alloc(size_t bytes, hssx_ctx_ **owner) {
  hssx_ctx_ *c = g_scope;
  void *p = nullptr;
  if (c) {
    p = c->a.alloc(bytes, g_scope_stream, c->a.user);
    if (!p) throw Error(HSSX_ENOMEM, "the context's allocator refused " + std::to_string(bytes) + " bytes");
    c->live_bytes += (long)bytes;
    c->allocs += 1;
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess)
      throw Error(HSSX_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  *owner = c;
  return p;
}

void dev_free(void *p, size_t bytes, hssx_ctx_ *owner) {
  if (owner) {
    owner->a.free(p, bytes, g_scope == owner ? g_scope_stream : nullptr, owner->a.user);
    owner->live_bytes -= (long)bytes;
    owner->frees += 1;
  } else {
    (void)hipFree(p);
  }
}

}  // namespace hssx
