// Internal shared definitions of the hssx library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <algorithm>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hssx.h"

namespace hssx {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  hssx_status code;
  Error(hssx_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HSSX_HIP(expr)                                                        \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::hssx::Error(HSSX_EHIP, std::string(#expr) + ": " +              \
                                         hipGetErrorString(e_));              \
  } while (0)

#define HSSX_CHECK(cond, code, msg)                                           \
  do {                                                                        \
    if (!(cond)) throw ::hssx::Error(code, msg);                              \
  } while (0)

// ---------------------------------------------------------------- complex
template <typename T> struct cplx {
  T re, im;
};
using c64 = cplx<float>;
using c128 = cplx<double>;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) {
  cplx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) {
  return mk(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) {
  return mk(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a) {
  return mk(-a.re, -a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> b) {
  return mk(s * b.re, s * b.im);
}
// a += b * c
template <typename T>
__host__ __device__ __forceinline__ void cfma(cplx<T> &a, cplx<T> b, cplx<T> c) {
  a.re += b.re * c.re - b.im * c.im;
  a.im += b.re * c.im + b.im * c.re;
}
// a -= b * c
template <typename T>
__host__ __device__ __forceinline__ void cfms(cplx<T> &a, cplx<T> b, cplx<T> c) {
  a.re -= b.re * c.re - b.im * c.im;
  a.im -= b.re * c.im + b.im * c.re;
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> conj(cplx<T> a) {
  return mk(a.re, -a.im);
}
template <typename T>
__host__ __device__ __forceinline__ T abs2(cplx<T> a) {
  return a.re * a.re + a.im * a.im;
}
// |re| + |im|: the pivot magnitude used by partial pivoting (LAPACK cabs1)
template <typename T>
__host__ __device__ __forceinline__ T cabs1(cplx<T> a) {
  return fabs(a.re) + fabs(a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cinv(cplx<T> a) {
  // Smith-free scaled reciprocal: 1/(a) = conj(a)/|a|^2 with scaling by the
  // larger component to avoid overflow/underflow.
  T s = fmax(fabs(a.re), fabs(a.im));
  T ar = a.re / s, ai = a.im / s;
  T d = s * (ar * ar + ai * ai);
  return mk(ar / d, -ai / d);
}
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cplx<To> ccast(cplx<Ti> a) {
  return mk((To)a.re, (To)a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> czero() {
  return mk((T)0, (T)0);
}

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads()
// it does not wait for the workgroup's outstanding global stores, so loops
// that write results to global memory every step do not stall on them.  Use
// it only where the other threads read nothing but LDS after the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Cross-lane moves within rows of 16 lanes on the VALU (DPP) instead of the
// LDS crossbar: xor 1 and xor 2 inside quads, the reversal of 8 lanes and the
// reversal of 16 lanes.  A sum or an argmax over a group of 8 or 16
// consecutive lanes is the quad butterflies followed by the reversals.
enum : int { kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };
template <int CTRL> __device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ int dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ double dpp(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// sum over aligned groups of G lanes (G = 1, 2, 4, 8 or 16), result in every lane
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
  if (G >= 2) v += dpp<kDppXor1>(v);
  if (G >= 4) v += dpp<kDppXor2>(v);
  if (G >= 8) v += dpp<kDppHalfMirror>(v);
  if (G >= 16) v += dpp<kDppMirror>(v);
  return v;
}
// one lane's value, read into a scalar register (every lane gets it)
__device__ __forceinline__ float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ int lane_value(int v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}
__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// argmax (ties: smaller index) over the whole wavefront, result in every
// lane: DPP butterflies within each row of 16 lanes, then the four rows'
// results compared through scalar reads of one lane per row (no LDS round
// trip).  Every lane of the wavefront must be active.
template <typename T> __device__ __forceinline__ void wave_argmax(T &v, int &idx) {
  auto step = [&](T ov, int oi) {
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  };
  step(dpp<kDppXor1>(v), dpp<kDppXor1>(idx));
  step(dpp<kDppXor2>(v), dpp<kDppXor2>(idx));
  step(dpp<kDppHalfMirror>(v), dpp<kDppHalfMirror>(idx));
  step(dpp<kDppMirror>(v), dpp<kDppMirror>(idx));
  T bv = lane_value(v, 0);
  int bi = lane_value(idx, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const T ov = lane_value(v, 16 * r);
    const int oi = lane_value(idx, 16 * r);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  v = bv;
  idx = bi;
}

// ---------------------------------------------------------------- memory
}  // namespace hssx
struct hssx_ctx_;
namespace hssx {

// Device memory of the library: taken from the allocator of the allocation
// scope's context when one is active on the calling thread (AllocScope),
// else from hipMalloc.  *owner receives the context that must free it.
void *dev_alloc(size_t bytes, hssx_ctx_ **owner);
void dev_free(void *p, size_t bytes, hssx_ctx_ *owner);

// The context (and stream) whose allocator serves this thread's device
// allocations while the scope lives; scopes nest.
struct AllocScope {
  hssx_ctx_ *prev;
  void *prev_stream;
  AllocScope(hssx_ctx_ *ctx, void *stream);
  ~AllocScope();
  AllocScope(const AllocScope &) = delete;
  AllocScope &operator=(const AllocScope &) = delete;
};
hssx_ctx_ *alloc_scope();

// Device buffer owned by the library (RAII, not copyable).
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  hssx_ctx_ *owner = nullptr;   // context whose allocator it came from
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), owner(o.owner) {
    o.p = nullptr; o.bytes = 0; o.owner = nullptr;
  }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; owner = o.owner;
      o.p = nullptr; o.bytes = 0; o.owner = nullptr;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 16;
    p = dev_alloc(b, &owner);
    bytes = b;
  }
  void release() {
    if (p) dev_free(p, bytes, owner);
    p = nullptr;
    bytes = 0;
    owner = nullptr;
  }
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// Blocking upload of set-up data (symbolic schedules); never in a timed loop.
template <typename T>
inline void upload(DevBuf &d, const std::vector<T> &h) {
  d.alloc(h.size() * sizeof(T));
  if (!h.empty())
    HSSX_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Device scratch arena: bump allocation from chunks that stay allocated and
// are reused.  release(mark) frees everything allocated after the mark; call
// it only once the stream has finished every use of that memory.
class Arena {
 public:
  struct Mark {
    size_t chunk, off;
  };
  Mark mark() const { return Mark{cur_, off_}; }
  void release(Mark m) {
    cur_ = m.chunk;
    off_ = m.off;
  }
  template <typename T> T *get(size_t count) {
    size_t need = ((std::max<size_t>(1, count * sizeof(T)) + 255) / 256) * 256;
    while (cur_ < chunks_.size() && off_ + need > chunks_[cur_]->bytes) {
      if (off_ == 0) {
        // an unused chunk that is too small: give its memory back (every
        // chunk from cur_ on is unused by the host; kernels queued before a
        // release may still read it, so the device is drained first)
        HSSX_HIP(hipDeviceSynchronize());
        chunks_.erase(chunks_.begin() + cur_);
        continue;
      }
      ++cur_;
      off_ = 0;
    }
    if (cur_ == chunks_.size()) {
      auto c = std::make_unique<DevBuf>();
      c->alloc(std::max(need, size_t(64) << 20));
      chunks_.push_back(std::move(c));
      off_ = 0;
    }
    T *p = reinterpret_cast<T *>(static_cast<char *>(chunks_[cur_]->p) + off_);
    off_ += need;
    return p;
  }

 private:
  std::vector<std::unique_ptr<DevBuf>> chunks_;
  size_t cur_ = 0, off_ = 0;
};

// Arenas kept per device between factorizations (a factorization takes one
// for its duration and returns it, so concurrent calls never share one).
std::unique_ptr<Arena> acquire_arena(int device);
void return_arena(int device, std::unique_ptr<Arena> a);

// Stream-ordered upload of small descriptor arrays: host data is copied into
// pinned chunks and sent with hipMemcpyAsync on the work stream, so uploads
// block neither the host nor the device.  Chunks are never freed or
// overwritten while their device copies may still be read; recycle() reuses
// them and may only be called after the stream has been synchronised and
// once no pointer returned by put() is used again.
class Staging;
// Pinned staging areas kept per device between factorizations, like arenas.
std::unique_ptr<Staging> acquire_staging(int device, hipStream_t st);
void return_staging(int device, std::unique_ptr<Staging> s);

class Staging {
 public:
  explicit Staging(hipStream_t st) : st_(st) {}
  Staging(const Staging &) = delete;
  Staging &operator=(const Staging &) = delete;
  ~Staging() {
    for (auto &c : chunks_)
      if (c.host) (void)hipHostFree(c.host);
  }
  // v uploaded; kernels may write to the device copy (a counter, a queue)
  template <typename T> T *put(const std::vector<T> &v) { return place(v, false); }
  // v uploaded for reading only: when the same bytes already sit at this
  // position on both sides from an upload known to have landed (synced()),
  // the copy is skipped (repeated factorizations of one pattern stage
  // identical job arrays at identical positions)
  template <typename T> T *put_const(const std::vector<T> &v) { return place(v, true); }
  // the stream has been synchronised: every copy issued so far has landed
  // and its bytes can be trusted by later put_const calls at that position
  void synced() {
    for (auto &c : chunks_)
      for (auto &g : c.state)
        if (g == kPending) g = kClean;
  }
  // start again at the first position (after a synchronisation, once no
  // pointer returned before is used again); uploads not followed by
  // synced() are forgotten
  void recycle() {
    for (auto &c : chunks_)
      for (auto &g : c.state)
        if (g == kPending) g = kUnknown;
    cur_ = 0;
    off_ = 0;
  }
  // bytes placed since the last recycle
  size_t used() const {
    size_t b = off_;
    for (size_t c = 0; c < cur_ && c < chunks_.size(); ++c) b += chunks_[c].cap;
    return b;
  }
  void set_stream(hipStream_t st) { st_ = st; }
  hipStream_t stream() const { return st_; }

 private:
  static constexpr size_t kGran = 256;
  // per granule: device bytes unknown (or writable by kernels), uploaded
  // since the last recycle, or equal to the host bytes
  enum : unsigned char { kUnknown = 0, kPending = 1, kClean = 2 };
  struct Chunk {
    void *host = nullptr;
    std::unique_ptr<DevBuf> dev;
    size_t cap = 0;
    std::vector<unsigned char> state;
  };
  template <typename T> T *place(const std::vector<T> &v, bool read_only) {
    size_t bytes = v.size() * sizeof(T);
    size_t need = ((bytes + kGran - 1) / kGran) * kGran;
    if (need == 0) need = kGran;
    while (cur_ < chunks_.size() && off_ + need > chunks_[cur_].cap) {
      ++cur_;
      off_ = 0;
    }
    if (cur_ == chunks_.size()) {
      Chunk c;
      c.cap = std::max(need, size_t(8) << 20);
      HSSX_HIP(hipHostMalloc(&c.host, c.cap, hipHostMallocDefault));
      c.dev = std::make_unique<DevBuf>();
      c.dev->alloc(c.cap);
      c.state.assign(c.cap / kGran, kUnknown);
      chunks_.push_back(std::move(c));
      off_ = 0;
    }
    Chunk &c = chunks_[cur_];
    char *h = static_cast<char *>(c.host) + off_;
    char *d = static_cast<char *>(c.dev->p) + off_;
    const size_t g0 = off_ / kGran, g1 = (off_ + need) / kGran;
    if (bytes) {
      bool same = read_only;
      for (size_t g = g0; same && g < g1; ++g) same = c.state[g] == kClean;
      same = same && std::memcmp(h, v.data(), bytes) == 0;
      if (!same) {
        // whole granules go up (the tail of the last one zeroed): a granule
        // marked clean then equals its host image in every byte, also where a
        // later placement at a shifted offset reaches past this one's end
        std::memcpy(h, v.data(), bytes);
        std::memset(h + bytes, 0, need - bytes);
        HSSX_HIP(hipMemcpyAsync(d, h, need, hipMemcpyHostToDevice, st_));
        for (size_t g = g0; g < g1; ++g) c.state[g] = read_only ? kPending : kUnknown;
      }
    }
    off_ += need;
    return reinterpret_cast<T *>(d);
  }
  hipStream_t st_;
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, off_ = 0;
};

}  // namespace hssx
