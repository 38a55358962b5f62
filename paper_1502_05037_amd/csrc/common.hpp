// Shared host-side helpers of the sarahip library: status handling, device buffers, launch checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/sarahip.h"

namespace sh {

// Thread-local message for the last non-OK status.
void set_error(const char* fmt, ...);
const char* last_error();

// Error propagation inside the library: functions return sh_status; SH_TRY returns early.
#define SH_TRY(expr)                        \
  do {                                      \
    sh_status _s = (expr);                  \
    if (_s != SH_OK) return _s;             \
  } while (0)

#define SH_HIP(expr)                                                                           \
  do {                                                                                         \
    hipError_t _e = (expr);                                                                    \
    if (_e != hipSuccess) {                                                                    \
      ::sh::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
      return _e == hipErrorOutOfMemory ? SH_ENOMEM : SH_EDEVICE;                               \
    }                                                                                          \
  } while (0)

#define SH_LAUNCHED()                                                                            \
  do {                                                                                           \
    hipError_t _e = hipGetLastError();                                                           \
    if (_e != hipSuccess) {                                                                      \
      ::sh::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(_e), __FILE__, __LINE__); \
      return SH_EDEVICE;                                                                         \
    }                                                                                            \
  } while (0)

#define SH_REQUIRE(cond, ...)          \
  do {                                 \
    if (!(cond)) {                     \
      ::sh::set_error(__VA_ARGS__);    \
      return SH_EINVAL;                \
    }                                  \
  } while (0)

// Caller-provided device memory (a workspace) handed out as a stack: each allocation is carved, 256-byte
// aligned, at the top; a release marks its block free and the top falls back over every free block at the
// top, so that scoped temporaries are reused in order.  The owner of the arena must outlive every buffer
// taken from it.
struct Arena {
  char* base = nullptr;
  size_t size = 0, top = 0, peak = 0;
  struct Blk {
    size_t off;
    bool freed;
  };
  std::vector<Blk> blocks;
  static constexpr size_t kAlign = 256;
  static size_t round(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }
  void* take(size_t bytes) {
    const size_t b = round(bytes);
    if (top + b > size) return nullptr;
    void* p = base + top;
    blocks.push_back({top, false});
    top += b;
    peak = top > peak ? top : peak;
    return p;
  }
  void give(void* p) {
    const size_t off = size_t(static_cast<char*>(p) - base);
    for (auto& b : blocks)
      if (b.off == off) b.freed = true;
    while (!blocks.empty() && blocks.back().freed) {
      top = blocks.back().off;
      blocks.pop_back();
    }
  }
};
// The arena that DevBuf allocations of this thread take their memory from (NULL: hipMalloc).
Arena*& arena_slot();
struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena* a) : prev(arena_slot()) { arena_slot() = a; }
  ~ArenaScope() { arena_slot() = prev; }
};

// Library-owned device memory: every hipMalloc of DevBuf reserves its bytes here first, and the reservation
// fails (SH_ENOMEM) when the environment variable SH_MAX_DEVICE_BYTES holds a positive byte count that the live
// total would exceed.  Caller workspaces are not counted (the library does not allocate them).
bool dev_reserve(size_t bytes);
void dev_unreserve(size_t bytes);

// The stream the uploads of this thread's DevBufs go to (NULL: hipMemcpy, synchronous on the null stream).
hipStream_t& upload_stream();
struct UploadStreamScope {
  hipStream_t prev;
  explicit UploadStreamScope(hipStream_t s) : prev(upload_stream()) { upload_stream() = s; }
  ~UploadStreamScope() { upload_stream() = prev; }
};

// Owning device allocation: hipMalloc / hipFree, or a block of the thread's current arena.
template <typename T>
struct DevBuf {
  T* ptr = nullptr;
  size_t count = 0;
  Arena* arena = nullptr;   // where ptr came from (NULL: hipMalloc)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), count(o.count), arena(o.arena) {
    o.ptr = nullptr;
    o.count = 0;
    o.arena = nullptr;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      ptr = o.ptr;
      count = o.count;
      arena = o.arena;
      o.ptr = nullptr;
      o.count = 0;
      o.arena = nullptr;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (ptr) {
      if (arena) {
        arena->give(ptr);
      } else {
        (void)hipFree(ptr);
        dev_unreserve(count * sizeof(T));
      }
    }
    ptr = nullptr;
    count = 0;
    arena = nullptr;
  }
  sh_status alloc(size_t n) {
    release();
    if (n == 0) return SH_OK;
    if (Arena* a = arena_slot()) {
      ptr = static_cast<T*>(a->take(n * sizeof(T)));
      if (!ptr) {
        ::sh::set_error("workspace of %zu bytes exhausted (%zu in use, %zu more requested)", a->size, a->top,
                        Arena::round(n * sizeof(T)));
        return SH_ENOMEM;
      }
      arena = a;
    } else {
      if (!dev_reserve(n * sizeof(T))) {
        ::sh::set_error("allocating %zu device bytes would exceed SH_MAX_DEVICE_BYTES", n * sizeof(T));
        return SH_ENOMEM;
      }
      const hipError_t e = hipMalloc((void**)&ptr, n * sizeof(T));
      if (e != hipSuccess) {
        ptr = nullptr;
        dev_unreserve(n * sizeof(T));
        ::sh::set_error("hipMalloc of %zu bytes failed: %s", n * sizeof(T), hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? SH_ENOMEM : SH_EDEVICE;
      }
    }
    count = n;
    return SH_OK;
  }
  sh_status upload(const T* host, size_t n) {
    SH_TRY(alloc(n));
    if (!n) return SH_OK;
    if (hipStream_t st = upload_stream()) {   // the caller's stream; the host array may go right after the call
      SH_HIP(hipMemcpyAsync(ptr, host, n * sizeof(T), hipMemcpyHostToDevice, st));
      SH_HIP(hipStreamSynchronize(st));
    } else {
      SH_HIP(hipMemcpy(ptr, host, n * sizeof(T), hipMemcpyHostToDevice));
    }
    return SH_OK;
  }
  sh_status upload(const std::vector<T>& v) { return upload(v.data(), v.size()); }
};

inline int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}
inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Kernel timing with HIP events on the launch stream (enabled by sh_profile_enable).
bool profiling_on();
struct ProfScope {
  hipEvent_t a = nullptr, b = nullptr;
  int slot = -1;
  hipStream_t st = nullptr;
  ProfScope(const char* name, hipStream_t stream);
  ~ProfScope();
};

}  // namespace sh

// Work-groups are dispatched to the 8 XCDs round-robin (block b -> XCD b % 8), and each XCD has its own
// L2.  This maps the hardware block index to a logical one so that every XCD works on one contiguous
// range of logical blocks: neighbouring work (adjacent FFT columns, neighbouring tiles) then shares an
// L2 instead of being fetched once per XCD.  A bijection on [0, nblocks).
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  const int per = nblocks >> 3, rem = nblocks & 7;
  const int x = bid & 7, k = bid >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

// The same idea for uneven work (gridding items): consecutive runs of G logical blocks go to one XCD,
// and the runs rotate over the XCDs, so neighbours share an L2 while heavy and light regions still
// spread over all XCDs.  A bijection on [0, nblocks).
__device__ __forceinline__ int xcd_block_runs(int bid, int nblocks, int G) {
  const int span = 8 * G;
  const int base = (bid / span) * span, b = bid - base;
  const int r = nblocks - base < span ? nblocks - base : span;   // blocks in this group
  const int x = b & 7, j = b >> 3;
  int start = 0;
  for (int y = 0; y < x; ++y) start += (r - y + 7) >> 3;          // blocks of XCDs 0..x-1 in the group
  return base + start + j;
}

// Device-side complex helpers.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
