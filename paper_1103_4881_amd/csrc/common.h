// Host helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "aolmi.h"

namespace aol {

aol_status fail(aol_status st, const char* fmt, ...);
aol_status ok();
aol_status hip_fail(hipError_t e, const char* what);
const char* last_error();

// One axis' filter as validated host data.
struct FilterHost {
  int p = 0, q = 0, taps = 0;
  std::vector<int> c;  // [p][taps]
  std::vector<int> s;  // [p] window starts
};

aol_status check_filter(const aol_polyphase* f, const char* name, FilterHost& out);
void default_starts(int p, int q, int taps, int32_t* out);

// Owned device allocation (freed on destruction).
struct DeviceBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DeviceBuf() = default;
  DeviceBuf(const DeviceBuf&) = delete;
  DeviceBuf& operator=(const DeviceBuf&) = delete;
  DeviceBuf(DeviceBuf&& o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
  DeviceBuf& operator=(DeviceBuf&& o) noexcept {
    if (this != &o) {
      reset();
      ptr = o.ptr;
      bytes = o.bytes;
      o.ptr = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DeviceBuf() { reset(); }
  void reset() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  aol_status alloc(size_t n) {
    reset();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
      ptr = nullptr;
      return e == hipErrorOutOfMemory ? fail(AOL_ERR_NOMEM, "hipMalloc(%zu): %s", n, hipGetErrorString(e))
                                      : hip_fail(e, "hipMalloc");
    }
    bytes = n;
    return AOL_OK;
  }
  // Synchronous upload at plan creation (never on a run path).
  aol_status upload(const void* src, size_t n) {
    aol_status st = alloc(n);
    if (st) return st;
    if (n) {
      hipError_t e = hipMemcpy(ptr, src, n, hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpy to device");
    }
    return AOL_OK;
  }
};

}  // namespace aol
