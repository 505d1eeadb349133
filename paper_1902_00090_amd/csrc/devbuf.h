// Scoped device scratch: freed on every return path (including the early
// returns of DD_HIP_CHECK).
#pragma once

#include <hip/hip_runtime.h>

struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};
