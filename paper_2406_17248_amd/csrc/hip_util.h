// Small host helpers shared by the C-ABI sources: status errors, grow-only device buffers.
#pragma once
#include <hip/hip_runtime_api.h>

#include <new>
#include <string>

#include "engine.h"

namespace qsv {

[[noreturn]] inline void raise(int status, const std::string& msg) { throw Error{status, msg}; }

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    raise(e == hipErrorOutOfMemory ? QSV_ENOMEM : QSV_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void reserve(size_t need) {
    if (need <= bytes) return;
    if (p) hip_check(hipFree(p), "hipFree");
    p = nullptr;
    bytes = 0;
    hip_check(hipMalloc(&p, need), "hipMalloc workspace");
    bytes = need;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Thread-local message of the last failed ABI call.
std::string& last_error();

// Run an ABI body, turning exceptions into status codes.
template <typename F>
int guarded(F&& f) {
  try {
    f();
    last_error().clear();
    return QSV_OK;
  } catch (const Error& e) {
    last_error() = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    last_error() = "host allocation failed";
    return QSV_ENOMEM;
  } catch (...) {
    last_error() = "unexpected internal error";
    return QSV_EINVAL;
  }
}

}  // namespace qsv
