// Fixed device scratch of the allocation-free expectation entry point.
//
// The array lives in the code object: every GPU the library runs on holds its own copy,
// at its own address, until the process ends.  Host code never uses the array's name as
// an address (in host code it names a host-side stand-in); it asks the runtime for this
// device's address once and passes that pointer to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hip_util.h"
#include "noalloc.h"

namespace {

static __device__ __align__(256) unsigned char scratch[qsv::kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

namespace qsv {

void* noalloc_scratch() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) raise(QSV_ERANGE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) raise(QSV_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace qsv
