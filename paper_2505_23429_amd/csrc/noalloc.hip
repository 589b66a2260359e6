// Fixed device scratch of the no-allocation entry point (tt_heff_apply_dev_noalloc).
//
// The array below is the only device memory that entry point uses besides the caller's
// operands: its intermediates and the MPO entry tables are carved from it.  Each GPU the
// library runs on holds its own copy until the process ends.  In host code the array's
// name is a host-side stand-in, never a device address: the address of a device's copy
// is looked up once per device (with that device current) and kept, and only that
// pointer is passed to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdexcept>
#include <string>

#include "engine.h"

namespace tt {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

void* noalloc_scratch(int device) {
  static std::mutex mu;
  static void* addr[256] = {};
  if (device < 0 || device >= 256) throw std::invalid_argument("device ordinal out of range");
  std::lock_guard<std::mutex> g(mu);
  if (!addr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device)
      throw HipError("no-allocation scratch: the device must be current when its address is looked up");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw HipError(std::string("hipGetSymbolAddress of the no-allocation scratch failed: ") + hipGetErrorString(e));
    addr[device] = p;
  }
  return addr[device];
}

}  // namespace tt
