// A fixed device scratch array for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops that forbid hipMalloc).
//
// The array lives in this code object; every GPU the library runs on holds its
// own copy, at its own address, until the process ends.  In host code the
// array's name is only a host-side stand-in, so its device address is taken
// once per device with hipGetSymbolAddress (with that device current) and
// kept; only that address is ever passed to kernels.
#include <mutex>

#include "pir_internal.h"

namespace pir {
namespace {

__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch_init(int device, void **ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace pir
