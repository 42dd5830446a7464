// sale_noalloc.hip -- the device array that holds the intermediates of the
// contexts made by sale_init_static, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation).
//
// `scratch` is a file-scope device array: every device the library runs
// sale_init_static on holds its own copy until the process ends. In host code
// its name is only a stand-in for the symbol, never a device address: the
// address on a device comes from hipGetSymbolAddress, looked up once per
// device with that device current and kept in a host table, and only that
// address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sale_impl.h"

namespace sale {
namespace {

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` per device (null: not looked up yet)

}  // namespace

hipError_t static_scratch(void **ptr) {
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || ((uintptr_t)p & 255u)) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return hipSuccess;
}

}  // namespace sale
