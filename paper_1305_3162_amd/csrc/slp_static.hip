// Static device workspace for the evaluation entry point that allocates
// nothing (slp_eval_single_layer_static). The array below exists once per
// device (each device that loads the library's code object holds its own copy
// until the process ends). In host code `scratch` is only the host-side shadow
// of the device symbol, never a device address: the device address is looked
// up once per device with hipGetSymbolAddress, with that device current, and
// every kernel argument and copy uses that address.
#include "slp_internal.hpp"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

static __device__ __align__(256) unsigned char scratch[slp::kStaticWorkspaceBytes];

std::mutex g_mu;
void *g_addr[slp::kMaxDevices] = {};   // device address of `scratch`, per device

}  // namespace

hipError_t slp::static_workspace(void **ptr) {
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[dev] = p;
  }
  *ptr = g_addr[dev];
  return hipSuccess;
}
