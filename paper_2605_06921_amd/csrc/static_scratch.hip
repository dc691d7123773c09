// Device scratch held by the library itself, for the entry point that
// allocates nothing (mqo_objective_grad_static).  Every GPU the library runs
// on holds its own copy of the array from module load until the process
// ends; calls on one GPU share it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mqo.h"
#include "kernels.h"

static __device__ __align__(256) unsigned char scratch[MQO_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

}  // namespace

namespace mqo {

// The address of the scratch array on the current device.  The name
// `scratch` stands for the array only in device code: host code must use the
// address hipGetSymbolAddress returns, looked up once per device with that
// device current.
hipError_t static_scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return hipSuccess;
}

}  // namespace mqo
