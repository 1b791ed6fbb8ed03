// Launch scratch for callers that cannot allocate device memory: a file-scope
// device array, one copy per GPU, that sqa_anneal_batch_noalloc uses for the
// handle descriptors, work items and work counters of its persistent launch.
//
// In host code the array's name is a host-side stand-in, not a device address:
// the address of each GPU's copy comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is ever handed to
// kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host_core.h"

namespace sqa {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

sqa_status noalloc_scratch(void **ptr_out) {
  *ptr_out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(SQA_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));     // the current device's copy
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress (launch scratch)");
    }
    g_ptr[dev] = p;
  }
  *ptr_out = g_ptr[dev];
  return SQA_OK;
}

}  // namespace sqa
