// Fixed device scratch for the entry point that allocates nothing (qqa_dev_eval_noalloc):
// the evaluation's per-replica integer accumulators [2][stride] for every replica stride
// the library accepts, 2 x 4096 uint64 = 64 KiB.  Each GPU the library runs on holds its
// own copy until the process ends; every call on a GPU shares it, so calls that overlap
// on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "qqa_internal.h"

namespace qqa {

namespace {
constexpr size_t kEvalScratchWords = 2 * (size_t)kMaxReplicas;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned long long scratch[kEvalScratchWords];

// Device address of `scratch` on the current device, looked up once per device with that
// device current.  In host code the array's name is only a host-side stand-in: kernels are
// given this address, never the name.
hipError_t eval_scratch(unsigned long long** out, size_t* words) {
  static std::mutex mu;
  static unsigned long long* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<unsigned long long*>(ptr);
  }
  *out = addr[dev];
  *words = kEvalScratchWords;
  return hipSuccess;
}

}  // namespace qqa
