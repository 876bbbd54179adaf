// Fixed device scratch for gt_query_batch_noalloc: query calls that must not
// allocate (code under graph capture, tight serving loops) run every
// per-call buffer -- query copies, frontiers, counters, candidates, result
// staging -- out of one file-scope device array of kScratchBytes.
//
// The array's name is a host-side stand-in, not a device address: host code
// uses only the pointer that hipGetSymbolAddress returned for it on each
// device, taken once per device at set-up (index build) with that device
// current.  Each device holds its own copy of the array until the process
// ends, and every call on a device shares it: it keeps the last call's
// contents (a call clears what must start at zero), and calls that overlap on
// one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gt_internal.h"

static __device__ __align__(256) unsigned char scratch[gt::kScratchBytes];

namespace gt {

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) {
    const hipError_t e2 = hipSetDevice(cur);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace gt
