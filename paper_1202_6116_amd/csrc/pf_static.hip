// The library's static device workspace: the memory of contexts made by
// pf_init_static, for callers that cannot allocate device memory.  One
// array per GPU, held until the process ends; at most one context uses a
// GPU's array at a time.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pf_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[pf::kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;

struct StaticSlots {
  std::mutex mu;
  void* ptr[kMaxDevices] = {};   // device address of each GPU's array (null: not looked up yet)
  bool busy[kMaxDevices] = {};   // a context holds the GPU's array
};

StaticSlots& slots() {
  static StaticSlots s;
  return s;
}

}  // namespace

namespace pf {

// Claims the array of the current device: *ptr receives its device address
// (looked up once per device with that device current).  Returns
// hipErrorInvalidDevice for a device index beyond the table, hipErrorAlreadyAcquired
// when a context already holds the array, or the lookup's error.
hipError_t static_workspace_acquire(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  StaticSlots& s = slots();
  std::lock_guard<std::mutex> g(s.mu);
  if (s.busy[device]) return hipErrorAlreadyAcquired;
  if (!s.ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    s.ptr[device] = p;
  }
  s.busy[device] = true;
  *ptr = s.ptr[device];
  return hipSuccess;
}

void static_workspace_release(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  StaticSlots& s = slots();
  std::lock_guard<std::mutex> g(s.mu);
  s.busy[device] = false;
}

}  // namespace pf
