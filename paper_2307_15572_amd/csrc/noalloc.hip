// rsvd_run_noalloc: rsvd_run with its workspace in a file-scope device array,
// for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array lives in this code object: every device the library runs on
// holds its own copy until the process ends. Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol); the
// device address is looked up once per device with hipGetSymbolAddress, with
// that device current, and that address is what the run receives as its
// workspace. rsvd_run itself allocates nothing and resets every word of the
// workspace it reads before writing (the device state record with its flags,
// counters and grid-barrier words is cleared by its first launch), so the
// contents a previous call left behind do not matter. Calls that overlap on
// one device share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rsvd.h"
#include "plan.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)RSVD_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up once per
// device, with that device current).
rsvd_status scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RSVD_EHIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RSVD_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RSVD_OK;
}

}  // namespace

extern "C" {

size_t rsvd_noalloc_max_bytes(void) { return kScratchBytes; }

rsvd_status rsvd_run_noalloc(rsvd_plan_t plan, const double* A, int64_t lda, const double* omega,
                             int64_t ldo, double* S, double* U, int64_t ldu, double* V,
                             int64_t ldv, rsvd_result* res_dev, void* stream) {
  if (!plan) return RSVD_EINVAL;
  // reject before any launch: the plan's workspace must fit the array
  if (plan->total > kScratchBytes) return RSVD_ENOMEM;
  void* work = nullptr;
  const rsvd_status r = scratch_for_current_device(&work);
  if (r != RSVD_OK) return r;
  return rsvd_run(plan, A, lda, omega, ldo, S, U, ldu, V, ldv, res_dev, work, kScratchBytes,
                  stream);
}

}  // extern "C"
