// The Strassen-Winograd entry point that allocates nothing on the device
// (mm_winograd_noalloc in mm.h), for callers that cannot call hipMalloc:
// code under HIP graph capture, tight serving loops, harnesses that forbid
// allocation.
//
// Its memory is one file-scope device array per GPU (below), held from the
// moment the library's code object is loaded on that GPU until the process
// ends.  The array's first MM_NOALLOC_TABLE_BYTES hold the plan's
// descriptor table (copied in at every call: another shape may have used
// the array since), the rest is the product's workspace.  The product runs
// the Two Temp schedule of Section 3.3 (Table 2): two temporaries per
// level, the smallest workspace of the paper's schedules that leaves A and B
// intact, so a modest array covers large products (float32 n = 4096 with two
// levels needs 40 MiB).
//
// Host code never passes the array's name to a kernel or a copy: the name
// is a host-side stand-in, not a device address.  The address is taken once
// per device with hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"
#include "mm.h"

namespace {

__device__ __align__(256) unsigned char scratch[MM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

// The device address of this device's copy of `scratch` (looked up on the
// first call with the device current).
int scratch_for_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return mm::set_error(MM_E_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return mm::set_error(MM_E_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return mm::set_error(MM_E_HIP, (std::string("hipGetSymbolAddress of the static scratch failed: ") +
                                      hipGetErrorString(e)).c_str());
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return MM_OK;
}

}  // namespace

extern "C" int mm_winograd_noalloc(int64_t m, int64_t n, int64_t k, const void* A, const void* B, void* C,
                                   int cutoff, int levels, int dtype, hipStream_t stream) {
  void* base = nullptr;
  const int rc = scratch_for_current_device(&base);
  if (rc != MM_OK) return rc;
  return mm::run_in_memory(MM_ALGO_WINOGRAD, MM_SCHED_TWO_TEMP, m, n, k, A, B, C, cutoff, levels, dtype, base,
                           MM_NOALLOC_TABLE_BYTES, static_cast<char*>(base) + MM_NOALLOC_TABLE_BYTES,
                           (size_t)MM_NOALLOC_SCRATCH_BYTES - MM_NOALLOC_TABLE_BYTES, stream);
}
