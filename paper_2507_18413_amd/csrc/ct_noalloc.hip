// ct_noalloc.hip -- device scratch of ct_propagate_batch_noalloc (include/ct.h).
//
// The batch entry point keeps its work-queue counters, the staged job
// descriptors and the search-node schedule's records in memory it allocates
// per stream.  Its no-allocation variant takes them from one static device
// array instead: every GPU the library runs on holds its own copy until the
// process ends, and every no-allocation call on that GPU shares it.  Host
// code never passes the array's name to a kernel or a copy (on the host the
// name is a stand-in, not a device address): it asks the runtime for the
// current device's address of the array once per device and uses that.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ct_device.h"

namespace ctk {

constexpr size_t NA_SCRATCH_BYTES = (size_t)16 << 20;

// [0, 256): work-queue counters (head, exit count, launches, error) and the
// error word of an earlier call; then descriptor staging (2 MiB); then the
// search-node records and granule flags (the rest)
static __device__ __align__(256) char scratch[NA_SCRATCH_BYTES];

namespace {

// Clears the work queue before a call: head and exit count (a launch that
// ended normally already left them at zero) and the error word, whose last
// value is kept in word 4 for ct_batch_status.
__global__ void noalloc_reset_kernel(int32_t* q) {
  if (threadIdx.x == 0) {
    if (q[3]) q[4] = q[3];
    q[0] = 0;
    q[1] = 0;
    q[3] = 0;
  }
}

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_mu;
char* g_ptr[NA_MAX_DEVICES];

}  // namespace

// The current device's address of the scratch array and its size; the
// address is looked up on a device's first use and kept.
hipError_t noalloc_scratch(char** ptr, size_t* bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NA_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = (char*)p;
  }
  *ptr = g_ptr[dev];
  *bytes = NA_SCRATCH_BYTES;
  return hipSuccess;
}

hipError_t launch_noalloc_reset(int32_t* q, hipStream_t stream) {
  hipLaunchKernelGGL(noalloc_reset_kernel, dim3(1), dim3(64), 0, stream, q);
  return hipGetLastError();
}

}  // namespace ctk
