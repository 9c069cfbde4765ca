// me_compute_channels_noalloc: the multi-subprocess entry point with its
// workspace in a fixed device array, for callers that cannot allocate device
// memory (code under stream capture, tight serving loops).
//
// The workspace of a channel request (event permutation, gathered momenta and
// results, per-block channel counts and offsets, an out-of-range flag) lives
// in `scratch`, one array per device that holds it from the library's first
// use on that device until the process ends.  The kernels receive its device
// address, looked up once per device with hipGetSymbolAddress (the array's
// name is not a device address in host code).  Nothing here calls
// hipMalloc, hipMallocAsync or any allocating routine.  Every call on a
// device shares that device's array, so calls that overlap on one device
// (different streams or threads) race; each call clears the flag it reads
// and overwrites everything else it uses.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "channels.hpp"
#include "handle.hpp"
#include "me.h"

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[ME_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's `scratch`, or nullptr (error recorded).
void* scratch_of(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      me::set_error(ME_EHIP, std::string("me_compute_channels_noalloc: hipGetSymbolAddress: ") +
                                 hipGetErrorString(e));
      return nullptr;
    }
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" me_status me_compute_channels_noalloc(const me_handle* handles, int32_t nchannels,
                                                 const double* d_momenta, const int32_t* d_channel,
                                                 const double* d_alphas, int64_t nevt, double* d_me,
                                                 void* hip_stream) {
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return me::set_error(ME_EHIP, std::string("me_compute_channels_noalloc: hipGetDevice: ") +
                                                         hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return me::set_error(ME_ENOTSUP, "me_compute_channels_noalloc: device index");
  void* ws = scratch_of(dev);
  if (!ws) return ME_EHIP;
  return me::compute_channels_on(handles, nchannels, d_momenta, d_channel, d_alphas, nevt, d_me,
                                 static_cast<hipStream_t>(hip_stream), ws, ME_NOALLOC_SCRATCH_BYTES,
                                 "me_compute_channels_noalloc");
}
