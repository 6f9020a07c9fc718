// rtcdf_noalloc.hip -- rtcdf_sort_noalloc: the plain sort with its workspace
// in a fixed device array of the library, for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  Same plan and kernels as rtcdf_sort_ws.
//
// The array `scratch` is a file-scope device variable: each GPU the library
// runs on holds its own copy (kNoAllocBytes) until the process ends.  In host
// code the name `scratch` is a host-side stand-in, not a device address; the
// device address is obtained once per device with hipGetSymbolAddress and only
// that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/rtcdf.h"
#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

constexpr size_t kNoAllocBytes = RTCDF_NOALLOC_MAX_WORKSPACE;
static_assert(kNoAllocBytes % 256 == 0, "whole 256-byte blocks");

static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of that device's `scratch`

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device (with that device current) and kept.
rtcdf_status_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (ptr == nullptr || (reinterpret_cast<uintptr_t>(ptr) & 255u)) return RTCDF_ERROR_NOT_SUPPORTED;
    it = g_scratch_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return RTCDF_SUCCESS;
}

}  // namespace
}  // namespace rtcdf

using namespace rtcdf;

extern "C" rtcdf_status_t rtcdf_sort_noalloc(const int32_t* keys_in, int32_t* keys_out, size_t n,
                                             int64_t minVal, int64_t maxVal, const rtcdf_config_t* cfg,
                                             hipStream_t stream) {
  rtcdf_status_t st = check_problem(keys_in, keys_out, n, minVal, maxVal);
  if (st != RTCDF_SUCCESS || n == 0) return st;
  DeviceInfo dev;
  st = device_info(&dev);
  if (st != RTCDF_SUCCESS) return st;
  void* ws = nullptr;
  st = scratch_address(dev.device, &ws);
  if (st != RTCDF_SUCCESS) return st;
  return sort_in_workspace(keys_in, keys_out, n, minVal, maxVal, cfg, ws, kNoAllocBytes, stream);
}
