// rtcdf_check.hip -- checked mode: counts the keys outside [minVal, maxVal).
//
// The keys lying in the declared range is a precondition of the method
// (Sec. 2.1) that the sort does not test; a key outside it leaves the output
// unspecified.  This kernel tests it with one more streaming read of the keys.
#include <hip/hip_runtime.h>

#include "rtcdf_device.h"
#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

using namespace dev;

// Checked mode: number of keys whose offset from minVal is not below R.
// Head (before the 16-byte aligned body) and tail are read by scalar loads.
__global__ __launch_bounds__(256) void k_count_out_of_range(const int32_t* __restrict__ keys,
                                                             uint64_t head, uint64_t n4, uint64_t n,
                                                             uint32_t min_u, uint32_t R,
                                                             unsigned long long* count) {
  __shared__ uint32_t wsum[256 / 64];
  const size_t stride = (size_t)gridDim.x * 256;
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  uint32_t c = 0;
  const v4i* body = reinterpret_cast<const v4i*>(keys + head);
  for (size_t i = t; i < n4; i += stride) {
    const v4i k = __builtin_nontemporal_load(&body[i]);
    c += ((uint32_t)k.x - min_u >= R) + ((uint32_t)k.y - min_u >= R) + ((uint32_t)k.z - min_u >= R) +
         ((uint32_t)k.w - min_u >= R);
  }
  const uint64_t tail0 = head + 4 * n4;
  if (t < head) c += (uint32_t)keys[t] - min_u >= R;
  if (t < n - tail0) c += (uint32_t)keys[tail0 + t] - min_u >= R;
  const uint32_t total = block_sum(c, wsum);
  if (threadIdx.x == 0 && total != 0) atomicAdd(count, (unsigned long long)total);
}

}  // namespace

hipError_t launch_count_out_of_range(const int32_t* keys, uint64_t n, uint32_t min_u, uint32_t R,
                                     uint64_t* count, int cus, hipStream_t s) {
  hipError_t e = launch_clear(reinterpret_cast<uint32_t*>(count), 2, s);
  if (e != hipSuccess || n == 0) return e;
  const uintptr_t a = reinterpret_cast<uintptr_t>(keys);
  uint64_t head = ((16 - (a & 15)) & 15) / 4;
  if (head > n) head = n;
  const uint64_t n4 = (n - head) / 4;
  uint64_t blocks = (n4 + 255) / 256;
  if (blocks > (uint64_t)cus * 4) blocks = (uint64_t)cus * 4;
  if (blocks == 0) blocks = 1;   // head and tail only (at most 3 keys each)
  hipLaunchKernelGGL(k_count_out_of_range, dim3((unsigned)blocks), dim3(256), 0, s, keys, head, n4, n,
                     min_u, R, reinterpret_cast<unsigned long long*>(count));
  return hipGetLastError();
}

}  // namespace rtcdf
