// rtcdf_pmax.hip -- the prefix-maximum output method (Alg. 3, "RefHP" of
// Sec. 2.2), selectable in place of the interval fill of Alg. 7 with
// RTCDF_FLAG_OUTPUT_PREFIX_MAX.  It starts from the same local CDFs C_t and
// tile offsets O[t] (Alg. 4-6), so the inclusive CDF of value d is
// P1[d] = O[t] + C_t[x], d = tT + x, and the output is byte-identical.
//
// Alg. 3 in four launches:
//   k_pmax_init   B[0, n) = minVal (the normalised value 0), and the chunk
//                 maxima M[] = 0.
//   k_pmax_step   for every value d in [1, R) with P1[d] > P1[d-1]:
//                 B[P1[d-1]] = minVal + d.  The thread of the last step of an
//                 output chunk also stores d as that chunk's maximum M[c] (the
//                 steps increase with position, so the chunk maximum of B is
//                 its last step; exactly one value qualifies per chunk that
//                 holds a step, so plain stores suffice).
//   k_pmax_carry  exclusive prefix maximum of M (one workgroup): the value
//                 carried into each chunk.
//   k_pmax_scan   the inclusive prefix maximum of B in place, one wave per
//                 chunk of kPmaxChunk positions, in windows of 256 positions
//                 (16 bytes a lane): eight windows are loaded, then each gets
//                 a lane-level and a wave-level (shuffle) maximum scan.
//
// Chunk c covers positions [q_c, q_{c+1}) with q_0 = 0 and
// q_c = out_head + c * kPmaxChunk for c >= 1, so every window after the
// scalar head starts on a 16-byte boundary of B.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rtcdf_device.h"
#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

using namespace dev;

constexpr uint32_t kPmaxWindow = 64 * 4;                    // positions per wave window (16 B a lane)
constexpr uint32_t kPmaxGroup = 8;                          // windows loaded before they are scanned
static_assert(kPmaxChunk % (kPmaxWindow * kPmaxGroup) == 0, "chunk is whole window groups");

__device__ __forceinline__ uint32_t pmax_chunk_of(uint64_t p, uint32_t head) {
  return p < head ? 0u : (uint32_t)((p - head) / kPmaxChunk);
}

__global__ __launch_bounds__(256) void k_pmax_init(int32_t* __restrict__ out, uint32_t n, uint32_t head,
                                                   int32_t fill, uint32_t* __restrict__ M, uint32_t nck) {
  const size_t stride = (size_t)gridDim.x * 256;
  const size_t gid = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (gid < head) out[gid] = fill;
  const uint32_t n4 = (n - head) / 4;
  v4i* body = reinterpret_cast<v4i*>(out + head);
  const v4i f = {fill, fill, fill, fill};
  for (size_t i = gid; i < n4; i += stride) body[i] = f;
  const uint32_t tail = head + n4 * 4;
  if (gid < n - tail) out[tail + gid] = fill;
  for (size_t i = gid; i < nck; i += stride) M[i] = 0u;
}

__global__ __launch_bounds__(256) void k_pmax_step(const uint32_t* __restrict__ cdf,
                                                   const uint32_t* __restrict__ O, uint32_t T, uint32_t R,
                                                   uint32_t n, uint32_t head, int32_t minVal,
                                                   int32_t* __restrict__ out, uint32_t* __restrict__ M) {
  const uint32_t d = blockIdx.x * 256 + threadIdx.x + 1;   // value 0 is the initial fill
  if (d >= R) return;
  const uint32_t t = d / T, x = d - t * T;
  const uint32_t base = O[t];
  const uint32_t e = base + cdf[d];                   // P1[d]
  const uint32_t s = x ? base + cdf[d - 1] : base;    // P1[d - 1]
  if (e <= s) return;                                 // no key with value d
  out[s] = minVal + (int32_t)d;
  const uint32_t c = pmax_chunk_of(s, head);
  const uint64_t hi = (uint64_t)head + (uint64_t)(c + 1) * kPmaxChunk;
  if (e >= hi || e == n) M[c] = d;                    // last step of chunk c
}

constexpr uint32_t kCarryBlock = 1024;

__global__ __launch_bounds__(kCarryBlock) void k_pmax_carry(uint32_t* __restrict__ M, uint32_t nck) {
  __shared__ uint32_t part[kCarryBlock];
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (nck + kCarryBlock - 1) / kCarryBlock;
  const uint32_t lo = min(nck, tid * per), hi = min(nck, lo + per);
  uint32_t mx = 0;
  for (uint32_t i = lo; i < hi; i++) mx = max(mx, M[i]);
  part[tid] = mx;
  __syncthreads();
  // inclusive maximum scan of the per-thread maxima (Hillis-Steele in LDS)
  for (uint32_t off = 1; off < kCarryBlock; off <<= 1) {
    const uint32_t v = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] = max(part[tid], v);
    __syncthreads();
  }
  uint32_t run = tid ? part[tid - 1] : 0u;
  for (uint32_t i = lo; i < hi; i++) {
    const uint32_t v = M[i];
    M[i] = run;                                       // carry into chunk i
    run = max(run, v);
  }
}

__device__ __forceinline__ int32_t wave_scan_max(int32_t v, uint32_t lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t u = __shfl_up(v, off, 64);
    if (lane >= (uint32_t)off) v = max(v, u);
  }
  return v;
}

__global__ __launch_bounds__(256) void k_pmax_scan(int32_t* __restrict__ out, uint32_t n, uint32_t head,
                                                   int32_t minVal, const uint32_t* __restrict__ carry,
                                                   uint32_t nck) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= nck) return;
  int32_t run = minVal + (int32_t)carry[c];
  if (c == 0) {
    // the scalar head: every lane computes the same running maximum
    for (uint32_t p = 0; p < head && p < n; p++) {
      run = max(run, out[p]);
      if (lane == 0) out[p] = run;
    }
  }
  const uint64_t start = (uint64_t)head + (uint64_t)c * kPmaxChunk;
  for (uint32_t g = 0; g < kPmaxChunk / kPmaxWindow; g += kPmaxGroup) {
    if (start + (uint64_t)g * kPmaxWindow >= n) break;
    v4i w[kPmaxGroup];
#pragma unroll
    for (uint32_t k = 0; k < kPmaxGroup; k++) {
      const uint64_t p = start + (uint64_t)(g + k) * kPmaxWindow + 4 * lane;
      if (p + 3 < n) {
        w[k] = *reinterpret_cast<const v4i*>(out + p);
      } else {
        w[k].x = p < n ? out[p] : INT32_MIN;
        w[k].y = p + 1 < n ? out[p + 1] : INT32_MIN;
        w[k].z = p + 2 < n ? out[p + 2] : INT32_MIN;
        w[k].w = INT32_MIN;
      }
    }
#pragma unroll
    for (uint32_t k = 0; k < kPmaxGroup; k++) {
      const uint64_t p = start + (uint64_t)(g + k) * kPmaxWindow + 4 * lane;
      v4i v = w[k];
      v.y = max(v.y, v.x);
      v.z = max(v.z, v.y);
      v.w = max(v.w, v.z);
      const int32_t incl = wave_scan_max(v.w, lane);
      int32_t excl = __shfl_up(incl, 1, 64);
      excl = lane ? max(run, excl) : run;
      v.x = max(v.x, excl);
      v.y = max(v.y, excl);
      v.z = max(v.z, excl);
      v.w = max(v.w, excl);
      if (p + 3 < n) {
        *reinterpret_cast<v4i*>(out + p) = v;
      } else {
        if (p < n) out[p] = v.x;
        if (p + 1 < n) out[p + 1] = v.y;
        if (p + 2 < n) out[p + 2] = v.z;
      }
      run = max(run, __shfl(incl, 63, 64));
    }
  }
}

}  // namespace

uint32_t pmax_chunks(uint64_t n, uint32_t head) {
  return 1 + ((n >= 1 && n - 1 >= head) ? (uint32_t)((n - 1 - head) / kPmaxChunk) : 0u);
}

hipError_t launch_output_pmax(const Plan& p, int32_t* out, uint8_t* ws, hipStream_t s) {
  const uint32_t n = (uint32_t)p.n;
  const uint32_t head = (uint32_t)std::min<uint64_t>(p.out_head, p.n);
  const uint32_t nck = p.pm_chunks;
  if (p.out_head > 3 || p.n > 0xffffffffull || nck != pmax_chunks(p.n, head) || p.pm_init_grid == 0)
    return hipErrorInvalidValue;
  uint32_t* M = reinterpret_cast<uint32_t*>(ws + p.off_pm);
  const int32_t minVal = (int32_t)p.min_u;
  hipLaunchKernelGGL(k_pmax_init, dim3(p.pm_init_grid), dim3(256), 0, s, out, n, head, minVal, M, nck);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.R > 1) {
    hipLaunchKernelGGL(k_pmax_step, dim3((p.R - 1 + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<const uint32_t*>(ws + p.off_cdf),
                       reinterpret_cast<const uint32_t*>(ws + p.off_O), p.T, p.R, n, head, minVal,
                       out, M);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_pmax_carry, dim3(1), dim3(kCarryBlock), 0, s, M, nck);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pmax_scan, dim3((nck + 3) / 4), dim3(256), 0, s, out, n, head, minVal,
                     static_cast<const uint32_t*>(M), nck);
  return hipGetLastError();
}

}  // namespace rtcdf
