// rtcdf_pmax.hip -- the prefix-maximum output method (Alg. 3, "RefHP" of
// Sec. 2.2), selectable in place of the search of Alg. 7 with
// RTCDF_FLAG_OUTPUT_PREFIX_MAX.  It starts from the same local CDFs C_t and
// tile offsets O[t] (Alg. 4-6), so the inclusive CDF of value d is
// P1[d] = O[t] + C_t[x], d = tT + x, and the output is byte-identical.
//
// Alg. 3 rides on the launches the sort makes anyway, so it costs no more
// launches than the search when there are at most 1024 chunks:
//   k_reduce      (rtcdf_kernels.hip) extra workgroups write B[0, n) = minVal
//                 (the normalised value 0) and clear the chunk maxima M[].
//   k_tilescan    (rtcdf_kernels.hip) the first workgroup of each tile, which
//                 holds the tile's CDF in LDS, writes B[P1[d-1]] = minVal + d
//                 for every value d >= 1 of the tile with keys.  The thread of
//                 the last step of an output chunk also stores d as that
//                 chunk's maximum M[c] (the steps increase with position, so
//                 the maximum of a chunk of B is its last step; exactly one
//                 value qualifies per chunk that holds a step).
//   k_pmax_carry  (here, only with more than 1024 chunks) exclusive prefix
//                 maximum of M in place: the value carried into each chunk.
//   k_pmax_scan   (here) the inclusive prefix maximum of B in place, one wave
//                 per chunk of pm_chunk positions, in windows of 256
//                 positions (16 bytes a lane): eight windows are loaded, then
//                 each gets a lane-level and a wave-level (shuffle) maximum
//                 scan.  With at most 1024 chunks each wave takes its carry
//                 as the maximum of M over the chunks before its own.
//
// Chunk c covers positions [q_c, q_{c+1}) with q_0 = 0 and
// q_c = h + c * pm_chunk for c >= 1, h = min(out_head, n), so every window
// after the scalar head starts on a 16-byte boundary of B.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rtcdf_device.h"
#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

using namespace dev;

constexpr uint32_t kPmaxWindow = 64 * 4;                    // positions per wave window (16 B a lane)
constexpr uint32_t kPmaxGroup = 8;                          // windows loaded before they are scanned
static_assert(kPmaxChunkSmall % (kPmaxWindow * kPmaxGroup) == 0 &&
                  kPmaxChunkLarge % (kPmaxWindow * kPmaxGroup) == 0,
              "chunks are whole window groups");

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

// INLINE: `carry` holds the chunk maxima M and each wave reduces M[0, c)
// itself; otherwise it holds the carries written by k_pmax_carry.
template <bool INLINE>
__global__ __launch_bounds__(256) void k_pmax_scan(int32_t* __restrict__ out, uint32_t n, uint32_t head,
                                                   int32_t minVal, const uint32_t* __restrict__ carry,
                                                   uint32_t nck, uint32_t chunk) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= nck) return;
  uint32_t cin;
  if constexpr (INLINE) {
    cin = 0;
    for (uint32_t j = lane; j < c; j += 64) cin = max(cin, carry[j]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cin = max(cin, (uint32_t)__shfl_xor((int)cin, off, 64));
  } else {
    cin = carry[c];
  }
  int32_t run = minVal + (int32_t)cin;
  if (c == 0) {
    // the scalar head: every lane computes the same running maximum
    for (uint32_t p = 0; p < head && p < n; p++) {
      run = max(run, out[p]);
      if (lane == 0) out[p] = run;
    }
  }
  const uint64_t start = (uint64_t)head + (uint64_t)c * chunk;
  for (uint32_t g = 0; g < chunk / kPmaxWindow; g += kPmaxGroup) {
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

uint32_t pmax_chunks(uint64_t n, uint32_t head, uint32_t chunk) {
  return 1 + ((n >= 1 && n - 1 >= head) ? (uint32_t)((n - 1 - head) / chunk) : 0u);
}

hipError_t launch_output_pmax(const Plan& p, int32_t* out, uint8_t* ws, hipStream_t s) {
  const uint32_t n = (uint32_t)p.n;
  const uint32_t head = (uint32_t)std::min<uint64_t>(p.out_head, p.n);
  const uint32_t nck = p.pm_chunks;
  if (!p.pmax || p.out_head > 3 || p.n > 0xffffffffull ||
      (p.pm_chunk != kPmaxChunkSmall && p.pm_chunk != kPmaxChunkLarge) ||
      nck != pmax_chunks(p.n, head, p.pm_chunk))
    return hipErrorInvalidValue;
  uint32_t* M = reinterpret_cast<uint32_t*>(ws + p.off_pm);
  const int32_t minVal = (int32_t)p.min_u;
  const dim3 grid((nck + 3) / 4);
  if (nck <= kCarryBlock) {
    hipLaunchKernelGGL(k_pmax_scan<true>, grid, dim3(256), 0, s, out, n, head, minVal,
                       static_cast<const uint32_t*>(M), nck, p.pm_chunk);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_pmax_carry, dim3(1), dim3(kCarryBlock), 0, s, M, nck);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pmax_scan<false>, grid, dim3(256), 0, s, out, n, head, minVal,
                     static_cast<const uint32_t*>(M), nck, p.pm_chunk);
  return hipGetLastError();
}

}  // namespace rtcdf
