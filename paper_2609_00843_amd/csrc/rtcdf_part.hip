// rtcdf_part.hip -- coarse partition of the keys by LDS pass, for wide ranges.
//
// When the range needs several LDS passes (R above the ~161792 bins of one
// pass of 8-bit counters), the histogram of Alg. 5 as built here reads every
// key once per pass.  The partition sorts the keys once by pass (bucket
// b = x / W of the normalised value x) into a workspace copy, so that each key
// is read once by the histogram, in its own pass: about 12 more bytes per key
// once (read for the counts, read and write for the scatter) instead of 4
// bytes per key per extra pass.  The histogram's workgroups cut the copy into
// equal ranges whatever the bucket sizes (k_hist).  It is a counting sort by
// bucket, in three launches:
//   k_part_count    workgroup g counts the keys of its slice of the input per
//                   bucket in LDS and writes the column cnt[b * G + g].
//   k_part_scan     one workgroup per bucket: exclusive scan of cnt[b * G + .]
//                   over the slices in place, bucket total into tot[b].
//   k_part_scatter  every workgroup forms the bucket starts (each bucket
//                   padded to a multiple of 4 keys) from the totals, then
//                   moves its slice tile by tile: the keys of a tile are
//                   grouped by bucket in LDS and written as runs at
//                   start[b] + cnt[b * G + g] + (keys of the bucket in earlier
//                   tiles).  Workgroup 0 writes the bucket starts for the
//                   histogram, fills the padding with a key that lies
//                   outside every pass, and writes each pass's partial-row
//                   range for the reduction.
// Keys outside [minVal, maxVal) go to no bucket (their output is unspecified,
// as on every path) and never index memory out of bounds.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rtcdf_device.h"
#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

using namespace dev;

constexpr uint32_t kPartBlock = 256;
constexpr uint32_t kPartItems = 32;                        // keys per thread per tile
constexpr uint32_t kPartTile = kPartBlock * kPartItems;    // 8192 keys
static_assert(kPartTile == kPartTileKeys, "the planner sizes slices in these tiles");

struct PartArgs {
  const int32_t* keys;
  uint32_t n, per;          // keys; keys per slice (workgroup)
  uint32_t min_u, R, W, P;  // P buckets of W values (the last one shorter)
  uint32_t SUB;             // LDS sub-counters per bucket (lane & (SUB - 1)): few buckets
                            // would otherwise put many lanes of a wave on one LDS word
  float invW;
  uint32_t G;               // slices
  uint32_t* cnt;            // P x G
  uint32_t* tot;            // P
  uint32_t* bound;          // P + 1 padded bucket starts
  int32_t* part;            // the partitioned keys
  // The histogram's partial rows of each bucket (its first row and their
  // number, 2 words per bucket), for hist_grid histogram workgroups that cut
  // the padded copy into equal ranges of 16-byte vectors (k_hist).
  uint32_t hist_grid;
  uint32_t* prow;
};

// Bucket of key k, or P for a key outside the range.
__device__ __forceinline__ uint32_t bucket_of(int32_t k, const PartArgs& a) {
  const uint32_t x = (uint32_t)k - a.min_u;
  if (x >= a.R) return a.P;
  // x < 2^28: the float quotient is off by at most one
  uint32_t b = (uint32_t)((float)x * a.invW);
  if (b * a.W > x) --b;
  else if ((b + 1) * a.W <= x) ++b;
  return b < a.P ? b : a.P - 1;
}

__global__ __launch_bounds__(kPartBlock) void k_part_count(PartArgs a) {
  extern __shared__ uint32_t L[];   // P x SUB counters
  const uint32_t g = blockIdx.x, tid = threadIdx.x;
  const uint32_t sub = tid & (a.SUB - 1), E = a.P * a.SUB;
  for (uint32_t b = tid; b < E; b += kPartBlock) L[b] = 0u;
  __syncthreads();
  const uint64_t lo = (uint64_t)g * a.per;
  const uint64_t hi = std::min<uint64_t>(lo + a.per, a.n);
  for (uint64_t t = lo; t < hi; t += kPartTile) {
    int32_t k[kPartItems];
#pragma unroll
    for (uint32_t j = 0; j < kPartItems; ++j) {
      const uint64_t i = t + j * kPartBlock + tid;
      k[j] = i < hi ? a.keys[i] : 0;
    }
#pragma unroll
    for (uint32_t j = 0; j < kPartItems; ++j) {
      const uint64_t i = t + j * kPartBlock + tid;
      const uint32_t b = bucket_of(k[j], a);
      if (i < hi && b < a.P) atomicAdd(&L[b * a.SUB + sub], 1u);
    }
  }
  __syncthreads();
  for (uint32_t b = tid; b < a.P; b += kPartBlock) {
    uint32_t c = 0;
    for (uint32_t q = 0; q < a.SUB; ++q) c += L[b * a.SUB + q];
    a.cnt[(size_t)b * a.G + g] = c;
  }
}

constexpr uint32_t kPartScanBlock = 1024;

__global__ __launch_bounds__(kPartScanBlock) void k_part_scan(PartArgs a) {
  __shared__ uint32_t wsum[kPartScanBlock / 64];
  const uint32_t b = blockIdx.x, tid = threadIdx.x;
  uint32_t* col = a.cnt + (size_t)b * a.G;
  uint32_t run = 0;
  for (uint32_t g0 = 0; g0 < a.G; g0 += kPartScanBlock) {
    const uint32_t g = g0 + tid;
    const uint32_t v = g < a.G ? col[g] : 0u;
    uint32_t total;
    const uint32_t inc = block_inclusive_scan(v, wsum, &total);
    if (g < a.G) col[g] = run + inc - v;
    run += total;
  }
  if (tid == 0) a.tot[b] = run;
}

__global__ __launch_bounds__(kPartBlock) void k_part_scatter(PartArgs a) {
  // LDS: base[P] (next output index of each bucket for this slice), the
  // tile's counters cntL[E] and their exclusive starts lstart[E + 1] in
  // bucket-major order (E = P x SUB), then the tile's keys.
  extern __shared__ uint32_t L[];
  __shared__ uint32_t wsum[kPartBlock / 64];
  const uint32_t E = a.P * a.SUB;
  uint32_t* base = L;
  uint32_t* cntL = L + a.P;
  uint32_t* lstart = cntL + E;
  int32_t* stage = reinterpret_cast<int32_t*>(lstart + E + 1);
  const uint32_t g = blockIdx.x, tid = threadIdx.x, sub = tid & (a.SUB - 1);
  const uint32_t per_t = (a.P + kPartBlock - 1) / kPartBlock;   // buckets per thread
  const uint32_t b0 = std::min(a.P, tid * per_t), b1 = std::min(a.P, b0 + per_t);
  const uint32_t per_e = (E + kPartBlock - 1) / kPartBlock;     // counters per thread
  const uint32_t e0 = std::min(E, tid * per_e), e1 = std::min(E, e0 + per_e);

  // Padded bucket starts: exclusive scan of round_up4(tot[b]).
  uint32_t s = 0;
  for (uint32_t b = b0; b < b1; ++b) s += (a.tot[b] + 3u) & ~3u;
  uint32_t total;
  uint32_t start = block_inclusive_scan(s, wsum, &total) - s;
  for (uint32_t b = b0; b < b1; ++b) {
    const uint32_t len = a.tot[b];
    base[b] = start + a.cnt[(size_t)b * a.G + g];
    if (g == 0) {
      a.bound[b] = start;
      const int32_t pad = (int32_t)(a.min_u - 1u);   // normalised value 2^32 - 1: outside every pass
      for (uint32_t q = len; q < ((len + 3u) & ~3u); ++q) a.part[start + q] = pad;
      // workgroups j0..j1 of the histogram hold the bucket's vectors
      // [s4, e4); their pieces are rows j + b
      const uint32_t per4 = (total / 4 + a.hist_grid - 1) / a.hist_grid;
      const uint32_t s4 = start / 4, e4 = (start + ((len + 3u) & ~3u)) / 4;
      const uint32_t j0 = e4 > s4 ? s4 / per4 : 0u, j1 = e4 > s4 ? (e4 - 1) / per4 : 0u;
      a.prow[2 * b] = j0 + b;
      a.prow[2 * b + 1] = e4 > s4 ? j1 - j0 + 1 : 0u;
    }
    start += (len + 3u) & ~3u;
  }
  if (g == 0 && tid == kPartBlock - 1) a.bound[a.P] = total;
  __syncthreads();

  const uint64_t lo = (uint64_t)g * a.per;
  const uint64_t hi = std::min<uint64_t>(lo + a.per, a.n);
  for (uint64_t t = lo; t < hi; t += kPartTile) {
    for (uint32_t q = tid; q < E; q += kPartBlock) cntL[q] = 0u;
    __syncthreads();
    int32_t k[kPartItems];
    uint32_t bk[kPartItems], rk[kPartItems];
#pragma unroll
    for (uint32_t j = 0; j < kPartItems; ++j) {
      const uint64_t i = t + j * kPartBlock + tid;
      k[j] = i < hi ? a.keys[i] : 0;
    }
#pragma unroll
    for (uint32_t j = 0; j < kPartItems; ++j) {
      const uint64_t i = t + j * kPartBlock + tid;
      bk[j] = i < hi ? bucket_of(k[j], a) : a.P;
      rk[j] = bk[j] < a.P ? atomicAdd(&cntL[bk[j] * a.SUB + sub], 1u) : 0u;
    }
    __syncthreads();
    // tile-local starts of every (bucket, sub-counter), bucket-major
    uint32_t c = 0;
    for (uint32_t q = e0; q < e1; ++q) c += cntL[q];
    uint32_t tile_keys;
    uint32_t ls = block_inclusive_scan(c, wsum, &tile_keys) - c;
    for (uint32_t q = e0; q < e1; ++q) {
      lstart[q] = ls;
      ls += cntL[q];
    }
    if (tid == 0) lstart[E] = tile_keys;
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kPartItems; ++j)
      if (bk[j] < a.P) stage[lstart[bk[j] * a.SUB + sub] + rk[j]] = k[j];
    __syncthreads();
    // runs of one bucket go to consecutive output indices
    for (uint32_t i = tid; i < tile_keys; i += kPartBlock) {
      const int32_t key = stage[i];
      const uint32_t b = bucket_of(key, a);
      a.part[base[b] + (i - lstart[b * a.SUB])] = key;
    }
    __syncthreads();
    for (uint32_t b = tid; b < a.P; b += kPartBlock) base[b] += lstart[(b + 1) * a.SUB] - lstart[b * a.SUB];
    __syncthreads();
  }
}

}  // namespace

// Sub-counters per bucket: up to 16, with at most 1024 counters in all
// (a power of two, so that lane & (SUB - 1) picks one).
static uint32_t partition_subcounters(uint32_t P) {
  uint32_t s = 16;
  while (s > 1 && (size_t)P * s > 1024) s >>= 1;
  return s;
}

size_t partition_lds_bytes(uint32_t P) {
  const size_t E = (size_t)P * partition_subcounters(P);
  return (P + 2 * E + 1 + kPartTile) * 4;
}

hipError_t launch_partition(const Plan& p, const int32_t* keys, uint8_t* ws, hipStream_t s) {
  if (!p.part || p.part_buckets != p.passes || p.part_grid == 0 || p.n > 0xffffffffull ||
      (uint64_t)p.part_per * p.part_grid < p.n || p.part_buckets > kPartMaxBuckets)
    return hipErrorInvalidValue;
  PartArgs a;
  a.keys = keys;
  a.n = (uint32_t)p.n;
  a.per = p.part_per;
  a.min_u = p.min_u;
  a.R = p.R;
  a.W = p.W;
  a.P = p.part_buckets;
  a.SUB = partition_subcounters(a.P);
  a.invW = 1.0f / (float)p.W;
  a.G = p.part_grid;
  a.cnt = reinterpret_cast<uint32_t*>(ws + p.off_pcnt);
  a.tot = reinterpret_cast<uint32_t*>(ws + p.off_ptot);
  a.bound = reinterpret_cast<uint32_t*>(ws + p.off_pbound);
  a.part = reinterpret_cast<int32_t*>(ws + p.off_pkeys);
  a.hist_grid = p.passes * p.G;
  a.prow = reinterpret_cast<uint32_t*>(ws + p.off_prow);
  hipLaunchKernelGGL(k_part_count, dim3(a.G), dim3(kPartBlock), (size_t)a.P * a.SUB * 4, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_part_scan, dim3(a.P), dim3(kPartScanBlock), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = partition_lds_bytes(a.P);
  // raised once, to the size for the most buckets
  e = ensure_dynamic_lds((const void*)k_part_scatter, (int)partition_lds_bytes(kPartMaxBuckets));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_part_scatter, dim3(a.G), dim3(kPartBlock), lds, s, a);
  return hipGetLastError();
}

}  // namespace rtcdf
