// rtcdf_batched.hip -- batched RT-CDF: thousands of independent arrays with
// uneven n and R sorted by one persistent launch.
//
// The work items are range tiles of the arrays ("segments"): a segment with
// R <= 32768 is one item, a wider one (R <= 2^16) two, one per half of its
// range.  Each workgroup (1024 threads, 1 per compute unit, 135 KiB of LDS)
// takes items from a device work queue and runs every step of Alg. 4 of the
// paper for it without touching another workgroup:
//   Alg. 5  histogram of the keys that fall in the item's tile, in LDS (32-bit
//           counters; keys outside the tile are not counted);
//   Alg. 4  local CDF of the tile by a blocked LDS scan;
//   Alg. 6  the tile's offset: 0 for the first tile; n minus the tile's own
//           population for the last one (no key lies above it), so the two
//           items of a segment never wait for each other;
//   Alg. 7  every output position of the tile gets b_t + min{x : C_t[x] >=
//           p' + 1}; each wave writes 256 consecutive positions per step and
//           carries the current value and its end from step to step.
// A one-workgroup ordering kernel runs first: it lists the items bucketed by
// log2(n + R) so that the queue hands out the largest first (longest
// processing time first; the two items of a segment side by side), and it
// resets the queue, so the pair of launches can be captured in a HIP graph
// and replayed.
#include <hip/hip_runtime.h>

#include "rtcdf_device.h"
#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

using namespace dev;

// Segment keys are reached through pointers read from device memory, which
// the compiler cannot place in an address space; these global (address space
// 1) types keep their loads and stores out of the flat form, whose counters
// would make every LDS wait also wait for them.
typedef __attribute__((address_space(1))) int32_t g_i32;
typedef __attribute__((address_space(1))) v4i g_v4i;

constexpr uint32_t kBBlock = 1024;
constexpr uint32_t kBTile = 32768;                   // values per local CDF tile
constexpr uint32_t kBLdsWords = 33792;               // pad32(kBTile): LDS words of one padded tile
constexpr uint32_t kBStageWords = kBBlock / 64 * 256;  // per-wave output staging (sparse steps)
constexpr uint32_t kBBuckets = 34;
static_assert(RTCDF_BATCH_MAX_RANGE <= 2 * kBTile, "a segment is at most two tiles");

struct BatchArgs {
  const rtcdf_segment_t* segs;
  uint32_t nseg;
  const uint32_t* order;   // work items: 2 x segment index + tile
  uint32_t* counters;      // [0] next queue slot, [1] number of items
};

// Whether a descriptor is sorted at all (others are skipped, output untouched).
__device__ __forceinline__ bool seg_valid(const rtcdf_segment_t& d) {
  return d.n != 0 && d.range != 0 && d.range <= RTCDF_BATCH_MAX_RANGE && d.keys_in != nullptr &&
         d.keys_out != nullptr;
}

__device__ __forceinline__ uint32_t seg_tiles(const rtcdf_segment_t& d) {
  return seg_valid(d) ? (d.range > kBTile ? 2u : 1u) : 0u;
}

__device__ __forceinline__ uint32_t seg_bucket(const rtcdf_segment_t& d) {
  const uint64_t size = (uint64_t)d.n + d.range + 1;
  const uint32_t lg = 63u - (uint32_t)__clzll((long long)size);
  return kBBuckets - 1 - (lg < kBBuckets - 1 ? lg : kBBuckets - 1);   // larger first
}

__global__ __launch_bounds__(1024) void k_batch_order(const rtcdf_segment_t* segs, uint32_t nseg,
                                                      uint32_t* order, uint32_t* counters) {
  __shared__ uint32_t hist[kBBuckets];
  if (threadIdx.x < kBBuckets) hist[threadIdx.x] = 0;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nseg; i += blockDim.x) {
    const uint32_t t = seg_tiles(segs[i]);
    if (t) atomicAdd(&hist[seg_bucket(segs[i])], t);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (uint32_t b = 0; b < kBBuckets; ++b) {
      const uint32_t c = hist[b];
      hist[b] = run;
      run += c;
    }
    counters[0] = 0;     // the queue starts empty at every launch
    counters[1] = run;   // items
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nseg; i += blockDim.x) {
    const uint32_t t = seg_tiles(segs[i]);
    if (t == 0) continue;
    const uint32_t at = atomicAdd(&hist[seg_bucket(segs[i])], t);
    for (uint32_t k = 0; k < t; ++k) order[at + k] = 2 * i + k;
  }
}

// In-place inclusive scan of the padded LDS array C[0..w); returns the total.
__device__ uint32_t scan_tile(uint32_t* C, uint32_t w, uint32_t* wsum) {
  const uint32_t tid = threadIdx.x;
  const uint32_t L = (w + kBBlock - 1) / kBBlock;
  const uint32_t s0 = tid * L < w ? tid * L : w;
  const uint32_t s1 = s0 + L < w ? s0 + L : w;
  uint32_t run = 0;
  for (uint32_t i = s0; i < s1; ++i) {
    run += C[pad32(i)];
    C[pad32(i)] = run;
  }
  uint32_t total;
  const uint32_t before = block_inclusive_scan(run, wsum, &total) - run;
  for (uint32_t i = s0; i < s1; ++i) C[pad32(i)] += before;
  __syncthreads();
  return total;
}

// Writes the positions [P0, P1) of one segment's output, which hold the values
// of the tile whose local CDF is the padded LDS array C[0..w); value x of the
// tile is written as base + x.  body_lo is the first 16-byte aligned position
// of the output.
__device__ void fill_tile(g_i32* out, const uint32_t* C, uint32_t w, uint32_t base, uint32_t P0,
                          uint32_t P1, uint32_t body_lo, uint32_t* stage) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t last = w - 1;
  // aligned vectors inside [P0, P1)
  const uint32_t a0 = P0 > body_lo ? P0 : body_lo;
  const uint32_t q_lo = body_lo + ((a0 - body_lo + 3u) & ~3u);
  const uint32_t q_hi = P1 > body_lo ? body_lo + ((P1 - body_lo) & ~3u) : body_lo;
  if (q_lo < q_hi) {
    g_v4i* body = (g_v4i*)(out + body_lo);
    const uint32_t i_lo = (q_lo - body_lo) >> 2, i_hi = (q_hi - body_lo) >> 2;
    uint32_t xw = 0, end = 0;
    bool started = false;
    // Each wave writes a contiguous run of 64-vector steps, so the value index
    // it carries from step to step moves by one step's worth of values.
    const uint32_t steps = (i_hi - i_lo + 63) / 64, per_wave = (steps + kBBlock / 64 - 1) / (kBBlock / 64);
    const uint32_t ib0 = i_lo + wave * per_wave * 64;
    const uint32_t ib1 = min(i_hi, ib0 + per_wave * 64);
    for (uint32_t ib = ib0; ib < ib1; ib += 64) {
      const uint32_t lp = body_lo + 4 * ib - P0;   // tile-local position of the step's first key
      if (!started) {
        xw = min(count_le_pad(C, w, lp), last);
        end = C[pad32(xw)];
        started = true;
      }
      // The carried value may end before this step (the previous step carried
      // the value at its last position).  A step crosses at most kWalk value
      // ends by a walk; where a look-ahead read shows more (sparse values,
      // most of them empty) it bisects or scatters instead.
      constexpr uint32_t kWalk = 8;
      if (xw < last && end <= lp) {
        if (C[pad32(min(xw + kWalk, last))] <= lp) {
          xw = upper_in_pad(C, xw, last, lp);
          end = C[pad32(xw)];
        } else {
          while (end <= lp) end = C[pad32(++xw)];
        }
      }
      v4i o;
      if (xw == last || past_step(end, lp, 256u)) {   // end > lp unless xw == last
        o = (v4i)(int32_t)(base + xw);
      } else {
        // the look-ahead and the next end are read together
        const uint32_t far = C[pad32(min(xw + kWalk, last))], e1 = C[pad32(xw + 1)];
        if (!past_step(far, lp, 256u)) {
          uint32_t* st = stage + wave * 256u;
          scatter_step([&](uint32_t x) { return C[pad32(x)]; }, xw, last, lp, st);
          const v4i sv = *reinterpret_cast<const v4i*>(st + 4 * lane);
          o = (v4i)(int32_t)base + sv;
          xw = min(st[255], last);   // the value at the step's last position
          end = C[pad32(xw)];
        } else {
          const uint32_t p = lp + 4 * lane;
          uint32_t c0 = end <= p, c1 = end <= p + 1, c2 = end <= p + 2, c3 = end <= p + 3;
          uint32_t xb = xw + 1, e = e1;
          while (xb < last && !past_step(e, lp, 256u)) {   // fewer than kWalk more ends
            c0 += e <= p;
            c1 += e <= p + 1;
            c2 += e <= p + 2;
            c3 += e <= p + 3;
            e = C[pad32(++xb)];
          }
          o.x = (int32_t)(base + xw + c0);
          o.y = (int32_t)(base + xw + c1);
          o.z = (int32_t)(base + xw + c2);
          o.w = (int32_t)(base + xw + c3);
          xw = xb;                   // the value at the step's last position
          end = e;
        }
      }
      const uint32_t i = ib + lane;
      if (i < i_hi) __builtin_nontemporal_store(o, &body[i]);
    }
  }
  // scalar positions: before the first and after the last aligned vector
  const uint32_t s_end = q_lo < q_hi ? q_lo : P1;
  // (64-bit positions, widened before the thread index is added: q_hi + tid
  // and p + kBBlock would wrap near 2^32)
  for (uint64_t p = (uint64_t)P0 + tid; p < s_end; p += kBBlock)
    out[p] = (int32_t)(base + min(count_le_pad(C, w, (uint32_t)p - P0), last));
  if (q_lo < q_hi)
    for (uint64_t p = (uint64_t)q_hi + tid; p < P1; p += kBBlock)
      out[p] = (int32_t)(base + min(count_le_pad(C, w, (uint32_t)p - P0), last));
}

// Counts the keys of `in` whose value lies in the tile [base, base + w)
// (normalised to x = key - base; others are not counted) into the padded
// 32-bit LDS counters S.
template <int V>
__device__ void count_tile(const g_i32* in, uint32_t n, uint32_t base, uint32_t w, uint32_t* S) {
  const uint32_t tid = threadIdx.x;
  const uintptr_t ia = (uintptr_t)in;
  uint32_t head = (uint32_t)(((16 - (ia & 15)) & 15) / 4);
  if (head > n) head = n;
  const uint32_t n4 = (n - head) / 4, tail = n - head - 4 * n4;
  const g_v4i* body = (const g_v4i*)(in + head);
  const v4i outside = (v4i)(int)(base - 1u);   // normalises to 0xffffffff: never counted
  HotBin hot;                                   // unused by the 32-bit form
  // Pipelined as in the plain histogram: unconditional loads from indices
  // clamped into [0, n4), `outside` for lanes past the end of the last tile.
  if (n4 > 0) {
    const uint32_t last = n4 - 1;
    v4i cur[V];
#pragma unroll
    for (int j = 0; j < V; ++j) cur[j] = __builtin_nontemporal_load(&body[min(tid + j * kBBlock, last)]);
    for (uint32_t tb = 0, t0 = tid; tb < n4; tb += kBBlock * V, t0 += kBBlock * V) {
      const uint32_t t1 = t0 + kBBlock * V;
      v4i nxt[V];
#pragma unroll
      for (int j = 0; j < V; ++j) nxt[j] = __builtin_nontemporal_load(&body[min(t1 + j * kBBlock, last)]);
      if (tb + kBBlock * V <= n4) {
#pragma unroll
        for (int j = 0; j < V; ++j) count4<32, true>(S, cur[j], base, w, nullptr, 0u, nullptr, hot);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
          count4<32, true>(S, t0 + j * kBBlock < n4 ? cur[j] : outside, base, w, nullptr, 0u, nullptr, hot);
      }
#pragma unroll
      for (int j = 0; j < V; ++j) cur[j] = nxt[j];
    }
  }
  if (tid < 64) {
    v4i e = outside;
    if (tid < head) e.x = in[tid];
    if (tid < tail) e.y = in[head + 4 * n4 + tid];
    count4<32, true>(S, e, base, w, nullptr, 0u, nullptr, hot);
  }
}

// Keys per thread per load step of the count phase, from the descriptor's
// config (4, 8 or 16; anything else is the default, 16).
__device__ __forceinline__ uint32_t seg_vectors(uint32_t config) {
  return config == 4 ? 1u : (config == 8 ? 2u : 4u);
}

// Work item `tile` of segment d: the tile's histogram, local CDF and output
// interval (see the file comment).
__device__ void sort_item(const rtcdf_segment_t& d, uint32_t tile, uint32_t* S, uint32_t* wsum) {
  const uint32_t tid = threadIdx.x;
  const uint32_t n = d.n, R = d.range;
  const g_i32* in = (const g_i32*)d.keys_in;
  g_i32* out = (g_i32*)d.keys_out;
  const uint32_t lo = tile * kBTile;
  const uint32_t w = R - lo < kBTile ? R - lo : kBTile;
  const uint32_t base = (uint32_t)d.minVal + lo;
  const uintptr_t oa = (uintptr_t)out;
  uint32_t body_lo = (uint32_t)(((16 - (oa & 15)) & 15) / 4);
  if (body_lo > n) body_lo = n;
  const uint32_t words = pad32(w - 1) + 1;
  for (uint32_t i = tid; i < words; i += kBBlock) S[i] = 0u;
  __syncthreads();
  switch (seg_vectors(d.config)) {
    case 1: count_tile<1>(in, n, base, w, S); break;
    case 2: count_tile<2>(in, n, base, w, S); break;
    default: count_tile<4>(in, n, base, w, S); break;
  }
  __syncthreads();
  const uint32_t Nt = scan_tile(S, w, wsum);
  // Alg. 6: the first tile starts at 0, the last one ends at n (no key lies
  // above it); Nt <= n, so the interval stays inside the output even if the
  // keys broke the range precondition.
  const uint32_t P0 = tile == 0 ? 0u : n - Nt;
  if (Nt) fill_tile(out, S, w, base, P0, P0 + Nt, body_lo, S + kBLdsWords);
  __syncthreads();   // LDS is reused by the next item
}

__global__ __launch_bounds__(kBBlock) void k_batched(BatchArgs a) {
  extern __shared__ uint32_t S[];
  __shared__ uint32_t wsum[kBBlock / 64];
  __shared__ uint32_t s_q;
  const uint32_t items = a.counters[1];
  for (;;) {
    if (threadIdx.x == 0) s_q = atomicAdd(&a.counters[0], 1u);
    __syncthreads();
    const uint32_t q = s_q;
    __syncthreads();
    if (q >= items) break;
    const uint32_t it = a.order[q];
    const rtcdf_segment_t d = a.segs[it >> 1];
    if (seg_valid(d)) sort_item(d, it & 1u, S, wsum);
  }
}

}  // namespace

size_t batched_order_words(uint32_t nseg) { return 2ull * nseg; }

hipError_t launch_batched(const rtcdf_segment_t* segs, uint32_t nseg, uint32_t* order, uint32_t* counters,
                          uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, segs, nseg, order, counters);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)(kBLdsWords + kBStageWords) * 4;
  e = ensure_dynamic_lds((const void*)k_batched, (int)lds);
  if (e != hipSuccess) return e;
  BatchArgs a;
  a.segs = segs;
  a.nseg = nseg;
  a.order = order;
  a.counters = counters;
  hipLaunchKernelGGL(k_batched, dim3(grid), dim3(kBBlock), lds, s, a);
  return hipGetLastError();
}

}  // namespace rtcdf
