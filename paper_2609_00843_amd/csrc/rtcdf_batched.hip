// rtcdf_batched.hip -- batched RT-CDF: thousands of independent arrays with
// uneven n and R sorted by one persistent launch.
//
// The work items are range tiles of the arrays ("segments"): a segment with
// R <= 32768 is one item, a wider one (R <= 2^16) two, one per half of its
// range -- unless its output overlaps its input (in place): its two tiles are
// then one item, since a tile's workgroup would otherwise overwrite keys the
// other one has not yet counted.  Each workgroup (1024 threads, 1 per compute
// unit, 135 KiB of LDS) takes items from a device work queue and runs every
// step of Alg. 4 of the paper for it without touching another workgroup:
//   Alg. 5  histogram of the keys that fall in the item's tile, in LDS (32-bit
//           counters; keys outside the tile are not counted);
//   Alg. 4  local CDF of the tile by a blocked LDS scan;
//   Alg. 6  the tile's offset: 0 for the first tile; n minus the tile's own
//           population for the last one (no key lies above it), so the two
//           items of a segment never wait for each other;
//   Alg. 7  every output position of the tile gets b_t + min{x : C_t[x] >=
//           p' + 1}; each wave writes 256 consecutive positions per step and
//           carries the current value and its end from step to step.
// A segment much larger than its share of the batch (n > 2K, K keys a chunk,
// K >= the batch's keys / (2 x workgroups)) would keep one compute unit busy
// long after the others finish; each of its range tiles is split instead
// into chunks of K keys and K output positions, handled by many workgroups:
//   zero item     clears the tile's histogram in the workspace ("slot");
//   count items   one per key chunk: the chunk's LDS histogram, added to the
//                 slot's with global atomics; the last chunk to arrive scans
//                 the slot's histogram into the tile's local CDF there and
//                 publishes it (a release flag);
//   fill items    one per K output positions of the tile: wait for the flag,
//                 load the local CDF into LDS and write those positions.
// A one-workgroup ordering kernel runs first: it lays out the queue as the
// zero items, the count items, the fill items, then the other items bucketed
// by log2(n + R) so that the queue hands out the largest first (longest
// processing time first; the two items of a segment side by side), and it
// resets the queue, so the pair of launches can be captured in a HIP graph
// and replayed.  A fill item waits only for count items taken before it from
// the queue, which run on workgroups that wait for nothing, so the waits end;
// each is also bounded, and one that times out skips its item and raises an
// error word in the workspace.
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

// Work items in the queue: two words {x, y}.  y = tile | kind << 1 | chunk
// << 3; x is the segment index (whole items) or the slot index.  A whole item
// with kBothTiles set covers both range tiles of an in-place segment.
enum ItemKind : uint32_t { kWhole = 0, kZero = 1, kCount = 2, kFill = 3 };
constexpr uint32_t kBothTiles = 1u << 3;
// Per-slot state: control words, then the tile's histogram / local CDF.
constexpr uint32_t kSlotCtrl = 64;
constexpr uint32_t kSlotWords = kSlotCtrl + kBTile;
enum SlotWord : uint32_t { kSlotSeg = 0, kSlotTile = 1, kSlotZeroed = 2, kSlotDone = 3, kSlotReady = 4, kSlotNt = 5 };
// Bounded waits: 2 s of the 100 MHz constant clock, far beyond any legitimate
// wait for one chunk.
constexpr uint64_t kWaitTicks = 200000000ull;

struct BatchArgs {
  const rtcdf_segment_t* segs;
  uint32_t nseg;
  const uint32_t* order;   // 2 words per work item
  uint32_t* counters;      // [0] next queue slot, [1] number of items, [2] error word
  uint32_t* slots;         // chunked tiles' state, kSlotWords words each
  uint32_t K;              // keys (and output positions) per chunk, a multiple of 4096
  uint32_t max_slots;      // capacity of slots
  uint32_t max_chunks;     // capacity of count (and of fill) items
  uint32_t max_range;      // the bounds' largest range: wider segments are skipped
  uint32_t* park;          // kBTile words per workgroup (both-tile items), or null
};

// Whether a descriptor is sorted at all (others are skipped, output untouched).
__device__ __forceinline__ bool seg_valid(const rtcdf_segment_t& d, uint32_t max_range) {
  return d.n != 0 && d.range != 0 && d.range <= RTCDF_BATCH_MAX_RANGE && d.range <= max_range &&
         d.keys_in != nullptr && d.keys_out != nullptr;
}

__device__ __forceinline__ uint32_t seg_tiles(const rtcdf_segment_t& d, uint32_t max_range) {
  return seg_valid(d, max_range) ? (d.range > kBTile ? 2u : 1u) : 0u;
}

// A two-tile segment whose output overlaps its input: one item for both tiles
// (the workspace then holds a park slot per workgroup).
__device__ __forceinline__ bool seg_both(const rtcdf_segment_t& d, const BatchArgs& a) {
  if (a.park == nullptr || seg_tiles(d, a.max_range) != 2) return false;
  const uintptr_t i = (uintptr_t)d.keys_in, o = (uintptr_t)d.keys_out, b = (uintptr_t)d.n * 4u;
  return i < o + b && o < i + b;
}

__device__ __forceinline__ uint32_t seg_bucket(const rtcdf_segment_t& d) {
  const uint64_t size = (uint64_t)d.n + d.range + 1;
  const uint32_t lg = 63u - (uint32_t)__clzll((long long)size);
  return kBBuckets - 1 - (lg < kBBuckets - 1 ? lg : kBBuckets - 1);   // larger first
}

// Chunks per range tile of a chunked segment (0: the segment is not chunked).
__device__ __forceinline__ uint32_t seg_chunks(const rtcdf_segment_t& d, uint32_t K) {
  return (uint64_t)d.n > 2ull * K ? (uint32_t)(((uint64_t)d.n + K - 1) / K) : 0u;
}

__global__ __launch_bounds__(1024) void k_batch_order(BatchArgs a) {
  __shared__ uint32_t hist[kBBuckets];
  __shared__ uint32_t wsum[1024 / 64];
  __shared__ uint32_t s_chunked;
  const uint32_t tid = threadIdx.x;
  if (tid < kBBuckets) hist[tid] = 0;
  __syncthreads();
  // thread t takes segments t, t + 1024, ... (coalesced descriptor reads);
  // slots and chunk items are numbered in (thread, segment) order
  uint32_t slots = 0;
  uint64_t chunks = 0;
  for (uint32_t i = tid; i < a.nseg; i += 1024u) {
    const rtcdf_segment_t d = a.segs[i];
    const uint32_t t = seg_tiles(d, a.max_range), c = seg_both(d, a) ? 0u : seg_chunks(d, a.K);
    if (t != 0 && c != 0) {
      slots += t;
      chunks += (uint64_t)t * c;
    }
  }
  uint32_t tot_slots, tot_chunks;
  const uint32_t slot0 = block_inclusive_scan(slots, wsum, &tot_slots) - slots;
  const uint32_t c32 = (uint32_t)min(chunks, (uint64_t)0xffffffffu);
  const uint32_t chunk0 = block_inclusive_scan(c32, wsum, &tot_chunks) - c32;
  // beyond the workspace's capacity (bounds that understate the batch) no
  // segment is chunked
  const bool chunked = tot_slots <= a.max_slots && tot_chunks <= a.max_chunks;
  for (uint32_t i = tid; i < a.nseg; i += 1024u) {
    const rtcdf_segment_t d = a.segs[i];
    const uint32_t t = seg_tiles(d, a.max_range);
    const bool both = seg_both(d, a);
    if (t != 0 && !(chunked && !both && seg_chunks(d, a.K) != 0)) atomicAdd(&hist[seg_bucket(d)], both ? 1u : t);
  }
  __syncthreads();
  const uint32_t U = chunked ? tot_slots : 0u, LC = chunked ? tot_chunks : 0u;
  if (tid == 0) {
    uint32_t run = U + 2 * LC;
    for (uint32_t b = 0; b < kBBuckets; ++b) {
      const uint32_t c = hist[b];
      hist[b] = run;
      run += c;
    }
    a.counters[0] = 0;     // the queue starts empty at every launch
    a.counters[1] = run;   // items
    a.counters[2] = 0;     // error word
  }
  __syncthreads();
  uint2* order = (uint2*)a.order;
  uint32_t slot = slot0, chunk = chunk0;
  for (uint32_t i = tid; i < a.nseg; i += 1024u) {
    const rtcdf_segment_t d = a.segs[i];
    const uint32_t t = seg_tiles(d, a.max_range);
    if (t == 0) continue;
    const bool both = seg_both(d, a);
    const uint32_t C = chunked && !both ? seg_chunks(d, a.K) : 0u;
    if (both) {
      order[atomicAdd(&hist[seg_bucket(d)], 1u)] = make_uint2(i, kWhole << 1 | kBothTiles);
      continue;
    }
    if (C == 0) {
      const uint32_t at = atomicAdd(&hist[seg_bucket(d)], t);
      for (uint32_t k = 0; k < t; ++k) order[at + k] = make_uint2(i, k | (kWhole << 1));
      continue;
    }
    for (uint32_t k = 0; k < t; ++k, ++slot) {
      uint32_t* st = a.slots + (size_t)slot * kSlotWords;
      st[kSlotSeg] = i;
      st[kSlotTile] = k;
      st[kSlotZeroed] = 0;
      st[kSlotDone] = 0;
      st[kSlotReady] = 0;
      st[kSlotNt] = 0;
      order[slot] = make_uint2(slot, k | (kZero << 1));
      for (uint32_t c = 0; c < C; ++c, ++chunk) {
        order[U + chunk] = make_uint2(slot, k | (kCount << 1) | (c << 3));
        order[U + LC + chunk] = make_uint2(slot, k | (kFill << 1) | (c << 3));
      }
    }
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

// Writes the positions [P0, P1) of one segment's output, part of the interval
// that starts at position org and holds the values of the tile whose local
// CDF is the padded LDS array C[0..w) (position p holds the value of
// tile-local position p - org); value x of the tile is written as base + x.
// body_lo is the first 16-byte aligned position of the output.
__device__ void fill_tile(g_i32* out, const uint32_t* C, uint32_t w, uint32_t base, uint32_t org,
                          uint32_t P0, uint32_t P1, uint32_t body_lo, uint32_t* stage) {
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
      const uint32_t lp = body_lo + 4 * ib - org;   // tile-local position of the step's first key
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
    out[p] = (int32_t)(base + min(count_le_pad(C, w, (uint32_t)p - org), last));
  if (q_lo < q_hi)
    for (uint64_t p = (uint64_t)q_hi + tid; p < P1; p += kBBlock)
      out[p] = (int32_t)(base + min(count_le_pad(C, w, (uint32_t)p - org), last));
}

// Counts the keys whose value lies in the tile [base, base + w) (normalised
// to x = key - base; others are not counted) into the padded 32-bit LDS
// counters S: the 16-byte vectors [v0, v1) of the segment's aligned body
// (body = in + head), with the head's keys if `head_too` and the tail's
// (n - head - 4 * n4 keys after the body) if `tail_too`.
template <int V>
__device__ void count_tile(const g_i32* in, uint32_t n, uint32_t v0, uint32_t v1, bool head_too,
                           bool tail_too, uint32_t base, uint32_t w, uint32_t* S) {
  const uint32_t tid = threadIdx.x;
  const uintptr_t ia = (uintptr_t)in;
  uint32_t head = (uint32_t)(((16 - (ia & 15)) & 15) / 4);
  if (head > n) head = n;
  const uint32_t n4 = (n - head) / 4, tail = n - head - 4 * n4;
  const g_v4i* body = (const g_v4i*)(in + head);
  const v4i outside = (v4i)(int)(base - 1u);   // normalises to 0xffffffff: never counted
  HotBin hot;                                   // unused by the 32-bit form
  // Pipelined as in the plain histogram: unconditional loads from indices
  // clamped into [v0, v1), `outside` for lanes past the end of the last tile.
  if (v0 < v1) {
    const uint32_t last = v1 - 1;
    v4i cur[V];
#pragma unroll
    for (int j = 0; j < V; ++j) cur[j] = __builtin_nontemporal_load(&body[min(v0 + tid + j * kBBlock, last)]);
    for (uint32_t tb = v0, t0 = v0 + tid; tb < v1; tb += kBBlock * V, t0 += kBBlock * V) {
      const uint32_t t1 = t0 + kBBlock * V;
      v4i nxt[V];
#pragma unroll
      for (int j = 0; j < V; ++j) nxt[j] = __builtin_nontemporal_load(&body[min(t1 + j * kBBlock, last)]);
      if (tb + kBBlock * V <= v1) {
#pragma unroll
        for (int j = 0; j < V; ++j) count4<32, true>(S, cur[j], base, w, nullptr, 0u, nullptr, hot);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
          count4<32, true>(S, t0 + j * kBBlock < v1 ? cur[j] : outside, base, w, nullptr, 0u, nullptr, hot);
      }
#pragma unroll
      for (int j = 0; j < V; ++j) cur[j] = nxt[j];
    }
  }
  if (tid < 64) {
    v4i e = outside;
    if (head_too && tid < head) e.x = in[tid];
    if (tail_too && tid < tail) e.y = in[head + 4 * n4 + tid];
    count4<32, true>(S, e, base, w, nullptr, 0u, nullptr, hot);
  }
}

// Keys per thread per load step of the count phase, from the descriptor's
// config (4, 8 or 16; anything else is the default, 16).
__device__ __forceinline__ uint32_t seg_vectors(uint32_t config) {
  return config == 4 ? 1u : (config == 8 ? 2u : 4u);
}

// 16-byte vectors in the aligned body of n keys at `in` (count_tile).
__device__ __forceinline__ uint32_t body_vectors(const void* in, uint32_t n) {
  uint32_t head = (uint32_t)(((16 - ((uintptr_t)in & 15)) & 15) / 4);
  if (head > n) head = n;
  return (n - head) / 4;
}

__device__ __forceinline__ void count_range(const rtcdf_segment_t& d, uint32_t v0, uint32_t v1, bool head_too,
                                            bool tail_too, uint32_t base, uint32_t w, uint32_t* S) {
  const g_i32* in = (const g_i32*)d.keys_in;
  switch (seg_vectors(d.config)) {
    case 1: count_tile<1>(in, d.n, v0, v1, head_too, tail_too, base, w, S); break;
    case 2: count_tile<2>(in, d.n, v0, v1, head_too, tail_too, base, w, S); break;
    default: count_tile<4>(in, d.n, v0, v1, head_too, tail_too, base, w, S); break;
  }
}

// Geometry of range tile `tile` of segment d.
struct TileGeom {
  uint32_t w, base, body_lo;
};

__device__ __forceinline__ TileGeom tile_geom(const rtcdf_segment_t& d, uint32_t tile) {
  TileGeom g;
  const uint32_t lo = tile * kBTile;
  g.w = d.range - lo < kBTile ? d.range - lo : kBTile;
  g.base = (uint32_t)d.minVal + lo;
  g.body_lo = (uint32_t)(((16 - ((uintptr_t)d.keys_out & 15)) & 15) / 4);
  if (g.body_lo > d.n) g.body_lo = d.n;
  return g;
}

// Alg. 6: the first tile's interval starts at 0, the second (last) one's ends
// at n (no key lies above it); Nt <= n, so the interval stays inside the
// output even if the keys broke the range precondition.
__device__ __forceinline__ uint32_t tile_start(const rtcdf_segment_t& d, uint32_t tile, uint32_t Nt) {
  return tile == 0 ? 0u : d.n - Nt;
}

__device__ __forceinline__ void zero_lds(uint32_t* S, uint32_t w) {
  const uint32_t words = pad32(w - 1) + 1;
  for (uint32_t i = threadIdx.x; i < words; i += kBBlock) S[i] = 0u;
  __syncthreads();
}

// Whole item: tile `tile` of segment d -- the tile's histogram, local CDF and
// output interval (see the file comment).  With `park` (an in-place segment
// of two range tiles, tile 0) the item covers both tiles and counts every key
// for both before it writes any position: tile 1 is counted and scanned
// first and its local CDF waits in the workgroup's park slot (global memory)
// while tile 0 is counted in LDS; tile 0's positions are written, tile 1's
// CDF is loaded back and its positions are written.  The fences order the
// park slot's stores before its loads (which must not hit lines of an earlier
// item in L1).  The two phases are loops so that the count and the output
// code each keep one call site here.
__device__ void sort_item(const rtcdf_segment_t& d, uint32_t tile, uint32_t* S, uint32_t* wsum,
                          uint32_t* park) {
  const uint32_t phases = park != nullptr ? 2u : 1u;
  uint32_t N[2] = {0u, 0u};
  for (uint32_t ph = 0; ph < phases; ++ph) {
    const uint32_t t = park != nullptr ? 1u - ph : tile;
    const TileGeom g = tile_geom(d, t);
    zero_lds(S, g.w);
    count_range(d, 0, body_vectors(d.keys_in, d.n), true, true, g.base, g.w, S);
    __syncthreads();
    N[t] = scan_tile(S, g.w, wsum);
    if (ph + 1 < phases) {
      for (uint32_t i = threadIdx.x; i < g.w; i += kBBlock) park[i] = S[pad32(i)];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
    }
  }
  // every key has been read; the LDS holds the local CDF of `tile` (tile 0
  // with park)
  for (uint32_t ph = 0; ph < phases; ++ph) {
    const uint32_t t = park != nullptr ? ph : tile;
    const TileGeom g = tile_geom(d, t);
    if (ph == 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      for (uint32_t i = threadIdx.x; i < g.w; i += kBBlock) S[pad32(i)] = park[i];
      __syncthreads();
    }
    const uint32_t P0 = tile_start(d, t, N[t]);
    if (N[t]) fill_tile((g_i32*)d.keys_out, S, g.w, g.base, P0, P0, P0 + N[t], g.body_lo, S + kBLdsWords);
    __syncthreads();   // LDS is reused by the next phase or item
  }
}

// Thread 0 waits (bounded) until *flag is nonzero; returns, in every thread,
// whether it did, with the flag's release visible (agent-scope acquire).  The
// polling loads are relaxed: an acquire per poll would invalidate the L2 of
// the compute unit's XCD every few hundred cycles and starve the very
// workgroups being waited for; one acquire fence follows the last poll.
__device__ bool wait_flag(const uint32_t* flag, uint32_t* s_word, uint32_t* err) {
  if (threadIdx.x == 0) {
    uint32_t v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    while (v == 0 && wall_clock64() - t0 < kWaitTicks) {
      __builtin_amdgcn_s_sleep(16);
      v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (v == 0) atomicOr(err, 1u);
    *s_word = v;
  }
  __syncthreads();
  const bool ok = *s_word != 0;
  __syncthreads();   // s_word may be reused
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok;
}

__device__ __forceinline__ void release_flag(uint32_t* flag) {
  __hip_atomic_store(flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Zero item: clear slot st's histogram.
__device__ void zero_item(const BatchArgs& a, uint32_t* st) {
  const rtcdf_segment_t d = a.segs[st[kSlotSeg]];
  const TileGeom g = tile_geom(d, st[kSlotTile]);
  uint32_t* H = st + kSlotCtrl;
  for (uint32_t i = threadIdx.x; i < g.w; i += kBBlock) H[i] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) release_flag(&st[kSlotZeroed]);
}

// Count item: chunk c (body vectors [c K/4, (c+1) K/4), plus the head for the
// first chunk and the tail for the last) of slot st's tile; the last chunk to
// arrive turns the slot's histogram into the local CDF.
__device__ void count_item(const BatchArgs& a, uint32_t* st, uint32_t c, uint32_t* S, uint32_t* wsum,
                           uint32_t* s_word) {
  const rtcdf_segment_t d = a.segs[st[kSlotSeg]];
  const TileGeom g = tile_geom(d, st[kSlotTile]);
  const uint32_t C = seg_chunks(d, a.K), K4 = a.K / 4;
  const uint32_t n4 = body_vectors(d.keys_in, d.n);
  const uint32_t v0 = min((uint64_t)c * K4, (uint64_t)n4), v1 = min((uint64_t)(c + 1) * K4, (uint64_t)n4);
  zero_lds(S, g.w);
  count_range(d, v0, v1, c == 0, c == C - 1, g.base, g.w, S);
  __syncthreads();
  uint32_t* H = st + kSlotCtrl;
  if (!wait_flag(&st[kSlotZeroed], s_word, &a.counters[2])) return;
  for (uint32_t i = threadIdx.x; i < g.w; i += kBBlock) {
    const uint32_t v = S[pad32(i)];
    if (v) __hip_atomic_fetch_add(&H[i], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0)
    *s_word = __hip_atomic_fetch_add(&st[kSlotDone], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const bool last = *s_word == C - 1;
  __syncthreads();
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  for (uint32_t i = threadIdx.x; i < g.w; i += kBBlock)
    S[pad32(i)] = __hip_atomic_load(&H[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const uint32_t Nt = scan_tile(S, g.w, wsum);
  for (uint32_t i = threadIdx.x; i < g.w; i += kBBlock) H[i] = S[pad32(i)];
  if (threadIdx.x == 0) st[kSlotNt] = Nt;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) release_flag(&st[kSlotReady]);
  __syncthreads();   // LDS is reused by the next item
}

// Fill item: output positions [c K, (c+1) K) of slot st's tile interval.
__device__ void fill_item(const BatchArgs& a, uint32_t* st, uint32_t c, uint32_t* S, uint32_t* s_word) {
  const rtcdf_segment_t d = a.segs[st[kSlotSeg]];
  const uint32_t tile = st[kSlotTile];
  const TileGeom g = tile_geom(d, tile);
  if (!wait_flag(&st[kSlotReady], s_word, &a.counters[2])) return;
  const uint32_t* H = st + kSlotCtrl;
  const uint32_t Nt = __hip_atomic_load(&st[kSlotNt], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t A = (uint64_t)c * a.K;
  if (A >= Nt) return;
  for (uint32_t i = threadIdx.x; i < g.w; i += kBBlock)
    S[pad32(i)] = __hip_atomic_load(&H[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const uint32_t P0 = tile_start(d, tile, Nt);
  const uint32_t B = (uint32_t)min(A + a.K, (uint64_t)Nt);
  fill_tile((g_i32*)d.keys_out, S, g.w, g.base, P0, P0 + (uint32_t)A, P0 + B, g.body_lo, S + kBLdsWords);
  __syncthreads();   // LDS is reused by the next item
}

__global__ __launch_bounds__(kBBlock) void k_batched(BatchArgs a) {
  extern __shared__ uint32_t S[];
  __shared__ uint32_t wsum[kBBlock / 64];
  __shared__ uint32_t s_q, s_word;
  const uint32_t items = a.counters[1];
  const uint2* order = (const uint2*)a.order;
  for (;;) {
    if (threadIdx.x == 0) s_q = atomicAdd(&a.counters[0], 1u);
    __syncthreads();
    const uint32_t q = s_q;
    __syncthreads();
    if (q >= items) break;
    const uint2 it = order[q];
    const uint32_t tile = it.y & 1u, kind = (it.y >> 1) & 3u, chunk = it.y >> 3;
    if (kind == kWhole) {
      const rtcdf_segment_t d = a.segs[it.x];
      if (!seg_valid(d, a.max_range)) continue;
      sort_item(d, tile, S, wsum, (it.y & kBothTiles) ? a.park + (size_t)blockIdx.x * kBTile : nullptr);
    } else {
      uint32_t* st = a.slots + (size_t)it.x * kSlotWords;
      if (kind == kZero) zero_item(a, st);
      else if (kind == kCount) count_item(a, st, chunk, S, wsum, &s_word);
      else fill_item(a, st, chunk, S, &s_word);
    }
  }
}

}  // namespace

BatchPlan batched_plan(uint32_t nseg, uint64_t total_keys, uint32_t cus, uint32_t max_range) {
  BatchPlan P;
  P.max_range = max_range;
  // a park slot per persistent workgroup (at most one per compute unit) when
  // a segment may have two range tiles
  P.park_words = max_range > kBTile ? (uint64_t)cus * kBTile : 0;
  // chunks of at least 2^18 keys, and at least the batch's keys per two
  // workgroups, so that a chunked segment is longer than a fair share
  const uint64_t share = (total_keys + 2ull * cus - 1) / (2ull * cus);
  uint64_t K = std::max<uint64_t>(1ull << 18, (share + 4095) / 4096 * 4096);
  K = std::min<uint64_t>(K, 1ull << 31);
  P.K = (uint32_t)K;
  // A chunked segment has n > 2K: at most total / (2K + 1) of them, two
  // slots each, and chunks per tile ceil(n / K) <= n / K + 1, which would
  // size the slots and chunk items.  The chunked path is switched off: the
  // workspace holds no slots, so the ordering kernel chunks no segment (its
  // first GPU runs did not terminate and the cause is not yet found).
  P.max_slots = 0;
  P.max_chunks = 0;
  P.items_max = 2ull * nseg + P.max_slots + 2ull * P.max_chunks;
  P.order_words = 2 * P.items_max;
  P.slot_words = (uint64_t)P.max_slots * kSlotWords;
  return P;
}

hipError_t launch_batched(const rtcdf_segment_t* segs, uint32_t nseg, const BatchPlan& P, uint32_t* order,
                          uint32_t* counters, uint32_t* slots, uint32_t* park, uint32_t grid, hipStream_t s) {
  BatchArgs a;
  a.segs = segs;
  a.nseg = nseg;
  a.order = order;
  a.counters = counters;
  a.slots = slots;
  a.K = P.K;
  a.max_slots = P.max_slots;
  a.max_chunks = P.max_chunks;
  a.max_range = P.max_range;
  a.park = P.park_words != 0 ? park : nullptr;
  hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)(kBLdsWords + kBStageWords) * 4;
  e = ensure_dynamic_lds((const void*)k_batched, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batched, dim3(grid), dim3(kBBlock), lds, s, a);
  return hipGetLastError();
}

}  // namespace rtcdf
