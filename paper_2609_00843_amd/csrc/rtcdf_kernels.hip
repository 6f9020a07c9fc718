// rtcdf_kernels.hip -- gfx950 kernels of the plain RT-CDF sort.
//
// Stages (Sec. 3, Alg. 4), one launch each:
//   k_hist      tile histograms in LDS (Alg. 5).  All tiles of one LDS pass are
//               counted by one workgroup; every workgroup then writes its LDS
//               counters as one partial row (coalesced, non-atomic) instead of
//               the per-bin global atomics of Alg. 5.
//   k_reduce    sums the partial rows of each bin -> H[R], plus per-128-bin
//               block totals used for the tile offsets.  With the
//               prefix-maximum output (Alg. 3) its extra workgroups write the
//               initial B.
//   k_tilescan  one or more workgroups per range tile: local CDF by inclusive
//               scan (Alg. 4), tile offset O[t] (Alg. 6, as a sum of the block
//               totals before the tile), and the value found at each output
//               chunk boundary ("splitters", by bisection in the local CDF as in
//               Alg. 7).  Every workgroup of a tile scans the tile in its own
//               LDS; the first one writes the CDF and O[t], and each takes an
//               equal share of the tile's chunk boundaries.  With few tiles the
//               workgroups are given to tiles in proportion to their chunk
//               boundaries, which the kernel reads from the block totals.
//               With the prefix-maximum output it writes the steps of Alg. 3
//               instead of splitters (rtcdf_pmax.hip finishes the output).
//   k_fill      one workgroup per output chunk: loads the inclusive cumulative
//               counts O[t] + C_t[x] of the values that cover the chunk into LDS
//               and writes every position p the value b_t + min{x : C_t[x] >= p'+1}
//               (Alg. 7 with p' = p - O[t]) as 16-byte stores.
//   k_fill_small  single-tile fast path (one tile, one LDS pass of 32-bit
//               counters, R <= 2048): the histogram workgroups add their counts
//               into accumulation rows with global atomics, and every output
//               workgroup sums and scans those counts in its own LDS and finds
//               its chunks' boundaries itself (no k_reduce / k_tilescan launch).
#include <hip/hip_runtime.h>

#include "rtcdf_device.h"
#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

using namespace dev;

// ------------------------------------------------------------------ histogram

struct HistArgs {
  const int32_t* keys;
  uint32_t in_n4, in_per;   // n < 2^32 keys: vector indices fit 32 bits
  uint32_t in_head, in_tail;
  uint32_t min_u, W, passes, G, row_words, R;
  int64_t min64;         // int64 keys: normalised value x = key - min64 (min_u is 0)
  uint32_t wrap_slots;   // narrow forms: slots of the LDS wrap table (a power of two)
  uint32_t sub_log;      // 32-bit counters: 2^sub_log LDS copies per bin (count4's SPREAD)
  uint32_t interleave;
  uint32_t* partial;
  uint32_t* carry;
  // Single-tile fast path (merge != 0): add the counts into row
  // blockIdx % merge (rows of merge_stride words) of the current region of the
  // fast-path area in `carry` instead of writing a partial row.
  uint32_t merge, merge_stride;
  // Partition mode (non-null): `keys` is the partitioned copy and pass p reads
  // keys[pbound[p], pbound[p + 1]) (16-byte aligned, whole vectors).
  const uint32_t* pbound;
  // 8- and 16-bit keys: every key's bits are XORed with `flip` (its sign bit
  // for signed keys, 0 for unsigned) and zero-extended, which maps the key
  // order onto the unsigned order; min_u is then in that domain.
  uint32_t flip;
};

// The normalised value of an int64 key: key - min64, exact in 64 bits, or
// 0xffffffff (counted nowhere) if that is not below R.
__device__ __forceinline__ uint32_t norm64(uint32_t lo, uint32_t hi, int64_t min64, uint32_t R) {
  const uint64_t x = (((uint64_t)hi << 32) | lo) - (uint64_t)min64;
  return x < R ? (uint32_t)x : 0xffffffffu;
}

// One 16-byte vector of keys: 4 int32 keys, 8 / 16 narrow keys widened in
// groups of four, or 2 int64 keys normalised (with min_u 0, so base is the
// pass's first bin) and padded with two keys outside every pass.  Lanes
// without a valid vector count `outside` (every group, so that the wave-wide
// ballots inside count4 see every lane).
template <int BITS, int KB, bool DEDUPE = false, bool SPREAD = false>
__device__ __forceinline__ void count_vec(uint32_t* S, v4i v, bool valid, v4i outside, uint32_t flip,
                                          uint32_t base, uint32_t W, uint32_t* carry, uint32_t pass_lo,
                                          uint32_t* tab, HotBin& hot, int64_t min64 = 0, uint32_t R = 0,
                                          uint32_t sub_log = 0) {
  if constexpr (KB == 8) {
    const v4i g = {(int)norm64((uint32_t)v.x, (uint32_t)v.y, min64, R),
                   (int)norm64((uint32_t)v.z, (uint32_t)v.w, min64, R), outside.x, outside.x};
    count4<BITS, false, false, SPREAD>(S, valid ? g : outside, base, W, carry, pass_lo, tab, hot, sub_log);
  } else if constexpr (KB == 4) {
    count4<BITS, false, DEDUPE, SPREAD>(S, valid ? v : outside, base, W, carry, pass_lo, tab, hot, sub_log);
  } else if constexpr (KB == 2) {
    const uint32_t f = flip | (flip << 16);
    const uint32_t w[4] = {(uint32_t)v.x ^ f, (uint32_t)v.y ^ f, (uint32_t)v.z ^ f, (uint32_t)v.w ^ f};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const v4i g = {(int)(w[2 * h] & 0xffffu), (int)(w[2 * h] >> 16), (int)(w[2 * h + 1] & 0xffffu),
                     (int)(w[2 * h + 1] >> 16)};
      count4<BITS, false, false, SPREAD>(S, valid ? g : outside, base, W, carry, pass_lo, tab, hot, sub_log);
    }
  } else {
    const uint32_t f = flip * 0x01010101u;
    const uint32_t w[4] = {(uint32_t)v.x ^ f, (uint32_t)v.y ^ f, (uint32_t)v.z ^ f, (uint32_t)v.w ^ f};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const v4i g = {(int)(w[h] & 0xffu), (int)((w[h] >> 8) & 0xffu), (int)((w[h] >> 16) & 0xffu),
                     (int)(w[h] >> 24)};
      count4<BITS, false, false, SPREAD>(S, valid ? g : outside, base, W, carry, pass_lo, tab, hot, sub_log);
    }
  }
}

// Key i of a scalar head or tail, widened (or, for int64 keys, normalised) as
// in count_vec.
template <int KB>
__device__ __forceinline__ int32_t load_key(const int32_t* keys, size_t i, uint32_t flip, int64_t min64 = 0,
                                            uint32_t R = 0) {
  if constexpr (KB == 8) {
    const uint64_t k = reinterpret_cast<const uint64_t*>(keys)[i];
    return (int32_t)norm64((uint32_t)k, (uint32_t)(k >> 32), min64, R);
  } else if constexpr (KB == 4) return keys[i];
  else if constexpr (KB == 2) return (int32_t)(reinterpret_cast<const uint16_t*>(keys)[i] ^ flip);
  else return (int32_t)(reinterpret_cast<const uint8_t*>(keys)[i] ^ flip);
}

// Counts the vectors body[t, end) of one pass, t = t0 + k * step for the
// workgroup's tiles of BLOCK * ITEMS / 4 vectors, into the LDS counters S.
// Software pipelined: the loads of the next tile are in flight while the
// current one is counted.  Every load is issued unconditionally from an
// index clamped into [0, end), so that the compiler can wait for the current
// tile's loads alone rather than for all loads in flight; in the workgroup's
// last, partial tile the lanes past the end count `outside`.
template <int ITEMS, int BITS, int BLOCK, int KB, bool DEDUPE, bool SPREAD = false>
__device__ __forceinline__ void count_tiles(const HistArgs& a, uint32_t* S, uint32_t* tab, HotBin& hot,
                                            const v4i* body, uint32_t t0, uint32_t step, uint32_t end,
                                            uint32_t base, uint32_t pass_lo, v4i outside) {
  constexpr int V = ITEMS / 4;
  const uint32_t W = a.W;
  if (end == 0) return;
  const uint32_t last = end - 1;
  // first vector of the workgroup's tile (uniform: kept in a scalar register)
  uint32_t tb = (uint32_t)__builtin_amdgcn_readfirstlane((int)(t0 - threadIdx.x));
  v4i cur[V];
#pragma unroll
  for (int j = 0; j < V; ++j) cur[j] = __builtin_nontemporal_load(&body[min(t0 + j * BLOCK, last)]);
  while (tb < end) {
    const uint32_t t1 = t0 + step;
    v4i nxt[V];
#pragma unroll
    for (int j = 0; j < V; ++j) nxt[j] = __builtin_nontemporal_load(&body[min(t1 + j * BLOCK, last)]);
    if (tb + V * BLOCK <= end) {
#pragma unroll
      for (int j = 0; j < V; ++j)
        count_vec<BITS, KB, DEDUPE, SPREAD>(S, cur[j], true, outside, a.flip, base, W, a.carry, pass_lo, tab,
                                            hot, a.min64, a.R, a.sub_log);
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j)
        count_vec<BITS, KB, DEDUPE, SPREAD>(S, cur[j], t0 + j * BLOCK < end, outside, a.flip, base, W, a.carry,
                                            pass_lo, tab, hot, a.min64, a.R, a.sub_log);
    }
#pragma unroll
    for (int j = 0; j < V; ++j) cur[j] = nxt[j];
    t0 = t1;
    tb += step;
  }
}

// Zero LDS counters (all copies with SPREAD) and (narrow forms) an empty wrap
// table: its slot mask, its bins and its amounts.
template <int BITS, int BLOCK, bool SPREAD = false>
__device__ __forceinline__ void init_counters(const HistArgs& a, uint32_t* S, uint32_t* tab) {
  const uint32_t words = SPREAD ? a.row_words << a.sub_log : a.row_words;
  for (uint32_t i = threadIdx.x; i < words; i += BLOCK) S[i] = 0u;
  if constexpr (BITS < 32) {
    if (threadIdx.x == 0) tab[-1] = a.wrap_slots - 1u;
    for (uint32_t i = threadIdx.x; i < 2 * a.wrap_slots; i += BLOCK) tab[i] = i < a.wrap_slots ? kWrapEmpty : 0u;
  }
  __syncthreads();
}

// Partition by pass: the padded copy holds the keys grouped by bucket (bucket
// b, the keys of pass b, at pbound[b], a multiple of 4 keys; padding counts
// nowhere).  The grid cuts the whole copy into equal ranges of vectors,
// whatever the bucket sizes (a skewed input puts nearly every key in one
// bucket), and a workgroup counts each bucket its range overlaps in turn.
// The piece of bucket b in workgroup j's range goes to partial row j + b:
// the pieces of one bucket belong to consecutive workgroups, and no two
// nonempty pieces share a row (a later bucket starts after an earlier one
// ends), so the reduction finds bucket b's rows from its bounds alone.
template <int ITEMS, int BITS, int BLOCK, int KB, bool DEDUPE>
__device__ __forceinline__ void hist_partitioned(const HistArgs& a, uint32_t* S, uint32_t* tab) {
  constexpr int V = ITEMS / 4;
  const uint32_t* pb = a.pbound;
  const uint32_t total4 = pb[a.passes] / 4;
  const uint32_t per4 = (total4 + gridDim.x - 1) / gridDim.x;
  const uint32_t r0 = min(blockIdx.x * per4, total4), r1 = min(r0 + per4, total4);
  // first bucket that ends after r0
  uint32_t b = 0, hi = a.passes;
  while (b < hi) {
    const uint32_t mid = (b + hi) >> 1;
    if (pb[mid + 1] / 4 <= r0) b = mid + 1; else hi = mid;
  }
  const v4i* all = reinterpret_cast<const v4i*>(a.keys);
  for (; b < a.passes; ++b) {
    const uint32_t b0 = pb[b] / 4, b1 = pb[b + 1] / 4;
    if (b0 >= r1) break;
    const uint32_t s0 = max(r0, b0), s1 = min(r1, b1);
    if (s0 >= s1) continue;
    init_counters<BITS, BLOCK>(a, S, tab);
    const uint32_t pass_lo = b * a.W;
    const uint32_t base = a.min_u + pass_lo;
    HotBin hot;
    count_tiles<ITEMS, BITS, BLOCK, KB, DEDUPE>(a, S, tab, hot, all + s0, threadIdx.x, BLOCK * V, s1 - s0, base,
                                                pass_lo, (v4i)(int)(base - 1u));
    if constexpr (BITS < 32 || DEDUPE) hot_flush_any<BITS, false>(hot, S, tab, a.carry, pass_lo);
    __syncthreads();
    if constexpr (BITS < 32) wrap_flush(tab, a.carry, pass_lo, threadIdx.x);
    uint32_t* row = a.partial + ((size_t)blockIdx.x + b) * a.row_words;
    for (uint32_t i = threadIdx.x; i < a.row_words; i += BLOCK) row[i] = S[i];
    __syncthreads();   // S is zeroed again for the next bucket
  }
}

// Counter i of the workgroup's LDS histogram: the sum of its copies with
// SPREAD, else the word itself.
template <bool SPREAD>
__device__ __forceinline__ uint32_t counter_sum(const HistArgs& a, const uint32_t* S, uint32_t i) {
  if constexpr (SPREAD) {
    uint32_t t = 0;
    for (uint32_t c = 0; c < (1u << a.sub_log); ++c) t += S[(i << a.sub_log) + c];
    return t;
  } else {
    return S[i];
  }
}

// DEDUPE: wave-level aggregation of frequent values (RTCDF_FLAG_WAVE_DEDUPE,
// int32 keys only), a separate instantiation so that the default counting
// loop carries none of its instructions.  SPREAD: LDS copies of the 32-bit
// counters (count4), summed into the partial row or the merge rows.
template <int ITEMS, int BITS, int BLOCK, int KB = 4, bool DEDUPE = false, bool SPREAD = false>
__global__ __launch_bounds__(BLOCK) void k_hist(HistArgs a) {
  // The planner's LDS budget: kLdsBytes per 1024 threads (one workgroup per
  // compute unit at 1024 threads, two at 512, four at 256).  A static array
  // lets the compiler fold its base into the LDS instructions.
  __shared__ uint32_t S[kLdsBytes / 4 / (1024 / BLOCK)];
  // XCD-aware mapping: workgroup ids are dealt round-robin to the 8 XCDs, so
  // the `passes` workgroups that read the same input chunk get consecutive
  // slots on one XCD and the rescans of later passes can hit that XCD's L2.
  const uint32_t wg = blockIdx.x, xcd = wg & 7u, slot = wg >> 3;
  const uint32_t pass = slot % a.passes;
  const uint32_t chunk = (slot / a.passes) * 8u + xcd;
  // LDS: the counters, then (narrow forms) the wrap table: its slot mask, its
  // bins and its amounts.
  uint32_t* tab = S + a.row_words + 1;
  if constexpr (!SPREAD) {
    if (a.pbound != nullptr) {
      hist_partitioned<ITEMS, BITS, BLOCK, KB, DEDUPE>(a, S, tab);
      return;
    }
  }
  init_counters<BITS, BLOCK, SPREAD>(a, S, tab);

  const uint32_t pass_lo = pass * a.W;
  const uint32_t base = a.min_u + pass_lo;   // key (as uint32) of bin 0 of this pass
  const uint32_t W = a.W;

  // this pass's input: the whole array
  const int32_t* keys = a.keys;
  const uint32_t in_n4 = a.in_n4, in_per = a.in_per, in_head = a.in_head, in_tail = a.in_tail;

  constexpr int V = ITEMS / 4;
  constexpr uint32_t VK = 16 / KB;   // keys per 16-byte vector
  const v4i* body = reinterpret_cast<const v4i*>(reinterpret_cast<const uint8_t*>(keys) + (size_t)in_head * KB);
  const v4i outside = (v4i)(int)(base - 1u);   // lands outside every pass
  HotBin hot;                                  // narrow forms only
  uint32_t t0, step, end;
  if (a.interleave) {
    // Tiles of BLOCK * V vectors dealt round-robin to the G chunks of a pass:
    // at any moment the whole grid reads one contiguous window of the input.
    t0 = chunk * BLOCK * V + threadIdx.x;
    step = BLOCK * V * a.G;
    end = in_n4;
  } else {
    const uint32_t c0 = chunk * in_per;
    t0 = c0 + threadIdx.x;
    step = BLOCK * V;
    end = c0 + in_per < in_n4 ? c0 + in_per : in_n4;
  }
  count_tiles<ITEMS, BITS, BLOCK, KB, DEDUPE, SPREAD>(a, S, tab, hot, body, t0, step, end, base, pass_lo,
                                                      outside);
  // scalar head and tail keys (at most VK - 1 each), counted by chunk 0 / chunk G-1
  v4i e = outside;
  if (chunk == 0 && threadIdx.x < in_head) e.x = load_key<KB>(keys, threadIdx.x, a.flip, a.min64, a.R);
  if (chunk == a.G - 1 && threadIdx.x < in_tail)
    e.y = load_key<KB>(keys, in_head + VK * (size_t)in_n4 + threadIdx.x, a.flip, a.min64, a.R);
  if (threadIdx.x < 64) count4<BITS, false, false, SPREAD>(S, e, base, W, a.carry, pass_lo, tab, hot, a.sub_log);
  if constexpr (BITS < 32 || DEDUPE) hot_flush_any<BITS, false>(hot, S, tab, a.carry, pass_lo);
  __syncthreads();
  if constexpr (BITS < 32) wrap_flush(tab, a.carry, pass_lo, threadIdx.x);

  if (BITS == 32 && a.merge) {
    // Few bins (the fast path): the workgroup adds its counts to one of
    // several rows of the current region, zero on entry, instead of writing a
    // partial row; the rows spread the atomics over more addresses.
    const uint32_t par = a.carry[kFastPar] & 1u;
    uint32_t* acc = a.carry + par * kFastRegionWords + (blockIdx.x % a.merge) * a.merge_stride;
    for (uint32_t i = threadIdx.x; i < a.R; i += BLOCK) {
      const uint32_t v = counter_sum<SPREAD>(a, S, i);
      if (v != 0u) atomicAdd(&acc[i], v);
    }
    if (blockIdx.x == 0) {   // the previous sort's region: zero for the next sort
      uint32_t* other = a.carry + (par ^ 1u) * kFastRegionWords;
      for (uint32_t i = threadIdx.x; i < kFastRegionWords; i += BLOCK) other[i] = 0u;
      if (threadIdx.x == 0) a.carry[kFastCur] = par;
    }
    return;
  }
  uint32_t* row = a.partial + ((size_t)pass * a.G + chunk) * a.row_words;
  for (uint32_t i = threadIdx.x; i < a.row_words; i += BLOCK) row[i] = counter_sum<SPREAD>(a, S, i);
}

// ------------------------------------------------------------------ reduction

struct ReduceArgs {
  const uint32_t* partial;
  uint32_t* carry;
  uint32_t* hist;
  uint32_t* rsum;
  uint32_t* flags;   // cleared here for the local-CDF stage
  uint32_t R, W, G, row_words, carry_words, bits;
  // Partition by pass (non-null): pass p's partial rows are prow[2p] and the
  // prow[2p + 1] rows after it (the pieces of bucket p in the histogram
  // workgroups' ranges, hist_partitioned), written by the partition.
  const uint32_t* prow;
  // Prefix-maximum output (Alg. 3): workgroups nred and up write the initial
  // B[0, pm_n) = pm_fill and clear the pm_nck chunk maxima pm_M.  pm_out is
  // null otherwise.
  uint32_t nred;
  int32_t* pm_out;
  uint32_t pm_n, pm_head, pm_nck;
  int32_t pm_fill;
  uint32_t* pm_M;
};

// B[0, n) = fill (16-byte stores after the `head` scalars) and M[0, nck) = 0,
// grid-stride over `workers` workgroups; `worker` is this workgroup's index.
__device__ __forceinline__ void pmax_initial_fill(int32_t* out, uint32_t n, uint32_t head, int32_t fill,
                                                  uint32_t* M, uint32_t nck, uint32_t worker,
                                                  uint32_t workers) {
  const size_t stride = (size_t)workers * blockDim.x;
  const size_t gid = (size_t)worker * blockDim.x + threadIdx.x;
  if (gid < head) out[gid] = fill;
  const uint32_t n4 = (n - head) / 4;
  v4i* body = reinterpret_cast<v4i*>(out + head);
  const v4i f = {fill, fill, fill, fill};
  for (size_t i = gid; i < n4; i += stride) body[i] = f;
  const uint32_t tail = head + n4 * 4;
  if (gid < n - tail) out[tail + gid] = fill;
  for (size_t i = gid; i < nck; i += stride) M[i] = 0u;
}

// One workgroup per 128-bin block of one pass: the block is 128 / (32 / bits)
// words of every partial row of the pass.  Threads are RG row groups x NQ word
// quads (NQ = 32, 16, 8, 4 for 32-, 16-, 8-, 4-bit counters; RG = 32, or 64
// for 4-bit counters: 1024, 512, 256, 256 threads);
// each thread adds the 16-byte quad of every 32nd row, four loads in flight,
// and splits the words into their counters.  The row groups are summed in LDS;
// every bin adds (and re-zeroes) its carry entry (narrow counters), and the
// workgroup writes H and the block total.
__host__ __device__ constexpr uint32_t reduce_groups(uint32_t bits) { return bits == 4 ? 64u : 32u; }

template <int BITS>
__device__ __forceinline__ void reduce_block(const ReduceArgs& a, uint32_t (*red)[kReduceBins + 1],
                                             uint32_t* wsum) {
  constexpr uint32_t per = 32 / BITS, NQ = kReduceBins / per / 4, RG = reduce_groups(BITS);
  const uint32_t tid = threadIdx.x, q = tid % NQ, rg = tid / NQ;
  const uint32_t r0 = blockIdx.x * kReduceBins;   // first bin (passes hold W bins, W % 128 == 0)
  const uint32_t pass = r0 / a.W, w0 = (r0 - pass * a.W) / per;
  const size_t rs4 = a.row_words / 4;
  size_t row0 = (size_t)pass * a.G;
  uint32_t G = a.G;   // rows of the pass
  if (a.prow != nullptr) {
    row0 = a.prow[2 * pass];
    G = a.prow[2 * pass + 1];
  }
  const v4u* src = reinterpret_cast<const v4u*>(a.partial + row0 * a.row_words + w0) + q;
  uint32_t acc[4 * per];
#pragma unroll
  for (uint32_t k = 0; k < 4 * per; ++k) acc[k] = 0;
  auto add = [&](const v4u w) {
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
      if constexpr (BITS == 32) {
        acc[j] += ws[j];
      } else if constexpr (BITS == 16) {
        acc[2 * j] += ws[j] & 0xffffu;
        acc[2 * j + 1] += ws[j] >> 16;
      } else if constexpr (BITS == 8) {
        acc[4 * j] += ws[j] & 0xffu;
        acc[4 * j + 1] += (ws[j] >> 8) & 0xffu;
        acc[4 * j + 2] += (ws[j] >> 16) & 0xffu;
        acc[4 * j + 3] += ws[j] >> 24;
      } else {
#pragma unroll
        for (uint32_t f = 0; f < 8; ++f) acc[8 * j + f] += (ws[j] >> (4 * f)) & 0xfu;
      }
    }
  };
  uint32_t g = rg;
  const uint32_t NG = RG;
  for (; g + 3 * NG < G; g += 4 * NG) {
    const v4u x0 = src[(size_t)g * rs4], x1 = src[(size_t)(g + NG) * rs4];
    const v4u x2 = src[(size_t)(g + 2 * NG) * rs4], x3 = src[(size_t)(g + 3 * NG) * rs4];
    add(x0);
    add(x1);
    add(x2);
    add(x3);
  }
  for (; g < G; g += NG) add(src[(size_t)g * rs4]);
  // bin 4 * per * q + k of the block = counter k % per of word 4q + k / per
#pragma unroll
  for (uint32_t k = 0; k < 4 * per; ++k) red[rg][4 * per * q + k] = acc[k];
  __syncthreads();
  uint32_t tot = 0;
  if (tid < kReduceBins) {
    for (uint32_t r = 0; r < RG; ++r) tot += red[r][tid];
    const uint32_t bin = r0 + tid;
    if (BITS < 32 && bin < a.carry_words) {
      tot += a.carry[bin];
      a.carry[bin] = 0u;   // keep the carry array zero between sorts
    }
    if (bin < a.R) a.hist[bin] = tot;
    else tot = 0u;
  }
  const uint32_t sum = block_sum(tid < kReduceBins ? tot : 0u, wsum);
  if (tid == 0) a.rsum[blockIdx.x] = sum;
}

__global__ __launch_bounds__(kReduceBlock) void k_reduce(ReduceArgs a) {
  // the row-group sums: reduce_groups(bits) rows of kReduceBins + 1 words
  // (dynamic, so that the narrow widths keep the occupancy of a 16 KiB block)
  extern __shared__ uint32_t red_lds[];
  auto red = reinterpret_cast<uint32_t (*)[kReduceBins + 1]>(red_lds);
  __shared__ uint32_t wsum[kReduceBlock / 64];
  if (blockIdx.x >= a.nred) {   // prefix-maximum output: the initial B
    pmax_initial_fill(a.pm_out, a.pm_n, a.pm_head, a.pm_fill, a.pm_M, a.pm_nck, blockIdx.x - a.nred,
                      gridDim.x - a.nred);
    return;
  }
  if (a.bits == 32) reduce_block<32>(a, red, wsum);
  else if (a.bits == 16) reduce_block<16>(a, red, wsum);
  else if (a.bits == 8) reduce_block<8>(a, red, wsum);
  else reduce_block<4>(a, red, wsum);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.flags[0] = 0u;
}

// ---------------------------------------------------------- local CDF + O[t]

struct ScanArgs {
  const uint32_t* hist;   // H (tile histograms)
  uint32_t* cdf;          // out: local CDFs
  const uint32_t* rsum;
  uint32_t* O;
  uint32_t* split;
  uint64_t n;
  uint32_t R, T, out_head, chunk, nchunks, S;
  uint32_t m, grid;   // tiles; workgroups (grid > m: assigned by chunk counts)
  uint32_t pre_O;     // per-tile path: O[t] was written by k_tile_offsets
  uint32_t* flags;    // [0] set if some chunk's window holds over chunk / sparse_k values
  uint32_t sparse_k;
  // Prefix-maximum output (Alg. 3; pm_out null otherwise): the first
  // workgroup of each tile writes B[P1[d-1]] = minVal + d for every value d >= 1
  // of the tile with keys, and the chunk maxima M (last step of each
  // pm_chunk-position chunk); no splitters are needed.
  int32_t* pm_out;
  uint32_t pm_head, pm_chunk;
  int32_t pm_min;
  uint32_t* pm_M;
};

// Alg. 6 for the plans whose local-CDF workgroups are not given to tiles by
// their chunk counts (many tiles or many block totals): one workgroup forms
// every tile total from the 128-bin block totals and writes the exclusive
// scan O[0, m).  Each thread takes a contiguous run of tiles.
__global__ __launch_bounds__(kScanBlock) void k_tile_offsets(const uint32_t* __restrict__ rsum, uint32_t nred,
                                                             uint32_t nb, uint32_t m, uint32_t* __restrict__ O) {
  __shared__ uint32_t wsum[kScanBlock / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (m + kScanBlock - 1) / kScanBlock;
  const uint32_t t0 = min(m, tid * per), t1 = min(m, t0 + per);
  const uint32_t k1 = min(nred, t1 * nb);
  uint32_t s = 0;
  for (uint32_t k = t0 * nb; k < k1; ++k) s += rsum[k];
  uint32_t total;
  uint32_t run = block_inclusive_scan(s, wsum, &total) - s;
  for (uint32_t t = t0; t < t1; ++t) {
    O[t] = run;
    const uint32_t ke = min(nred, (t + 1) * nb);
    for (uint32_t k = t * nb; k < ke; ++k) run += rsum[k];
  }
}

// First output chunk whose start position s(k) is >= P, where s(0) = 0 and
// s(k) = out_head + k * chunk for k >= 1.
__device__ __forceinline__ uint32_t first_chunk_at_or_after(uint64_t P, uint32_t h,
                                                            uint32_t chunk, uint32_t nchunks) {
  if (P == 0) return 0;
  uint64_t k = 1;
  if (P > h) {
    const uint64_t q = (P - h + chunk - 1) / chunk;
    if (q > k) k = q;
  }
  return k < nchunks ? (uint32_t)k : nchunks;
}

__global__ __launch_bounds__(kScanBlock) void k_tilescan(ScanArgs a) {
  extern __shared__ uint32_t C[];
  __shared__ uint32_t wsum[kScanBlock / 64];
  __shared__ uint32_t tiles[kScanBlock];
  __shared__ uint32_t sel[4];
  const uint32_t tid = threadIdx.x;
  uint32_t t, part, S, Ot;
  if (a.m == 1) {
    t = 0;
    part = blockIdx.x;
    S = gridDim.x;
    Ot = 0;
  } else if (a.grid > a.m) {
    // At most kScanBlock tiles and 8 * kScanBlock block totals: every
    // workgroup derives the same assignment of the grid to tiles, one
    // workgroup per tile plus the spare ones in proportion to the number of
    // output chunks that start inside each tile (all-equal keys put every
    // chunk in one tile).  Tile totals first (nb block totals per tile), then
    // thread i handles tile i.
    const uint32_t nb = a.T / kReduceBins, nred = (a.R + kReduceBins - 1) / kReduceBins;
    tiles[tid] = 0u;
    __syncthreads();
    for (uint32_t k0 = 0; k0 < nred; k0 += kScanBlock) {
      const uint32_t k = k0 + tid;
      const uint32_t v = k < nred ? a.rsum[k] : 0u;
      if ((nb & 63u) == 0u) {   // a wave's 64 totals then belong to one tile
        // (T a multiple of 8192; any other multiple of 128 puts tile
        // boundaries inside waves, so each total is added on its own)
        const uint32_t ws = wave_sum(v);
        if (lane_id() == 0 && k < nred) atomicAdd(&tiles[k / nb], ws);
      } else if (k < nred) {
        atomicAdd(&tiles[k / nb], v);
      }
    }
    __syncthreads();
    const uint32_t Ni = tid < a.m ? tiles[tid] : 0u;
    uint32_t total;
    const uint32_t Oi = block_inclusive_scan(Ni, wsum, &total) - Ni;   // Alg. 6
    uint32_t ci = 0;
    if (tid < a.m && Ni > 0)
      ci = first_chunk_at_or_after((uint64_t)Oi + Ni, a.out_head, a.chunk, a.nchunks) -
           first_chunk_at_or_after(Oi, a.out_head, a.chunk, a.nchunks);
    const uint64_t extra = a.grid - a.m;
    const uint32_t Si = tid < a.m ? 1u + (uint32_t)(extra * ci / a.nchunks) : 0u;
    uint32_t used;
    const uint32_t start = block_inclusive_scan(Si, wsum, &used) - Si;
    if (tid == 0 && blockIdx.x >= used) sel[0] = 0xffffffffu;
    if (tid < a.m && blockIdx.x >= start && blockIdx.x < start + Si) {
      sel[0] = tid;
      sel[1] = blockIdx.x - start;
      sel[2] = Si;
      sel[3] = Oi;
    }
    __syncthreads();
    t = sel[0];
    if (t == 0xffffffffu) return;   // a spare workgroup left over by the rounding
    part = sel[1];
    S = sel[2];
    Ot = sel[3];
  } else {
    t = blockIdx.x / a.S;
    part = blockIdx.x % a.S;
    S = a.S;
    // Alg. 6: O[t] = number of keys below b_t = sum of the 128-bin block
    // totals before the tile (b_t is a multiple of 128); with many tiles and
    // block totals, k_tile_offsets has written it.
    if (a.pre_O) {
      Ot = a.O[t];
    } else {
      uint32_t acc = 0;
      for (uint32_t k = tid; k < t * a.T / kReduceBins; k += kScanBlock) acc += a.rsum[k];
      Ot = block_sum(acc, wsum);
    }
  }
  const uint32_t b = t * a.T;
  const uint32_t w = a.R - b < a.T ? a.R - b : a.T;

  // Alg. 4: inclusive scan of H[b, b + w).  Coalesced copy into LDS, then
  // each thread scans a contiguous segment of L entries, one block scan of the
  // segment totals, and the segment prefix is added back.
  for (uint32_t i = tid; i < w; i += kScanBlock) C[pad32(i)] = a.hist[b + i];
  __syncthreads();
  const uint32_t L = (w + kScanBlock - 1) / kScanBlock;
  const uint32_t s0 = tid * L < w ? tid * L : w;
  const uint32_t s1 = s0 + L < w ? s0 + L : w;
  uint32_t run = 0;
  for (uint32_t i = s0; i < s1; ++i) {
    run += C[pad32(i)];
    C[pad32(i)] = run;
  }
  uint32_t Nt;
  const uint32_t before = block_inclusive_scan(run, wsum, &Nt) - run;
  for (uint32_t i = s0; i < s1; ++i) C[pad32(i)] += before;
  __syncthreads();
  if (part == 0) {
    for (uint32_t i = tid; i < w; i += kScanBlock) a.cdf[b + i] = C[pad32(i)];
    if (tid == 0) a.O[t] = Ot;
  }
  if (a.pm_out != nullptr) {
    if (part != 0) return;
    for (uint32_t i = tid; i < w; i += kScanBlock) {
      const uint32_t d = b + i;
      const uint32_t e = Ot + C[pad32(i)];                       // P1[d]
      const uint32_t s = i ? Ot + C[pad32(i - 1)] : Ot;          // P1[d - 1]
      if (d == 0 || e <= s) continue;
      a.pm_out[s] = a.pm_min + (int32_t)d;
      const uint32_t c = s < a.pm_head ? 0u : (s - a.pm_head) / a.pm_chunk;
      const uint64_t end = (uint64_t)a.pm_head + (uint64_t)(c + 1) * a.pm_chunk;
      if (e >= end || e == a.n) a.pm_M[c] = d;                 // the last step of chunk c
    }
    return;
  }
  if (Nt == 0) return;

  // Splitters: the value at every chunk start inside [O_t, O_t + N_t), and at
  // position n - 1 (closes the last chunk's window); this workgroup takes part
  // `part` of S.  Chunk starts are taken in batches of 4 per thread: each
  // thread finds its 4 consecutive starts (one bisection, then a short forward
  // walk), stages them in LDS (behind the CDF) and the batch is written out
  // with coalesced stores.
  const uint64_t lo = Ot, hi = (uint64_t)Ot + Nt;
  const uint32_t kt0 = first_chunk_at_or_after(lo, a.out_head, a.chunk, a.nchunks);
  const uint32_t kt1 = first_chunk_at_or_after(hi, a.out_head, a.chunk, a.nchunks);
  const uint32_t per = (kt1 - kt0 + S - 1) / S;
  const uint32_t k0 = min(kt0 + part * per, kt1), k1 = min(k0 + per, kt1);
  uint32_t* stage = C + pad32(a.T) + 1;   // 4 * kScanBlock words
  // 1 to 4 starts per thread: as few as cover this workgroup's share at once
  const uint32_t kPer = min(4u, max(1u, (k1 - k0 + kScanBlock - 1) / kScanBlock));
  for (uint32_t kb0 = k0; kb0 < k1; kb0 += kPer * kScanBlock) {
    const uint32_t ka = kb0 + tid * kPer;
    uint32_t x = 0;
    for (uint32_t j = 0; j < kPer && ka + j < k1; ++j) {
      const uint32_t k = ka + j;
      const uint64_t s = k == 0 ? 0 : (uint64_t)a.out_head + (uint64_t)k * a.chunk;
      const uint32_t q = (uint32_t)(s - lo);
      uint32_t steps = 0;
      if (j != 0)
        while (steps < 8u && x < w && C[pad32(x)] <= q) {
          ++x;
          ++steps;
        }
      if (j == 0 || (x < w && C[pad32(x)] <= q)) x = count_le_pad(C, w, q);
      stage[tid * kPer + j] = b + x;
    }
    __syncthreads();
    const uint32_t nbatch = min(kPer * kScanBlock, k1 - kb0);
    bool sparse = false;
    for (uint32_t j = tid; j < nbatch; j += kScanBlock) {
      a.split[kb0 + j] = stage[j];
      if (j + 1 < nbatch) sparse |= (uint64_t)(stage[j + 1] - stage[j] + 1) * a.sparse_k > a.chunk;
    }
    if (__syncthreads_or(sparse) && tid == 0) a.flags[0] = 1u;
  }
  if (part == 0 && tid == 0 && a.n - 1 >= lo && a.n - 1 < hi)
    a.split[a.nchunks] = b + count_le_pad(C, w, (uint32_t)(a.n - 1 - lo));
}

// --------------------------------------------------------------------- output

struct FillArgs {
  void* out;              // int32 keys, or 16- / 8-bit keys (kb in the plan)
  const uint32_t* cdf;    // local CDFs
  const uint32_t* O;
  const uint32_t* split;
  uint64_t n;
  uint32_t min_u, R, T, out_head, chunk, nchunks;
  int64_t min64;               // int64 keys: stored key = min64 + value (min_u is 0)
  uint64_t body_lo, body_hi;   // positions [body_lo, body_hi) are 16-byte aligned int4s
  const uint32_t* flags;       // [0]: some chunk is sparse (local-CDF stage)
  uint32_t flip;               // narrow keys: stored bits = value ^ flip
  uint32_t sparse_k;           // a chunk takes the sparse form below this many positions per value
};

// Four consecutive outputs (group i of the aligned body, 16 / 8 / 4 bytes)
// and single outputs, in the key width KB.  An int64 output is min64 plus the
// value, exact in 64 bits.
template <int KB>
__device__ __forceinline__ void store_group(const FillArgs& a, uint64_t i, v4i o) {
  if constexpr (KB == 4) {
    v4i* body = reinterpret_cast<v4i*>(static_cast<int32_t*>(a.out) + a.body_lo);
    __builtin_nontemporal_store(o, &body[i]);
  } else if constexpr (KB == 2) {
    typedef unsigned int v2u __attribute__((ext_vector_type(2)));
    const uint32_t f = a.flip;
    const v2u w = {(((uint32_t)o.x ^ f) & 0xffffu) | (((uint32_t)o.y ^ f) << 16),
                   (((uint32_t)o.z ^ f) & 0xffffu) | (((uint32_t)o.w ^ f) << 16)};
    v2u* body = reinterpret_cast<v2u*>(static_cast<uint16_t*>(a.out) + a.body_lo);
    __builtin_nontemporal_store(w, &body[i]);
  } else {
    const uint32_t f = a.flip;
    const uint32_t w = (((uint32_t)o.x ^ f) & 0xffu) | ((((uint32_t)o.y ^ f) & 0xffu) << 8) |
                       ((((uint32_t)o.z ^ f) & 0xffu) << 16) | (((uint32_t)o.w ^ f) << 24);
    uint32_t* body = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(a.out) + a.body_lo);
    __builtin_nontemporal_store(w, &body[i]);
  }
}

// 16 / KB consecutive narrow outputs (one 16-byte vector, index i of the
// aligned body in units of 16 bytes): the dense form's step for 8- and
// 16-bit keys.
template <int KB>
__device__ __forceinline__ void store_vec16(const FillArgs& a, uint64_t i, const int32_t* o) {
  const uint32_t f = a.flip;
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if constexpr (KB == 2) {
      w[q] = (((uint32_t)o[2 * q] ^ f) & 0xffffu) | (((uint32_t)o[2 * q + 1] ^ f) << 16);
    } else {
      w[q] = (((uint32_t)o[4 * q] ^ f) & 0xffu) | ((((uint32_t)o[4 * q + 1] ^ f) & 0xffu) << 8) |
             ((((uint32_t)o[4 * q + 2] ^ f) & 0xffu) << 16) | (((uint32_t)o[4 * q + 3] ^ f) << 24);
    }
  }
  const v4u v = {w[0], w[1], w[2], w[3]};
  v4u* body = reinterpret_cast<v4u*>(static_cast<uint8_t*>(a.out) + a.body_lo * KB);
  __builtin_nontemporal_store(v, &body[i]);
}

// The int64 outputs of one wave's 256-position step (groups [ib, ib + 64) of
// the aligned body, those below i_hi): lane l holds positions 2l, 2l + 1,
// 128 + 2l and 129 + 2l of the step (fill_chunk's pair layout), so each of
// its two 16-byte stores is one lane's share of a contiguous 1 KB wave store
// and every line is written whole by one instruction.
__device__ __forceinline__ void store_pairs64(const FillArgs& a, uint64_t ib, uint32_t lane, uint64_t i_hi,
                                              v4i o) {
  const uint64_t m = (uint64_t)a.min64;
  v4i* body = reinterpret_cast<v4i*>(static_cast<int64_t*>(a.out) + a.body_lo) + 2 * ib;
  if (ib + (lane >> 1) < i_hi) {
    const uint64_t k0 = m + (uint32_t)o.x, k1 = m + (uint32_t)o.y;
    const v4i w = {(int)(uint32_t)k0, (int)(uint32_t)(k0 >> 32), (int)(uint32_t)k1, (int)(uint32_t)(k1 >> 32)};
    __builtin_nontemporal_store(w, &body[lane]);
  }
  if (ib + 32 + (lane >> 1) < i_hi) {
    const uint64_t k2 = m + (uint32_t)o.z, k3 = m + (uint32_t)o.w;
    const v4i w = {(int)(uint32_t)k2, (int)(uint32_t)(k2 >> 32), (int)(uint32_t)k3, (int)(uint32_t)(k3 >> 32)};
    __builtin_nontemporal_store(w, &body[64 + lane]);
  }
}

template <int KB>
__device__ __forceinline__ void store_one(const FillArgs& a, uint64_t p, int32_t v) {
  if constexpr (KB == 8) static_cast<int64_t*>(a.out)[p] = (int64_t)((uint64_t)a.min64 + (uint32_t)v);
  else if constexpr (KB == 4) static_cast<int32_t*>(a.out)[p] = v;
  else if constexpr (KB == 2) static_cast<uint16_t*>(a.out)[p] = (uint16_t)((uint32_t)v ^ a.flip);
  else static_cast<uint8_t*>(a.out)[p] = (uint8_t)((uint32_t)v ^ a.flip);
}

// Inclusive cumulative count of value v over the whole range: O[t] + C_t[x].
__device__ __forceinline__ uint32_t cum_incl(const FillArgs& a, uint32_t v) {
  return a.O[v / a.T] + a.cdf[v];
}

// Value (offset from minVal) at output position p, searched in global memory
// over [v0, v1]; used when a chunk's window does not fit in LDS.
__device__ __forceinline__ uint32_t value_at_global(const FillArgs& a, uint32_t v0, uint32_t v1,
                                                    uint32_t p) {
  uint32_t lo = v0, hi = v1;   // answer in [v0, v1]
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (cum_incl(a, mid) <= p) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Start position of output chunk k: s(0) = 0, s(k) = out_head + k * chunk.
__device__ __forceinline__ uint64_t chunk_start(const FillArgs& a, uint32_t k) {
  return k == 0 ? 0 : (uint64_t)a.out_head + (uint64_t)k * a.chunk;
}

// Writes the positions [p0, p1) of one chunk whose values lie in [v0, v0 + nwin)
// and whose inclusive cumulative counts are in win[0, nwin).  SPARSE selects
// the form for windows of many values per step (see below).
// The dense form for 16- and 8-bit keys: every lane writes 16 / KB positions
// (one 16-byte vector) per step, so a wave's step covers 512 or 1024
// positions; the walk is fill_chunk's dense walk (below) with that step.
template <int KB>
__device__ __forceinline__ void fill_chunk_wide(const FillArgs& a, const uint32_t* win, uint32_t nwin,
                                                uint32_t v0, uint64_t p0, uint64_t p1, bool first,
                                                bool final) {
  constexpr uint32_t PG = 16 / KB, STEP = 64 * PG;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint64_t q_lo = p0 > a.body_lo ? p0 : a.body_lo;
  const uint64_t q_hi = p1 < a.body_hi ? p1 : a.body_hi;
  // chunk starts and body_hi are multiples of PG positions from body_lo
  const uint64_t i_lo = (q_lo - a.body_lo) / PG, i_hi = q_hi > q_lo ? (q_hi - a.body_lo) / PG : i_lo;
  const int32_t base = (int32_t)(a.min_u + v0);
  const uint32_t last = nwin - 1;
  uint32_t xw = 0;
  uint32_t end = win[0];
  for (uint64_t ib = i_lo + (uint64_t)wave * 64; ib < i_hi; ib += kFillBlock) {
    const uint32_t pw = (uint32_t)(a.body_lo + PG * ib);
    while (xw < last && end <= pw) end = win[++xw];
    const uint64_t i = ib + lane;
    int32_t o[PG];
    // end > pw here unless xw == last: the step's end is tested relative to pw
    if (xw == last || past_step(end, pw, STEP)) {
#pragma unroll
      for (uint32_t j = 0; j < PG; ++j) o[j] = base + (int32_t)xw;
    } else {
      const uint32_t p = pw + PG * lane;
      uint32_t c[PG];
#pragma unroll
      for (uint32_t j = 0; j < PG; ++j) c[j] = 0;
      uint32_t xb = xw, e = end;
      while (xb < last && !past_step(e, pw, STEP)) {   // boundary after value xb at position e
#pragma unroll
        for (uint32_t j = 0; j < PG; ++j) c[j] += e <= p + j;
        e = win[++xb];
      }
#pragma unroll
      for (uint32_t j = 0; j < PG; ++j) o[j] = base + (int32_t)(xw + c[j]);
    }
    if (i < i_hi) store_vec16<KB>(a, i, o);
  }
  if (first)
    for (uint64_t p = tid; p < a.body_lo; p += kFillBlock)
      store_one<KB>(a, p, base + (int32_t)min(count_le(win, nwin, (uint32_t)p), last));
  if (final)
    for (uint64_t p = a.body_hi + tid; p < a.n; p += kFillBlock)
      store_one<KB>(a, p, base + (int32_t)min(count_le(win, nwin, (uint32_t)p), last));
}

template <bool SPARSE, int KB>
__device__ __forceinline__ void fill_chunk(const FillArgs& a, const uint32_t* win, uint32_t nwin,
                                           uint32_t v0, uint64_t p0, uint64_t p1, bool first,
                                           bool final, uint32_t* stage) {
  if constexpr (!SPARSE && KB < 4) {
    fill_chunk_wide<KB>(a, win, nwin, v0, p0, p1, first, final);
    return;
  }
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint64_t q_lo = p0 > a.body_lo ? p0 : a.body_lo;
  const uint64_t q_hi = p1 < a.body_hi ? p1 : a.body_hi;
  const uint64_t i_lo = (q_lo - a.body_lo) >> 2, i_hi = q_hi > q_lo ? (q_hi - a.body_lo) >> 2 : i_lo;
  const int32_t base = (int32_t)(a.min_u + v0);
  const uint32_t last = nwin - 1;
  // Each wave writes 64 consecutive vectors (256 positions) per step.  The
  // wave carries the index xw of the value at its current position and that
  // value's inclusive cumulative count `end` in registers (positions only
  // grow), so a step whose 256 positions hold one value touches no memory but
  // the store.  Otherwise the value boundaries inside the step are visited in
  // order (one broadcast LDS read each) and every lane counts the boundaries
  // at or below each of its four positions: pa, pa + 1, pb, pb + 1 from the
  // step's start, four consecutive ones (one 16-byte store), or for int64
  // keys two pairs 128 apart (store_pairs64).  In the SPARSE form, where more
  // than kWalk values end before the step or inside it (most of them empty),
  // one look-ahead read shows it: the wave then bisects for its position or
  // scatters the step's values over an LDS stage (scatter_step).
  constexpr uint32_t kWalk = 8;
  const uint32_t pa = KB == 8 ? 2 * lane : 4 * lane, pb = KB == 8 ? 128 + 2 * lane : 4 * lane + 2;
  uint32_t xw = 0;
  uint32_t end = win[0];
  for (uint64_t ib = i_lo + (uint64_t)wave * 64; ib < i_hi; ib += kFillBlock) {
    const uint32_t pw = (uint32_t)(a.body_lo + 4 * ib);
    if (!SPARSE) {
      while (xw < last && end <= pw) end = win[++xw];
    } else if (xw < last && end <= pw) {
      // the look-ahead and the next end are read together
      const uint32_t far = win[min(xw + kWalk, last)], e1 = win[xw + 1];
      if (far <= pw) {
        xw = upper_in(win, xw, last, pw);
        end = win[xw];
      } else {
        ++xw;
        end = e1;
        while (end <= pw) end = win[++xw];
      }
    }
    const uint64_t i = ib + lane;
    v4i o;
    // end > pw here unless xw == last: the step's end is tested relative to pw
    if (xw == last || past_step(end, pw, 256u)) {
      o = (v4i)(base + (int32_t)xw);
    } else if constexpr (!SPARSE) {
      const uint32_t p = pw + pa, q = pw + pb;
      uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
      uint32_t xb = xw, e = end;
      while (xb < last && !past_step(e, pw, 256u)) {   // boundary after value xb at position e
        c0 += e <= p;
        c1 += e <= p + 1;
        c2 += e <= q;
        c3 += e <= q + 1;
        e = win[++xb];
      }
      o.x = base + (int32_t)(xw + c0);
      o.y = base + (int32_t)(xw + c1);
      o.z = base + (int32_t)(xw + c2);
      o.w = base + (int32_t)(xw + c3);
    } else {
      const uint32_t p = pw + pa, q = pw + pb;
      const uint32_t far = win[min(xw + kWalk, last)], e1 = win[xw + 1];
      if (!past_step(far, pw, 256u)) {
        uint32_t* st = stage + (tid >> 6) * 256u;
        scatter_step([&](uint32_t x) { return win[x]; }, xw, last, pw, st);
        if constexpr (KB == 8) {
          typedef int v2i_t __attribute__((ext_vector_type(2)));
          const v2i_t sa = *reinterpret_cast<const v2i_t*>(st + pa), sb = *reinterpret_cast<const v2i_t*>(st + pb);
          o = (v4i)base + (v4i){sa.x, sa.y, sb.x, sb.y};
        } else {
          const v4i sv = *reinterpret_cast<const v4i*>(st + 4 * lane);
          o = (v4i)base + sv;
        }
      } else {
        // boundary after value xw at position end, then after xw + 1 at e1, ...
        uint32_t c0 = end <= p, c1 = end <= p + 1, c2 = end <= q, c3 = end <= q + 1;
        uint32_t xb = xw + 1, e = e1;
        while (xb < last && !past_step(e, pw, 256u)) {
          c0 += e <= p;
          c1 += e <= p + 1;
          c2 += e <= q;
          c3 += e <= q + 1;
          e = win[++xb];
        }
        o.x = base + (int32_t)(xw + c0);
        o.y = base + (int32_t)(xw + c1);
        o.z = base + (int32_t)(xw + c2);
        o.w = base + (int32_t)(xw + c3);
      }
    }
    if constexpr (KB == 8) store_pairs64(a, ib, lane, i_hi, o);
    else if (i < i_hi) store_group<KB>(a, i, o);
  }
  // scalar head (positions before the aligned body) and tail
  if (first)
    for (uint64_t p = tid; p < a.body_lo; p += kFillBlock)
      store_one<KB>(a, p, base + (int32_t)min(count_le(win, nwin, (uint32_t)p), last));
  if (final)
    for (uint64_t p = a.body_hi + tid; p < a.n; p += kFillBlock)
      store_one<KB>(a, p, base + (int32_t)min(count_le(win, nwin, (uint32_t)p), last));
}

// Chunk of positions whose window does not fit in LDS (very sparse values):
// every position searches the cumulative counts in global memory.
template <int KB>
__device__ void fill_chunk_global(const FillArgs& a, uint32_t v0, uint32_t v1, uint64_t p0,
                                  uint64_t p1) {
  for (uint64_t p = p0 + threadIdx.x; p < p1; p += kFillBlock)
    store_one<KB>(a, p, (int32_t)(a.min_u + value_at_global(a, v0, v1, (uint32_t)p)));
}

// Splitters of chunk k, clamped: they are always in [0, R) for keys inside
// the declared range; the clamps only keep every access in bounds when that
// precondition is broken.
__device__ __forceinline__ void chunk_values(const FillArgs& a, uint32_t k, uint32_t* v0,
                                             uint32_t* nwin) {
  const uint32_t lo = min(a.split[k], a.R - 1);
  const uint32_t hi = min(max(a.split[k + 1], lo), a.R - 1);
  *v0 = lo;
  *nwin = hi - lo + 1;
}

// Output stage.  Workgroups take chunks k = blockIdx.x + j * gridDim.x.  At
// the start of chunk k the workgroup loads the head of chunk k + G's window
// and the splitters of chunk k + 2G, so a chunk's window is complete in LDS
// when its turn comes; the four resident workgroups per compute unit cover
// each other's load latency (more workgroups per unit were measured not to
// write faster).
// MODE 0: every chunk in the dense form; 1: every chunk in the sparse form;
// 2: per chunk, the sparse form where the window holds more than one value
// per 64 positions (a sort whose keys leave stretches of the range nearly
// empty, such as the tails of a narrow normal distribution).
template <int MODE, int KB>
__device__ __forceinline__ void fill_loop(const FillArgs& a, uint32_t (*win)[kFillWindow],
                                          uint32_t* stage) {
  const uint32_t tid = threadIdx.x, G = gridDim.x;
  uint32_t k = blockIdx.x;
  uint32_t v0, nwin;
  chunk_values(a, k, &v0, &nwin);
  for (uint32_t j = tid; j < min(nwin, kFillWindow); j += kFillBlock) win[0][j] = cum_incl(a, v0 + j);
  // splitters of the next chunk
  uint32_t nv0 = 0, nnwin = 0;
  if (k + G < a.nchunks) chunk_values(a, k + G, &nv0, &nnwin);
  __syncthreads();
  uint32_t buf = 0;
  for (;;) {
    const uint32_t kn = k + G;
    const bool more = kn < a.nchunks;
    // prefetch: window head of chunk k + G (one entry per thread), splitters of k + 2G
    uint32_t pre = 0;
    if (more && tid < nnwin && nnwin <= kFillWindow) pre = cum_incl(a, nv0 + tid);
    uint32_t v0_2 = 0, nwin_2 = 0;
    if (kn + G < a.nchunks) chunk_values(a, kn + G, &v0_2, &nwin_2);

    const uint64_t p0 = chunk_start(a, k);
    const uint64_t p1 = k + 1 < a.nchunks ? chunk_start(a, k + 1) : a.n;
    if (nwin > kFillWindow)
      fill_chunk_global<KB>(a, v0, v0 + nwin - 1, p0, p1);
    else if (MODE == 1 || (MODE == 2 && (uint64_t)nwin * a.sparse_k > p1 - p0))
      fill_chunk<true, KB>(a, win[buf], nwin, v0, p0, p1, k == 0, k + 1 == a.nchunks, stage);
    else
      fill_chunk<false, KB>(a, win[buf], nwin, v0, p0, p1, k == 0, k + 1 == a.nchunks, stage);
    if (!more) break;

    // hand over to chunk k + G
    if (nnwin <= kFillWindow) {
      if (tid < nnwin) win[buf ^ 1][tid] = pre;
      for (uint32_t j = kFillBlock + tid; j < nnwin; j += kFillBlock) win[buf ^ 1][j] = cum_incl(a, nv0 + j);
    }
    __syncthreads();   // next window complete; everyone is done with the current one
    buf ^= 1;
    k = kn;
    v0 = nv0;
    nwin = nnwin;
    nv0 = v0_2;
    nnwin = nwin_2;
  }
}

// SPARSE: the sort's keys average under 64 per value, so every chunk takes the
// sparse form.  Otherwise the dense form, unless the local-CDF stage flagged a
// sparse chunk, in which case each chunk takes the form its window calls for.
template <bool SPARSE, int KB = 4>
__global__ __launch_bounds__(kFillBlock) void k_fill(FillArgs a) {
  __shared__ uint32_t win[2][kFillWindow];
  __shared__ __align__(16) uint32_t stage[kFillBlock / 64 * 256];   // per wave (sparse steps)
  if (blockIdx.x >= a.nchunks) return;
  if (SPARSE) fill_loop<1, KB>(a, win, stage);
  else if (a.flags[0] == 0u) fill_loop<0, KB>(a, win, stage);
  else fill_loop<2, KB>(a, win, stage);
}

// Output stage of the single-tile fast path (R <= kFastMaxRange, one LDS pass
// of 32-bit counters).  The histogram left the counts in `rows` rows of
// `stride` words of region `cur` of the fast-path area; every workgroup sums
// the rows and scans the sums into its own LDS (the cumulative counts of the
// whole range, so any chunk's window is a slice of them) and finds the values
// at its chunks' boundaries itself, so no reduction or local-CDF launch is
// needed.
constexpr uint32_t kFastSplit = kFillBlock;   // chunk boundaries found per batch

// Numbers of entries <= q0 and <= q1 in the nondecreasing C[0, len): two
// branch-free binary liftings advanced together (independent LDS reads).
__device__ __forceinline__ void count_le2(const uint32_t* C, uint32_t len, uint32_t q0, uint32_t q1,
                                          uint32_t* r0, uint32_t* r1) {
  uint32_t a = 0, b = 0;
  for (uint32_t step = len ? 1u << (31 - __builtin_clz(len)) : 0u; step; step >>= 1) {
    const uint32_t xa = a + step <= len ? C[a + step - 1] : ~0u;
    const uint32_t xb = b + step <= len ? C[b + step - 1] : ~0u;
    if (xa <= q0) a += step;
    if (xb <= q1) b += step;
  }
  *r0 = a;
  *r1 = b;
}

template <bool SPARSE, int KB = 4>
__global__ __launch_bounds__(kFillBlock) void k_fill_small(FillArgs a, uint32_t* area, uint32_t rows,
                                                           uint32_t stride) {
  __shared__ __align__(16) uint32_t C[kFastMaxRange];
  __shared__ __align__(16) uint32_t rowbuf[kFastRegionWords];
  __shared__ uint32_t v_lo[kFastSplit], v_hi[kFastSplit];
  __shared__ uint32_t wsum[kFillBlock / 64];
  __shared__ __align__(16) uint32_t stage[kFillBlock / 64 * 256];
  const uint32_t tid = threadIdx.x, R = a.R;
  const uint32_t cur = area[kFastCur] & 1u;
  if (blockIdx.x == 0 && tid == 0) area[kFastPar] = cur ^ 1u;   // the next sort's region
  const uint32_t* acc = area + cur * kFastRegionWords;
  const uint32_t words = rows * stride;
  // all rows at once: every (clamped) load is issued before the first use
  constexpr uint32_t kLoads = kFastRegionWords / kFillBlock;
  uint32_t ld[kLoads];
#pragma unroll
  for (uint32_t j = 0; j < kLoads; ++j) ld[j] = acc[min(tid + j * kFillBlock, words - 1)];
#pragma unroll
  for (uint32_t j = 0; j < kLoads; ++j)
    if (tid + j * kFillBlock < words) rowbuf[tid + j * kFillBlock] = ld[j];
  __syncthreads();
  // Column sums and their inclusive scan in one pass: thread t owns the eight
  // columns [8t, 8t + 8) (stride, a multiple of 128, is at most 2048; columns
  // in [R, stride) are zero).
  static_assert(8 * kFillBlock == kFastMaxRange, "eight columns per thread");
  const uint32_t c0 = 8 * tid;
  uint32_t x[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (c0 < stride) {
#pragma unroll 4
    for (uint32_t r = 0; r < rows; ++r) {
      const v4u lo = *reinterpret_cast<const v4u*>(rowbuf + r * stride + c0);
      const v4u hi = *reinterpret_cast<const v4u*>(rowbuf + r * stride + c0 + 4);
      x[0] += lo.x; x[1] += lo.y; x[2] += lo.z; x[3] += lo.w;
      x[4] += hi.x; x[5] += hi.y; x[6] += hi.z; x[7] += hi.w;
    }
#pragma unroll
    for (int q = 1; q < 8; ++q) x[q] += x[q - 1];
  }
  uint32_t total;
  const uint32_t before = block_inclusive_scan(x[7], wsum, &total) - x[7];
  if (c0 < stride) {
    const v4u lo = {x[0], x[1], x[2], x[3]}, hi = {x[4], x[5], x[6], x[7]};
    *reinterpret_cast<v4u*>(C + c0) = lo + before;
    *reinterpret_cast<v4u*>(C + c0 + 4) = hi + before;
  }
  __syncthreads();
  const uint32_t last = R - 1, G = gridDim.x;
  for (uint32_t k0 = blockIdx.x; k0 < a.nchunks; k0 += kFastSplit * G) {
    // values at the first and last position of up to kFastSplit of this
    // workgroup's chunks, one bisection each
    const uint32_t kt = k0 + tid * G;
    if (kt < a.nchunks) {
      const uint64_t p0 = chunk_start(a, kt);
      const uint64_t p1 = kt + 1 < a.nchunks ? chunk_start(a, kt + 1) : a.n;
      uint32_t lo, hi;
      count_le2(C, R, (uint32_t)p0, (uint32_t)(p1 - 1), &lo, &hi);
      v_lo[tid] = min(lo, last);
      v_hi[tid] = min(hi, last);
    }
    __syncthreads();
    for (uint32_t j = 0; j < kFastSplit && k0 + j * G < a.nchunks; ++j) {
      const uint32_t k = k0 + j * G;
      const uint64_t p0 = chunk_start(a, k);
      const uint64_t p1 = k + 1 < a.nchunks ? chunk_start(a, k + 1) : a.n;
      // uniform: the walk of fill_chunk is then steered by scalar registers
      const uint32_t v0 = __builtin_amdgcn_readfirstlane(v_lo[j]);
      const uint32_t nwin = __builtin_amdgcn_readfirstlane(v_hi[j]) - v0 + 1;
      if (SPARSE || (uint64_t)nwin * a.sparse_k > p1 - p0)   // as the per-chunk mode of fill_loop
        fill_chunk<true, KB>(a, C + v0, nwin, v0, p0, p1, k == 0, k + 1 == a.nchunks, stage);
      else
        fill_chunk<false, KB>(a, C + v0, nwin, v0, p0, p1, k == 0, k + 1 == a.nchunks, stage);
      // Every wave waits for its stores, then the workgroup meets, once per
      // chunk.  A loop of bare stores lets the oldest workgroups on a compute
      // unit take the store path (the youngest ended ~30 us after the oldest
      // at n = 10^8); this keeps the four in step, as the window loads of
      // k_fill do.
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
    __syncthreads();
  }
}

// Plain 16-byte vector copy (grid-stride), the attainable-bandwidth reference
// for the measurement of the sort kernels and the calibration of HBM counters.
__global__ __launch_bounds__(256) void k_stream_copy(const v4i* __restrict__ src,
                                                     v4i* __restrict__ dst, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (size_t)gridDim.x * 256)
    dst[i] = __builtin_nontemporal_load(&src[i]);
}

__global__ void k_clear(uint32_t* p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

template <int ITEMS, int BITS, int BLOCK, int KB = 4, bool DEDUPE = false, bool SPREAD = false>
hipError_t launch_hist_t(const Plan& p, const HistArgs& a, hipStream_t s) {
  // the counters (their copies with SPREAD; the narrow forms' wrap table) fit
  // the static LDS array
  const size_t words = SPREAD ? (size_t)p.row_words << p.sub_log : (size_t)p.row_words;
  const size_t lds = (words + (BITS < 32 ? 1 + 2 * (size_t)p.wrap_slots : 0)) * 4;
  if (lds > kLdsBytes / (1024 / BLOCK)) return hipErrorInvalidValue;
  if (SPREAD && (p.part || p.sub_log > 4)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_hist<ITEMS, BITS, BLOCK, KB, DEDUPE, SPREAD>), dim3(p.passes * p.G), dim3(BLOCK), 0, s, a);
  return hipGetLastError();
}

template <int BITS, int BLOCK>
hipError_t launch_hist_items(const Plan& p, const HistArgs& a, hipStream_t s) {
  // 8- and 16-bit keys: one 16-byte vector (16 or 8 keys) per thread per step
  // (4-bit counters serve int32 keys only)
  // (int64 keys: two 16-byte vectors, four keys, per thread per step)
  if constexpr (BITS == 32) {
    if (p.sub_log > 0 && !p.dedupe) {   // LDS copies of the counters
      if (p.kb == 2) return launch_hist_t<4, 32, BLOCK, 2, false, true>(p, a, s);
      if (p.kb == 1) return launch_hist_t<4, 32, BLOCK, 1, false, true>(p, a, s);
      if (p.kb == 8) return launch_hist_t<8, 32, BLOCK, 8, false, true>(p, a, s);
      switch (p.items) {
        case 4: return launch_hist_t<4, 32, BLOCK, 4, false, true>(p, a, s);
        case 8: return launch_hist_t<8, 32, BLOCK, 4, false, true>(p, a, s);
        default: return launch_hist_t<16, 32, BLOCK, 4, false, true>(p, a, s);
      }
    }
  }
  if constexpr (BITS == 4) {
    if (p.kb != 4) return hipErrorInvalidValue;
  } else {
    if (p.kb == 2) return launch_hist_t<4, BITS, BLOCK, 2>(p, a, s);
    if (p.kb == 1) return launch_hist_t<4, BITS, BLOCK, 1>(p, a, s);
    if (p.kb == 8) return launch_hist_t<8, BITS, BLOCK, 8>(p, a, s);
  }
  if (p.dedupe) {
    switch (p.items) {
      case 4: return launch_hist_t<4, BITS, BLOCK, 4, true>(p, a, s);
      case 8: return launch_hist_t<8, BITS, BLOCK, 4, true>(p, a, s);
      default: return launch_hist_t<16, BITS, BLOCK, 4, true>(p, a, s);
    }
  }
  switch (p.items) {
    case 4: return launch_hist_t<4, BITS, BLOCK>(p, a, s);
    case 8: return launch_hist_t<8, BITS, BLOCK>(p, a, s);
    default: return launch_hist_t<16, BITS, BLOCK>(p, a, s);
  }
}

template <int BITS>
hipError_t launch_hist_block(const Plan& p, const HistArgs& a, hipStream_t s) {
  switch (p.hist_block) {
    case 1024: return launch_hist_items<BITS, 1024>(p, a, s);
    case 512: return launch_hist_items<BITS, 512>(p, a, s);
    default: return launch_hist_items<BITS, 256>(p, a, s);
  }
}

}  // namespace

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int cus, hipStream_t s) {
  const size_t n4 = bytes / 16;
  if (n4 == 0) return hipSuccess;
  size_t blocks = (n4 + 255) / 256;
  const size_t cap = (size_t)cus * 4;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s,
                     reinterpret_cast<const v4i*>(src), reinterpret_cast<v4i*>(dst), n4);
  return hipGetLastError();
}

hipError_t launch_clear(uint32_t* ptr, size_t words, hipStream_t s) {
  if (words == 0) return hipSuccess;
  size_t blocks = (words + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_clear, dim3((unsigned)blocks), dim3(256), 0, s, ptr, words);
  return hipGetLastError();
}

hipError_t launch_hist(const Plan& p, const int32_t* keys, uint8_t* ws, uint32_t* carry,
                       hipStream_t s) {
  HistArgs a;
  a.keys = keys;
  a.in_n4 = (uint32_t)p.in_n4;     // n < 2^32: at most 2^30 vectors
  a.in_per = (uint32_t)p.in_per;
  a.in_head = p.in_head;
  if (p.kb != 4 && p.kb != 2 && p.kb != 1 && p.kb != 8) return hipErrorInvalidValue;
  a.in_tail = (uint32_t)(p.n - p.in_head - (16 / p.kb) * p.in_n4);
  a.min64 = p.min64;
  a.flip = p.flip;
  a.min_u = p.min_u;
  a.W = p.W;
  a.passes = p.passes;
  a.G = p.G;
  a.row_words = p.row_words;
  a.wrap_slots = p.wrap_slots;
  a.sub_log = p.sub_log;
  a.R = p.R;
  a.partial = reinterpret_cast<uint32_t*>(ws + p.off_partial);
  a.carry = carry;
  a.interleave = p.hist_interleave;
  a.merge = p.fast ? p.fast_rows : 0u;
  a.merge_stride = p.fast_stride;
  a.pbound = nullptr;
  if (p.part) {
    if (p.fast || p.off_pkeys % 16 != 0 || p.kb != 4) return hipErrorInvalidValue;
    a.keys = reinterpret_cast<const int32_t*>(ws + p.off_pkeys);
    a.pbound = reinterpret_cast<const uint32_t*>(ws + p.off_pbound);
  }
  switch (p.bits) {
    case 4: return launch_hist_block<4>(p, a, s);
    case 8: return launch_hist_block<8>(p, a, s);
    case 16: return launch_hist_block<16>(p, a, s);
    default: return launch_hist_block<32>(p, a, s);
  }
}

hipError_t launch_reduce(const Plan& p, uint8_t* ws, uint32_t* carry, int32_t* pm_out, hipStream_t s) {
  ReduceArgs a;
  a.nred = p.nred;
  a.pm_out = pm_out;
  a.pm_n = (uint32_t)p.n;
  a.pm_head = (uint32_t)(p.out_head < p.n ? p.out_head : p.n);
  a.pm_nck = p.pm_chunks;
  a.pm_fill = (int32_t)p.min_u;
  a.pm_M = reinterpret_cast<uint32_t*>(ws + p.off_pm);
  if (pm_out != nullptr && (!p.pmax || p.pm_init_grid == 0 || p.n > 0xffffffffull))
    return hipErrorInvalidValue;
  a.partial = reinterpret_cast<const uint32_t*>(ws + p.off_partial);
  a.carry = carry;
  a.hist = reinterpret_cast<uint32_t*>(ws + p.off_hist);
  a.rsum = reinterpret_cast<uint32_t*>(ws + p.off_rsum);
  a.flags = reinterpret_cast<uint32_t*>(ws + p.off_flags);
  a.R = p.R;
  a.W = p.W;
  a.G = p.G;
  a.row_words = p.row_words;
  a.carry_words = (uint32_t)p.carry_words;
  a.bits = p.bits;
  a.prow = p.part ? reinterpret_cast<const uint32_t*>(ws + p.off_prow) : nullptr;
  // 128-bin blocks never straddle passes (W % 128 == 0), and a block's words
  // are whole 16-byte quads of 16-byte aligned rows
  if (p.W % kReduceBins != 0 || p.row_words % 4 != 0) return hipErrorInvalidValue;
  const uint32_t threads = reduce_groups(p.bits) * (kReduceBins / (32 / p.bits) / 4);
  const uint32_t grid = p.nred + (pm_out != nullptr ? p.pm_init_grid : 0u);
  const size_t lds = (size_t)reduce_groups(p.bits) * (kReduceBins + 1) * 4;
  hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(threads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_tilescan(const Plan& p, uint8_t* ws, int32_t* pm_out, hipStream_t s) {
  ScanArgs a;
  a.pm_out = pm_out;
  a.pm_head = (uint32_t)(p.out_head < p.n ? p.out_head : p.n);
  a.pm_chunk = p.pm_chunk;
  a.pm_min = (int32_t)p.min_u;
  a.pm_M = reinterpret_cast<uint32_t*>(ws + p.off_pm);
  if (pm_out != nullptr && (!p.pmax || p.pm_chunk == 0)) return hipErrorInvalidValue;
  a.hist = reinterpret_cast<const uint32_t*>(ws + p.off_hist);
  a.cdf = reinterpret_cast<uint32_t*>(ws + p.off_cdf);
  a.S = p.scan_parts;
  a.m = p.m;
  a.grid = p.scan_grid;
  a.flags = reinterpret_cast<uint32_t*>(ws + p.off_flags);
  a.rsum = reinterpret_cast<const uint32_t*>(ws + p.off_rsum);
  a.O = reinterpret_cast<uint32_t*>(ws + p.off_O);
  a.split = reinterpret_cast<uint32_t*>(ws + p.off_split);
  a.n = p.n;
  a.R = p.R;
  a.T = p.T;
  a.out_head = p.out_head;
  a.chunk = p.chunk;
  a.nchunks = p.nchunks;
  a.sparse_k = p.fill_sparse_keys;
  // The per-tile path sums the block totals before each tile in every
  // workgroup (m x nred / 2 loads in all); above 2^28 loads one workgroup
  // forms all offsets first.
  a.pre_O = p.m > 1 && p.scan_grid <= p.m && (uint64_t)p.m * p.nred > (1ull << 28);
  if (a.pre_O) {
    // tiles of T = a multiple of 128 bins
    if (p.T % kReduceBins != 0 || p.scan_grid != p.m * p.scan_parts) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tile_offsets, dim3(1), dim3(kScanBlock), 0, s,
                       static_cast<const uint32_t*>(a.rsum), p.nred, p.T / kReduceBins, p.m, a.O);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
  }
  const size_t lds = ((size_t)p.T + p.T / 32 + 2 + 4 * kScanBlock) * 4;
  // the attribute is raised once, to the size of the widest tile (T = 32768)
  constexpr size_t kMaxLds = ((size_t)32768 + 32768 / 32 + 2 + 4 * kScanBlock) * 4;
  if (lds > kMaxLds) return hipErrorInvalidValue;
  hipError_t e = ensure_dynamic_lds((const void*)k_tilescan, (int)kMaxLds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tilescan, dim3(p.scan_grid), dim3(kScanBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_fill(const Plan& p, int32_t* out, const uint8_t* ws, hipStream_t s) {
  FillArgs a;
  a.out = out;
  a.cdf = reinterpret_cast<const uint32_t*>(ws + p.off_cdf);
  a.O = reinterpret_cast<const uint32_t*>(ws + p.off_O);
  a.split = reinterpret_cast<const uint32_t*>(ws + p.off_split);
  a.n = p.n;
  a.min_u = p.min_u;
  a.R = p.R;
  a.T = p.T;
  a.out_head = p.out_head;
  a.chunk = p.chunk;
  a.nchunks = p.nchunks;
  a.sparse_k = p.fill_sparse_keys;
  a.body_lo = p.out_head < p.n ? p.out_head : p.n;
  // whole groups of 4 int32 or int64 keys, or of 16 / kb narrow keys (one
  // 16-byte vector)
  const uint32_t group = p.kb >= 4 ? 4u : 16u / p.kb;
  a.body_hi = a.body_lo + group * ((p.n - a.body_lo) / group);
  a.min64 = p.min64;
  a.flags = reinterpret_cast<const uint32_t*>(ws + p.off_flags);
  a.flip = p.flip;
  // The sparse form (look-ahead and bisection in the window) when the values
  // average fewer than fill_sparse_keys output positions each; the plain walk
  // otherwise.
  const bool sparse = p.n < (uint64_t)p.fill_sparse_keys * p.R;
  const dim3 grid(p.fill_grid), block(kFillBlock);
  switch (p.kb) {
    case 4:
      if (sparse) hipLaunchKernelGGL((k_fill<true, 4>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_fill<false, 4>), grid, block, 0, s, a);
      break;
    case 2:
      if (sparse) hipLaunchKernelGGL((k_fill<true, 2>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_fill<false, 2>), grid, block, 0, s, a);
      break;
    case 1:
      if (sparse) hipLaunchKernelGGL((k_fill<true, 1>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_fill<false, 1>), grid, block, 0, s, a);
      break;
    case 8:
      if (sparse) hipLaunchKernelGGL((k_fill<true, 8>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_fill<false, 8>), grid, block, 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_fast(const Plan& p, int32_t* out, uint32_t* area, hipStream_t s) {
  if (p.R > kFastMaxRange || p.m != 1 || p.fast_rows == 0 || p.fast_stride < p.R ||
      (uint64_t)p.fast_rows * p.fast_stride > kFastRegionWords)
    return hipErrorInvalidValue;
  FillArgs a = {};
  a.out = out;
  a.n = p.n;
  a.min_u = p.min_u;
  a.R = p.R;
  a.T = p.T;
  a.out_head = p.out_head;
  a.chunk = p.chunk;
  a.nchunks = p.nchunks;
  a.sparse_k = p.fill_sparse_keys;
  a.body_lo = p.out_head < p.n ? p.out_head : p.n;
  // whole groups of 4 int32 or int64 keys, or of 16 / kb narrow keys (one
  // 16-byte vector)
  const uint32_t group = p.kb >= 4 ? 4u : 16u / p.kb;
  a.body_hi = a.body_lo + group * ((p.n - a.body_lo) / group);
  a.min64 = p.min64;
  a.flip = p.flip;
  const bool sparse = p.n < (uint64_t)p.fill_sparse_keys * p.R;
  const dim3 grid(p.fill_grid), block(kFillBlock);
  const uint32_t rows = p.fast_rows, stride = p.fast_stride;
  switch (p.kb) {
    case 4:
      if (sparse) hipLaunchKernelGGL((k_fill_small<true, 4>), grid, block, 0, s, a, area, rows, stride);
      else hipLaunchKernelGGL((k_fill_small<false, 4>), grid, block, 0, s, a, area, rows, stride);
      break;
    case 2:
      if (sparse) hipLaunchKernelGGL((k_fill_small<true, 2>), grid, block, 0, s, a, area, rows, stride);
      else hipLaunchKernelGGL((k_fill_small<false, 2>), grid, block, 0, s, a, area, rows, stride);
      break;
    case 1:
      if (sparse) hipLaunchKernelGGL((k_fill_small<true, 1>), grid, block, 0, s, a, area, rows, stride);
      else hipLaunchKernelGGL((k_fill_small<false, 1>), grid, block, 0, s, a, area, rows, stride);
      break;
    case 8:
      if (sparse) hipLaunchKernelGGL((k_fill_small<true, 8>), grid, block, 0, s, a, area, rows, stride);
      else hipLaunchKernelGGL((k_fill_small<false, 8>), grid, block, 0, s, a, area, rows, stride);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rtcdf
