// rtcdf_device.h -- device helpers shared by the RT-CDF kernels (wave and
// block scans, searches in cumulative counts, LDS histogram counting).
// Internal; included by the kernel translation units only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtcdf {
namespace dev {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- wave helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive prefix sum across a 64-lane wave with DPP row shifts and row
// broadcasts (rows of 16 lanes, then lane 15 -> next row, lane 31 -> upper half).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
  uint32_t s = wave_inclusive_scan(x);
  return (uint32_t)__builtin_amdgcn_readlane((int)s, 63);
}

// Block-wide inclusive scan of one value per thread (blockDim.x multiple of 64,
// at most 1024).  Returns the inclusive prefix; *total receives the block sum.
// wsum must hold blockDim.x / 64 words of LDS.  Contains two barriers.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t* wsum,
                                                         uint32_t* total) {
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    uint32_t s = lane < nw ? wsum[lane] : 0u;
    s = wave_inclusive_scan(s);
    if (lane < nw) wsum[lane] = s;
  }
  __syncthreads();
  const uint32_t before = wave ? wsum[wave - 1] : 0u;
  *total = wsum[nw - 1];
  __syncthreads();  // wsum may be reused by the caller right away
  return inc + before;
}

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* wsum) {
  uint32_t t;
  (void)block_inclusive_scan(v, wsum, &t);
  return t;
}

// Number of entries of the nondecreasing a[0..len) that are <= q.
__device__ __forceinline__ uint32_t count_le(const uint32_t* a, uint32_t len, uint32_t q) {
  uint32_t lo = 0, hi = len;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= q) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// First index x in [lo, hi] with a[x] > q in the nondecreasing a, or hi if
// there is none.
__device__ __forceinline__ uint32_t upper_in(const uint32_t* a, uint32_t lo, uint32_t hi, uint32_t q) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= q) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Output positions and inclusive cumulative counts are uint32 (n < 2^32), so
// the end of a step of `span` positions starting at p, p + span, wraps when p
// lies within span of 2^32.  Every test against a step's end is therefore made
// relative to its start: for e >= p, e lies at or past the step's end iff
// e - p >= span.  The callers guarantee e >= p (e is the end of a value that
// covers or follows position p).
__host__ __device__ __forceinline__ bool past_step(uint32_t e, uint32_t p, uint32_t span) {
  return e - p >= span;
}

// Writes, for one wave, the value index of each of the 256 positions
// [q, q + 256) into stage[0, 256) (this wave's LDS staging area).  E(x) is
// the inclusive cumulative count of value x, so value x occupies positions
// [E(x - 1), E(x)); x0 is the value at position q and last the last value
// index (E(last) is past every position asked for).  The lanes take 64
// consecutive values at a time and each writes its value over its positions
// inside the step: about two LDS reads per 64 values, however many of them
// are empty, where a search per position would read log2(last) entries in
// sequence.
template <typename GetE>
__device__ __forceinline__ void scatter_step(GetE E, uint32_t x0, uint32_t last, uint32_t q,
                                             uint32_t* stage) {
  const uint32_t lane = lane_id();
  uint32_t xb = x0, start = q;   // start: where the run of value xb begins, clipped to q
  for (;;) {
    // Every run starts and ends at or after q (value x0 covers q), so the
    // bounds are kept relative to q: q + 256 may exceed 2^32 - 1.  Lanes past
    // the last value get start = end = 0xffffffff, an empty run.
    const uint32_t x = xb + lane;
    const uint32_t e = x <= last ? E(x) : 0xffffffffu;
    const uint32_t s = lane == 0 ? start : (x <= last ? E(x - 1) : 0xffffffffu);
    const uint32_t er = e - q, sr = s - q;
    const uint32_t lo = sr, hi = er < 256u ? er : 256u;
    for (uint32_t r = lo; r < hi; ++r) stage[r] = x;
    const uint32_t e63 = (uint32_t)__builtin_amdgcn_readlane((int)e, 63);
    if (xb + 63u >= last || past_step(e63, q, 256u)) break;
    start = e63;
    xb += 64u;
  }
  // all lanes' writes are ordered before the reads that follow (LDS operations
  // of one wave execute in order); the fence only keeps the compiler from
  // moving them
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Local CDFs are kept in LDS with one padding word per 32 entries, so the
// per-thread segments of the blocked scan fall into distinct banks.
__device__ __forceinline__ uint32_t pad32(uint32_t i) { return i + (i >> 5); }

// upper_in for a wave-uniform search: every probe is read into a scalar
// register, so the loop runs on the scalar unit.
__device__ __forceinline__ uint32_t upper_in_uniform(const uint32_t* a, uint32_t lo, uint32_t hi,
                                                     uint32_t q) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((uint32_t)__builtin_amdgcn_readfirstlane((int)a[mid]) <= q) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// upper_in over the padded array C.
__device__ __forceinline__ uint32_t upper_in_pad(const uint32_t* C, uint32_t lo, uint32_t hi, uint32_t q) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (C[pad32(mid)] <= q) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Number of entries of the nondecreasing padded array C[0..len) that are <= q.
__device__ __forceinline__ uint32_t count_le_pad(const uint32_t* C, uint32_t len, uint32_t q) {
  uint32_t lo = 0, hi = len;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (C[pad32(mid)] <= q) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Two 16-bit counters per LDS word (bin x in half x & 1 of word x >> 1).  The
// returned old word shows whether an add of c wrapped a half; the lost 2^16
// (and the +1 a wrap of the low half pushed into the high half) is repaired
// exactly in the global carry array, which the reduction adds back.
__device__ __forceinline__ void fix_u16(uint32_t old, uint32_t x, uint32_t c, uint32_t* carry,
                                        uint32_t pass_lo) {
  if ((x & 1u) == 0) {
    if ((old & 0xffffu) + c > 0xffffu) {
      const uint32_t c2 = ((old >> 16) + 1u) >> 16;  // high half wrapped by the carry
      atomicAdd(&carry[pass_lo + x], 65536u);
      atomicAdd(&carry[pass_lo + x + 1u], 65536u * c2 - 1u);
    }
  } else if ((old >> 16) + c > 0xffffu) {
    atomicAdd(&carry[pass_lo + x], 65536u);
  }
}

__device__ __forceinline__ void add_u16(uint32_t* S, uint32_t x, uint32_t c, uint32_t* carry,
                                        uint32_t pass_lo) {
  const uint32_t old = atomicAdd(&S[x >> 1], c << ((x & 1u) << 4));
  fix_u16(old, x, c, carry, pass_lo);
}

// Wrap table of the narrow forms: S (bin, amount) pairs in LDS that collect
// the repairs of one workgroup, so that a heavily hit bin costs one global
// atomic per workgroup at the end instead of one per wrap.  S is a power of
// two from kWrapSlots up to kWrapSlotsMax, as many as the LDS left over by the
// counters holds; tab[-1] holds S - 1.  Slot bin % S belongs to the first bin
// that claims it; a repair whose slot is held by another bin goes straight to
// the global carry array.
constexpr uint32_t kWrapEmpty = 0xffffffffu;

__device__ __forceinline__ void wrap_add(uint32_t* tab, uint32_t bin, uint32_t d, uint32_t* carry,
                                         uint32_t pass_lo) {
  const uint32_t mask = tab[-1];
  uint32_t* slot = tab + (bin & mask);
  const uint32_t prev = atomicCAS(slot, kWrapEmpty, bin);
  // Workgroup scope for the LDS add, device scope for the global one: the
  // compiler then keeps them apart instead of merging them into one flat
  // atomic, whose counters would stop it from pipelining the input loads.
  if (prev == kWrapEmpty || prev == bin)
    __hip_atomic_fetch_add(slot + mask + 1u, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else
    __hip_atomic_fetch_add(&carry[pass_lo + bin], d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Moves the table's amounts to the global carry array (the workgroup's
// threads stride over the slots, after its last count).
__device__ __forceinline__ void wrap_flush(const uint32_t* tab, uint32_t* carry, uint32_t pass_lo,
                                           uint32_t t) {
  const uint32_t slots = tab[-1] + 1u;
  for (; t < slots; t += blockDim.x) {
    const uint32_t bin = tab[t], d = tab[t + slots];
    if (bin != kWrapEmpty && d != 0u) atomicAdd(&carry[pass_lo + bin], d);
  }
}

// Wave-uniform accumulator of the narrow forms' all-equal fast path: a wave
// whose four keys per lane are one value adds them to this register (an add
// of 256 would wrap a byte counter every time, and a returning LDS atomic per
// vector would stall the wave); it goes to the wrap table when the value
// changes and at the end.
struct HotBin {
  uint32_t bin = kWrapEmpty;
  uint32_t cnt = 0;
};

__device__ __forceinline__ void hot_flush(HotBin& hot, uint32_t* tab, uint32_t* carry, uint32_t pass_lo) {
  if (hot.cnt && lane_id() == (uint32_t)(__ffsll((unsigned long long)__ballot(1)) - 1))
    wrap_add(tab, hot.bin, hot.cnt, carry, pass_lo);
  hot.cnt = 0;
}

// Flush of the hot-bin register in every counter width: into the wrap table
// for the narrow forms, straight into the LDS counter for 32-bit counters
// (which cannot wrap).
template <int BITS, bool PAD>
__device__ __forceinline__ void hot_flush_any(HotBin& hot, uint32_t* S, uint32_t* tab, uint32_t* carry,
                                              uint32_t pass_lo) {
  if constexpr (BITS < 32) {
    hot_flush(hot, tab, carry, pass_lo);
  } else {
    if (hot.cnt && lane_id() == (uint32_t)(__ffsll((unsigned long long)__ballot(1)) - 1))
      atomicAdd(&S[PAD ? pad32(hot.bin) : hot.bin], hot.cnt);
    hot.cnt = 0;
  }
}

// Wave-level aggregation (RTCDF_FLAG_WAVE_DEDUPE): a candidate value with at
// least this many copies among a wave's 4 x 64 keys is counted once.  (Up to
// four candidates per vector were measured slower on every workload: the
// extra ballots cost more than the LDS conflicts they remove.)
constexpr uint32_t kDedupeMin = 8;

// 32 / BITS packed counters per LDS word (8-bit: bin x in byte x & 3 of word
// x >> 2; 4-bit: nibble x & 7 of word x >> 3).  An add of c << (BITS s)
// changes the fields above s through carries; every field whose represented
// change differs from its true change (c for field s, 0 above) is repaired,
// modulo 2^32, through the wrap table.  Rare for spread-out keys.
template <int BITS>
__device__ __forceinline__ void fix_packed(uint32_t old, uint32_t x, uint32_t c, uint32_t* tab,
                                           uint32_t* carry, uint32_t pass_lo) {
  constexpr uint32_t F = 32 / BITS, M = (1u << BITS) - 1u;
  const uint32_t s = x & (F - 1u);
  const uint32_t nw = old + (c << (BITS * s));
  const uint32_t base = x & ~(F - 1u);
  for (uint32_t j = s; j < F; ++j) {
    const int32_t rep = (int32_t)((nw >> (BITS * j)) & M) - (int32_t)((old >> (BITS * j)) & M);
    const int32_t tru = j == s ? (int32_t)c : 0;
    if (rep != tru) wrap_add(tab, base + j, (uint32_t)(tru - rep), carry, pass_lo);
  }
}

// Counts the four keys of one vector per lane with BITS-bit LDS counters (32,
// 16, 8 or 4).  If every active lane of the wave holds four copies of one value
// (all-equal or heavily skewed keys), a single lane adds them with one LDS
// atomic instead of 4 x 64 atomics on the same address (8-bit form: into the
// wave's hot-bin register in the narrow forms).  Otherwise
// every key inside the pass takes one LDS atomic; keys outside it are masked
// off.  In the narrow forms the four returning atomics are issued back to
// back and a counter that just wrapped is repaired after a single wave-wide
// test.  PAD selects the padded 32-bit layout (bin x at x + x / 32).  `tab`
// and `hot` (the wrap table and the hot-bin register) are used by the 4-, 8-
// and 16-bit forms; the 16-bit form may run without a table (tab == nullptr).
// 1 << (s mod 32): the hardware shift reads only the low five bits of the
// amount, so no mask is needed (the compiler emits one when it can prove the
// amount's low bits are zero, as for x << 3).
__device__ __forceinline__ uint32_t shl1(uint32_t s) {
  uint32_t r;
  asm("v_lshlrev_b32_e64 %0, %1, 1" : "=v"(r) : "v"(s));
  return r;
}

// DEDUPE (RTCDF_FLAG_WAVE_DEDUPE; the hot-bin register must then be flushed
// with hot_flush_any after the last count): when the wave's keys are not all
// one value, a candidate value -- the wave's hot bin, else the first lane's
// first key -- is matched against the wave's 4 x 64 keys with four ballots;
// if it has kDedupeMin or more copies they are added to the hot-bin register
// at once and skip their LDS atomics (a frequent value would otherwise put
// many lanes of one atomic on one LDS word, and wrap 8-bit counters).
// SPREAD (32-bit counters, few bins): bin x has 2^sub_log copies at words
// (x << sub_log) + c, and lane l adds into copy l mod 2^sub_log, so lanes
// that hit one bin in the same atomic mostly hit different words; the copies
// are summed when the counters are written out.
template <int BITS, bool PAD = false, bool DEDUPE = false, bool SPREAD = false>
__device__ __forceinline__ void count4(uint32_t* S, v4i k, uint32_t base, uint32_t W,
                                       uint32_t* carry, uint32_t pass_lo, uint32_t* tab, HotBin& hot,
                                       uint32_t sub_log = 0) {
  static_assert(!SPREAD || (BITS == 32 && !PAD && !DEDUPE), "copies of 32-bit unpadded counters only");
  uint32_t x0 = (uint32_t)k.x - base, x1 = (uint32_t)k.y - base;
  uint32_t x2 = (uint32_t)k.z - base, x3 = (uint32_t)k.w - base;
  const uint32_t lead = (uint32_t)__builtin_amdgcn_readfirstlane((int)x0);
  const uint64_t active = __ballot(1);
  // the other three keys are compared only when every first key matches
  bool all_same = __ballot(x0 == lead) == active;
  if (all_same) all_same = (__ballot(x1 == lead) & __ballot(x2 == lead) & __ballot(x3 == lead)) == active;
  if (all_same) {
    if (lead < W) {
      const uint32_t c = 4u * (uint32_t)__popcll(active);
      if constexpr (BITS < 32) {
        if (tab != nullptr) {
          if (lead != hot.bin) {
            hot_flush(hot, tab, carry, pass_lo);
            hot.bin = lead;
          }
          hot.cnt += c;
        } else if (lane_id() == (uint32_t)(__ffsll((unsigned long long)active) - 1)) {
          add_u16(S, lead, c, carry, pass_lo);   // 16-bit form without a wrap table
        }
      } else if (lane_id() == (uint32_t)(__ffsll((unsigned long long)active) - 1)) {
        atomicAdd(&S[PAD ? pad32(lead) : (SPREAD ? lead << sub_log : lead)], c);
      }
    }
    return;
  }
  if constexpr (DEDUPE) {
    uint32_t cand = hot.bin != kWrapEmpty ? hot.bin : lead;
    uint32_t c = (uint32_t)(__popcll(__ballot(x0 == cand)) + __popcll(__ballot(x1 == cand)) +
                            __popcll(__ballot(x2 == cand)) + __popcll(__ballot(x3 == cand)));
    if (c < kDedupeMin && cand != lead) {
      cand = lead;
      c = (uint32_t)(__popcll(__ballot(x0 == cand)) + __popcll(__ballot(x1 == cand)) +
                     __popcll(__ballot(x2 == cand)) + __popcll(__ballot(x3 == cand)));
    }
    if (c >= kDedupeMin) {
      if (cand < W) {
        if (cand != hot.bin) {
          hot_flush_any<BITS, PAD>(hot, S, tab, carry, pass_lo);
          hot.bin = cand;
        }
        hot.cnt += c;
      }
      // the copies are counted (or lie outside this pass): none takes an atomic
      constexpr uint32_t kNone = 0xffffffffu;
      x0 = x0 == cand ? kNone : x0;
      x1 = x1 == cand ? kNone : x1;
      x2 = x2 == cand ? kNone : x2;
      x3 = x3 == cand ? kNone : x3;
    }
  }
  if constexpr (BITS == 16 || BITS == 8 || BITS == 4) {
    // Bin x is the field at bit (x & (32 / BITS - 1)) * BITS of word x >> LOG.
    // That offset is (x << SH) & 31, and the hardware shifts and bit-field
    // extracts read only the low 5 bits of an offset, so the masks fold away.
    constexpr uint32_t LOG = BITS == 16 ? 1 : (BITS == 8 ? 2 : 3), SH = BITS == 16 ? 4 : (BITS == 8 ? 3 : 2);
    constexpr uint32_t FULL = (1u << BITS) - 1u;
    const uint32_t s0 = x0 << SH, s1 = x1 << SH, s2 = x2 << SH, s3 = x3 << SH;
    uint32_t o0 = 0, o1 = 0, o2 = 0, o3 = 0;
    if (x0 < W) o0 = atomicAdd(&S[x0 >> LOG], shl1(s0));
    if (x1 < W) o1 = atomicAdd(&S[x1 >> LOG], shl1(s1));
    if (x2 < W) o2 = atomicAdd(&S[x2 >> LOG], shl1(s2));
    if (x3 < W) o3 = atomicAdd(&S[x3 >> LOG], shl1(s3));
    // One test for the four: a counter wrapped iff its old field was FULL.
    // Keys outside the pass kept o = 0, whose fields are 0.
    const uint32_t f0 = __builtin_amdgcn_ubfe(o0, s0, BITS), f1 = __builtin_amdgcn_ubfe(o1, s1, BITS);
    const uint32_t f2 = __builtin_amdgcn_ubfe(o2, s2, BITS), f3 = __builtin_amdgcn_ubfe(o3, s3, BITS);
    if (__ballot(max(max(f0, f1), max(f2, f3)) == FULL)) {
      const bool w0 = f0 == FULL, w1 = f1 == FULL, w2 = f2 == FULL, w3 = f3 == FULL;
      if constexpr (BITS == 16) {
        if (w0) fix_u16(o0, x0, 1u, carry, pass_lo);
        if (w1) fix_u16(o1, x1, 1u, carry, pass_lo);
        if (w2) fix_u16(o2, x2, 1u, carry, pass_lo);
        if (w3) fix_u16(o3, x3, 1u, carry, pass_lo);
      } else {
        if (w0) fix_packed<BITS>(o0, x0, 1u, tab, carry, pass_lo);
        if (w1) fix_packed<BITS>(o1, x1, 1u, tab, carry, pass_lo);
        if (w2) fix_packed<BITS>(o2, x2, 1u, tab, carry, pass_lo);
        if (w3) fix_packed<BITS>(o3, x3, 1u, tab, carry, pass_lo);
      }
    }
  } else if constexpr (SPREAD) {
    const uint32_t c = lane_id() & ((1u << sub_log) - 1u);
    if (x0 < W) atomicAdd(&S[(x0 << sub_log) | c], 1u);
    if (x1 < W) atomicAdd(&S[(x1 << sub_log) | c], 1u);
    if (x2 < W) atomicAdd(&S[(x2 << sub_log) | c], 1u);
    if (x3 < W) atomicAdd(&S[(x3 << sub_log) | c], 1u);
  } else {
    const uint32_t y0 = PAD ? pad32(x0) : x0, y1 = PAD ? pad32(x1) : x1;
    const uint32_t y2 = PAD ? pad32(x2) : x2, y3 = PAD ? pad32(x3) : x3;
    if (x0 < W) atomicAdd(&S[y0], 1u);
    if (x1 < W) atomicAdd(&S[y1], 1u);
    if (x2 < W) atomicAdd(&S[y2], 1u);
    if (x3 < W) atomicAdd(&S[y3], 1u);
  }
}

}  // namespace dev
}  // namespace rtcdf
