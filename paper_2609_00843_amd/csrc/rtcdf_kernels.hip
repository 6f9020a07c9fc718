// rtcdf_kernels.hip -- gfx950 kernels of the plain RT-CDF sort.
//
// Stages (Sec. 3, Alg. 4), one launch each:
//   k_hist      tile histograms in LDS (Alg. 5).  All tiles of one LDS pass are
//               counted by one workgroup; every workgroup then writes its LDS
//               counters as one partial row (coalesced, non-atomic) instead of
//               the per-bin global atomics of Alg. 5.
//   k_reduce    sums the partial rows of each bin -> H[R], plus per-128-bin
//               block totals used for the tile offsets.
//   k_tilescan  one workgroup per range tile: local CDF by inclusive scan
//               (Alg. 4), tile offset O[t] (Alg. 6, as a sum of the block
//               totals before the tile), and the value found at each output
//               chunk boundary ("splitters", by bisection in the local CDF as in
//               Alg. 7).
//   k_fill      one workgroup per output chunk: loads the inclusive cumulative
//               counts O[t] + C_t[x] of the values that cover the chunk into LDS
//               and writes every position p the value b_t + min{x : C_t[x] >= p'+1}
//               (Alg. 7 with p' = p - O[t]) as 16-byte stores.
#include <hip/hip_runtime.h>

#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

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

// ------------------------------------------------------------------ histogram

struct HistArgs {
  const int32_t* keys;
  uint64_t in_n4, in_per;
  uint32_t in_head, in_tail;
  uint32_t min_u, W, passes, G, row_words, R;
  uint32_t* partial;
  uint32_t* carry;
};

// Counts one normalised value x (x >= W means "not in this pass").  Lanes of a
// wave holding the same value as the wave's first active lane are merged into
// a single LDS atomic, so all-equal and heavily skewed keys do not serialise
// on one LDS address.
__device__ __forceinline__ void count_u32(uint32_t* S, uint32_t x, uint32_t W) {
  const uint32_t lead = (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
  const uint64_t same = __ballot(x == lead);
  if (x == lead) {
    if (lead < W && lane_id() == (uint32_t)(__ffsll((unsigned long long)same) - 1))
      atomicAdd(&S[lead], (uint32_t)__popcll(same));
  } else if (x < W) {
    atomicAdd(&S[x], 1u);
  }
}

// Two 16-bit counters per LDS word (bin x in half x & 1 of word x >> 1).  The
// returned old word shows whether the add wrapped a half; the lost 2^16 (and
// the +1 a wrap of the low half pushed into the high half) is repaired exactly
// in the global carry array, which the reduction adds back.
__device__ __forceinline__ void count_u16(uint32_t* S, uint32_t x, uint32_t W,
                                          uint32_t* carry, uint32_t pass_lo) {
  const uint32_t lead = (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
  const uint64_t same = __ballot(x == lead);
  uint32_t c = 1;
  bool act;
  if (x == lead) {
    act = lead < W && lane_id() == (uint32_t)(__ffsll((unsigned long long)same) - 1);
    c = (uint32_t)__popcll(same);
  } else {
    act = x < W;
  }
  if (act) {
    const uint32_t sh = (x & 1u) << 4;
    const uint32_t old = atomicAdd(&S[x >> 1], c << sh);
    if (sh == 0) {
      if ((old & 0xffffu) + c > 0xffffu) {
        const uint32_t c2 = ((old >> 16) + 1u) >> 16;  // high half wrapped by the carry
        atomicAdd(&carry[pass_lo + x], 65536u);
        atomicAdd(&carry[pass_lo + x + 1u], 65536u * c2 - 1u);
      }
    } else if ((old >> 16) + c > 0xffffu) {
      atomicAdd(&carry[pass_lo + x], 65536u);
    }
  }
}

template <int ITEMS, bool PACKED, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_hist(HistArgs a) {
  extern __shared__ uint32_t S[];
  // XCD-aware mapping: workgroup ids are dealt round-robin to the 8 XCDs, so
  // the `passes` workgroups that read the same input chunk get consecutive
  // slots on one XCD and the rescans of later passes can hit that XCD's L2.
  const uint32_t wg = blockIdx.x, xcd = wg & 7u, slot = wg >> 3;
  const uint32_t pass = slot % a.passes;
  const uint32_t chunk = (slot / a.passes) * 8u + xcd;
  for (uint32_t i = threadIdx.x; i < a.row_words; i += BLOCK) S[i] = 0u;
  __syncthreads();

  const uint32_t pass_lo = pass * a.W;
  const uint32_t base = a.min_u + pass_lo;   // key (as uint32) of bin 0 of this pass
  const uint32_t W = a.W;
  auto count = [&](int32_t key) {
    const uint32_t x = (uint32_t)key - base;
    if constexpr (PACKED) count_u16(S, x, W, a.carry, pass_lo);
    else count_u32(S, x, W);
  };

  constexpr int V = ITEMS / 4;
  const v4i* body = reinterpret_cast<const v4i*>(a.keys + a.in_head);
  const uint64_t c0 = (uint64_t)chunk * a.in_per;
  const uint64_t c1 = c0 + a.in_per < a.in_n4 ? c0 + a.in_per : a.in_n4;
  for (uint64_t i = c0 + threadIdx.x; i < c1; i += (uint64_t)BLOCK * V) {
    v4i v[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const uint64_t idx = i + (uint64_t)j * BLOCK;
      if (idx < c1) v[j] = __builtin_nontemporal_load(&body[idx]);
      else v[j] = (v4i)(int)(base - 1u);   // lands outside every pass
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      count(v[j].x);
      count(v[j].y);
      count(v[j].z);
      count(v[j].w);
    }
  }
  if (chunk == 0 && threadIdx.x < a.in_head) count(a.keys[threadIdx.x]);
  if (chunk == a.G - 1 && threadIdx.x < a.in_tail)
    count(a.keys[a.in_head + 4 * a.in_n4 + threadIdx.x]);
  __syncthreads();

  uint32_t* row = a.partial + ((size_t)pass * a.G + chunk) * a.row_words;
  for (uint32_t i = threadIdx.x; i < a.row_words; i += BLOCK) row[i] = S[i];
}

// ------------------------------------------------------------------ reduction

struct ReduceArgs {
  const uint32_t* partial;
  uint32_t* carry;
  uint32_t* hist;
  uint32_t* rsum;
  uint32_t R, W, G, row_words, carry_words;
  bool packed;
};

__global__ __launch_bounds__(kReduceBlock) void k_reduce(ReduceArgs a) {
  __shared__ uint32_t red[16][kReduceBins + 1];
  __shared__ uint32_t wsum[kReduceBlock / 64];
  const uint32_t r0 = blockIdx.x * kReduceBins;
  const uint32_t pass = r0 / a.W, o = r0 - pass * a.W;
  const uint32_t* rows = a.partial + (size_t)pass * a.G * a.row_words;
  const uint32_t tid = threadIdx.x;
  if (a.packed) {
    const uint32_t c = tid & 63u, rg = tid >> 6;   // 64 words x 16 row groups
    uint32_t lo = 0, hi = 0;
    for (uint32_t g = rg; g < a.G; g += 16) {
      const uint32_t w = rows[(size_t)g * a.row_words + (o >> 1) + c];
      lo += w & 0xffffu;
      hi += w >> 16;
    }
    red[rg][2 * c] = lo;
    red[rg][2 * c + 1] = hi;
  } else {
    const uint32_t c = tid & 127u, rg = tid >> 7;  // 128 words x 8 row groups
    uint32_t s = 0;
    for (uint32_t g = rg; g < a.G; g += 8) s += rows[(size_t)g * a.row_words + o + c];
    red[rg][c] = s;
  }
  __syncthreads();
  uint32_t tot = 0;
  if (tid < kReduceBins) {
    const uint32_t ngroups = a.packed ? 16u : 8u;
    for (uint32_t g = 0; g < ngroups; ++g) tot += red[g][tid];
    const uint32_t bin = r0 + tid;
    if (a.packed && bin < a.carry_words) {
      tot += a.carry[bin];
      a.carry[bin] = 0u;   // keep the carry array zero between sorts
    }
    if (bin < a.R) a.hist[bin] = tot;
    else tot = 0u;
  }
  const uint32_t s = block_sum(tid < kReduceBins ? tot : 0u, wsum);
  if (tid == 0) a.rsum[blockIdx.x] = s;
}

// ---------------------------------------------------------- local CDF + O[t]

struct ScanArgs {
  uint32_t* hist;         // in: H; out: local CDFs (in place)
  const uint32_t* rsum;
  uint32_t* O;
  uint32_t* split;
  uint64_t n;
  uint32_t R, T, out_head, chunk, nchunks;
};

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
  const uint32_t t = blockIdx.x, tid = threadIdx.x;
  const uint32_t b = t * a.T;
  const uint32_t w = a.R - b < a.T ? a.R - b : a.T;

  // Alg. 6: O[t] = number of keys below b_t = sum of the 128-bin block totals
  // before the tile (b_t is a multiple of 128).
  uint32_t acc = 0;
  for (uint32_t k = tid; k < b / kReduceBins; k += kScanBlock) acc += a.rsum[k];
  const uint32_t Ot = block_sum(acc, wsum);

  // Alg. 4: in-place inclusive scan of H[b, b + w), 1024 bins per step.
  uint32_t run = 0;
  for (uint32_t r0 = 0; r0 < w; r0 += kScanBlock) {
    const uint32_t i = r0 + tid;
    const uint32_t v = i < w ? a.hist[b + i] : 0u;
    uint32_t total;
    const uint32_t inc = block_inclusive_scan(v, wsum, &total);
    if (i < w) {
      C[i] = run + inc;
      a.hist[b + i] = run + inc;
    }
    run += total;
  }
  if (tid == 0) a.O[t] = Ot;
  __syncthreads();
  const uint32_t Nt = run;  // = C[w - 1], the tile's population
  if (Nt == 0) return;

  // Splitters: the value at every chunk start inside [O_t, O_t + N_t), and at
  // position n - 1 (closes the last chunk's window).
  const uint64_t lo = Ot, hi = (uint64_t)Ot + Nt;
  const uint32_t k0 = first_chunk_at_or_after(lo, a.out_head, a.chunk, a.nchunks);
  const uint32_t k1 = first_chunk_at_or_after(hi, a.out_head, a.chunk, a.nchunks);
  for (uint32_t k = k0 + tid; k < k1; k += kScanBlock) {
    const uint64_t s = k == 0 ? 0 : (uint64_t)a.out_head + (uint64_t)k * a.chunk;
    a.split[k] = b + count_le(C, w, (uint32_t)(s - lo));
  }
  if (tid == 0 && a.n - 1 >= lo && a.n - 1 < hi)
    a.split[a.nchunks] = b + count_le(C, w, (uint32_t)(a.n - 1 - lo));
}

// --------------------------------------------------------------------- output

struct FillArgs {
  int32_t* out;
  const uint32_t* cdf;    // local CDFs
  const uint32_t* O;
  const uint32_t* split;
  uint64_t n;
  uint32_t min_u, R, T, out_head, chunk, nchunks;
  uint64_t body_lo, body_hi;   // positions [body_lo, body_hi) are 16-byte aligned int4s
};

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

template <int V>
__global__ __launch_bounds__(kFillBlock) void k_fill(FillArgs a) {
  __shared__ uint32_t win[kFillWindow];
  const uint32_t tid = threadIdx.x;
  for (uint32_t k = blockIdx.x; k < a.nchunks; k += gridDim.x) {
    const uint64_t p0 = k == 0 ? 0 : (uint64_t)a.out_head + (uint64_t)k * a.chunk;
    const uint64_t p1 = k + 1 < a.nchunks ? (uint64_t)a.out_head + (uint64_t)(k + 1) * a.chunk : a.n;
    // Splitters are always in [0, R) for keys inside the declared range; the
    // clamps only keep every access in bounds when that precondition is broken.
    const uint32_t v0 = min(a.split[k], a.R - 1);
    const uint32_t v1 = min(max(a.split[k + 1], v0), a.R - 1);
    const uint32_t nwin = v1 - v0 + 1;
    const uint64_t q_lo = p0 > a.body_lo ? p0 : a.body_lo;
    const uint64_t q_hi = p1 < a.body_hi ? p1 : a.body_hi;
    v4i* body = reinterpret_cast<v4i*>(a.out + a.body_lo);
    const uint64_t i_lo = (q_lo - a.body_lo) >> 2, i_hi = q_hi > q_lo ? (q_hi - a.body_lo) >> 2 : i_lo;
    const int32_t base = (int32_t)(a.min_u + v0);
    if (nwin <= kFillWindow) {
      for (uint32_t j = tid; j < nwin; j += kFillBlock) win[j] = cum_incl(a, v0 + j);
      __syncthreads();
      for (uint64_t i = i_lo + tid; i < i_hi; i += (uint64_t)kFillBlock * V) {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const uint64_t ii = i + (uint64_t)u * kFillBlock;
          if (ii < i_hi) {
            const uint32_t p = (uint32_t)(a.body_lo + 4 * ii);
            const uint32_t last = nwin - 1;
            uint32_t x = min(count_le(win, nwin, p), last);
            v4i o;
            o.x = base + (int32_t)x;
            while (x < last && win[x] <= p + 1) ++x;
            o.y = base + (int32_t)x;
            while (x < last && win[x] <= p + 2) ++x;
            o.z = base + (int32_t)x;
            while (x < last && win[x] <= p + 3) ++x;
            o.w = base + (int32_t)x;
            body[ii] = o;
          }
        }
      }
      // scalar head (positions before the aligned body) and tail
      if (k == 0)
        for (uint64_t p = tid; p < a.body_lo; p += kFillBlock)
          a.out[p] = base + (int32_t)count_le(win, nwin, (uint32_t)p);
      if (k + 1 == a.nchunks)
        for (uint64_t p = a.body_hi + tid; p < a.n; p += kFillBlock)
          a.out[p] = base + (int32_t)count_le(win, nwin, (uint32_t)p);
      __syncthreads();   // window is rewritten by the next chunk
    } else {
      for (uint64_t i = i_lo + tid; i < i_hi; i += kFillBlock) {
        const uint32_t p = (uint32_t)(a.body_lo + 4 * i);
        v4i o;
        o.x = (int32_t)(a.min_u + value_at_global(a, v0, v1, p));
        o.y = (int32_t)(a.min_u + value_at_global(a, v0, v1, p + 1));
        o.z = (int32_t)(a.min_u + value_at_global(a, v0, v1, p + 2));
        o.w = (int32_t)(a.min_u + value_at_global(a, v0, v1, p + 3));
        body[i] = o;
      }
      if (k == 0)
        for (uint64_t p = tid; p < a.body_lo; p += kFillBlock)
          a.out[p] = (int32_t)(a.min_u + value_at_global(a, v0, v1, (uint32_t)p));
      if (k + 1 == a.nchunks)
        for (uint64_t p = a.body_hi + tid; p < a.n; p += kFillBlock)
          a.out[p] = (int32_t)(a.min_u + value_at_global(a, v0, v1, (uint32_t)p));
    }
  }
}

__global__ void k_clear(uint32_t* p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

template <int ITEMS, bool PACKED, int BLOCK>
hipError_t launch_hist_t(const Plan& p, const HistArgs& a, hipStream_t s) {
  const size_t lds = (size_t)p.row_words * 4;
  auto kern = k_hist<ITEMS, PACKED, BLOCK>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(p.passes * p.G), dim3(BLOCK), lds, s, a);
  return hipGetLastError();
}

template <bool PACKED, int BLOCK>
hipError_t launch_hist_items(const Plan& p, const HistArgs& a, hipStream_t s) {
  switch (p.items) {
    case 4: return launch_hist_t<4, PACKED, BLOCK>(p, a, s);
    case 8: return launch_hist_t<8, PACKED, BLOCK>(p, a, s);
    default: return launch_hist_t<16, PACKED, BLOCK>(p, a, s);
  }
}

template <bool PACKED>
hipError_t launch_hist_block(const Plan& p, const HistArgs& a, hipStream_t s) {
  switch (p.hist_block) {
    case 1024: return launch_hist_items<PACKED, 1024>(p, a, s);
    case 512: return launch_hist_items<PACKED, 512>(p, a, s);
    default: return launch_hist_items<PACKED, 256>(p, a, s);
  }
}

}  // namespace

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
  a.in_n4 = p.in_n4;
  a.in_per = p.in_per;
  a.in_head = p.in_head;
  a.in_tail = (uint32_t)(p.n - p.in_head - 4 * p.in_n4);
  a.min_u = p.min_u;
  a.W = p.W;
  a.passes = p.passes;
  a.G = p.G;
  a.row_words = p.row_words;
  a.R = p.R;
  a.partial = reinterpret_cast<uint32_t*>(ws + p.off_partial);
  a.carry = carry;
  return p.packed16 ? launch_hist_block<true>(p, a, s) : launch_hist_block<false>(p, a, s);
}

hipError_t launch_reduce(const Plan& p, uint8_t* ws, uint32_t* carry, hipStream_t s) {
  ReduceArgs a;
  a.partial = reinterpret_cast<const uint32_t*>(ws + p.off_partial);
  a.carry = carry;
  a.hist = reinterpret_cast<uint32_t*>(ws + p.off_hist);
  a.rsum = reinterpret_cast<uint32_t*>(ws + p.off_rsum);
  a.R = p.R;
  a.W = p.W;
  a.G = p.G;
  a.row_words = p.row_words;
  a.carry_words = (uint32_t)p.carry_words;
  a.packed = p.packed16;
  hipLaunchKernelGGL(k_reduce, dim3(p.nred), dim3(kReduceBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tilescan(const Plan& p, uint8_t* ws, hipStream_t s) {
  ScanArgs a;
  a.hist = reinterpret_cast<uint32_t*>(ws + p.off_hist);
  a.rsum = reinterpret_cast<const uint32_t*>(ws + p.off_rsum);
  a.O = reinterpret_cast<uint32_t*>(ws + p.off_O);
  a.split = reinterpret_cast<uint32_t*>(ws + p.off_split);
  a.n = p.n;
  a.R = p.R;
  a.T = p.T;
  a.out_head = p.out_head;
  a.chunk = p.chunk;
  a.nchunks = p.nchunks;
  const size_t lds = (size_t)p.T * 4;
  hipError_t e = hipFuncSetAttribute((const void*)k_tilescan,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tilescan, dim3(p.m), dim3(kScanBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_fill(const Plan& p, int32_t* out, const uint8_t* ws, hipStream_t s) {
  FillArgs a;
  a.out = out;
  a.cdf = reinterpret_cast<const uint32_t*>(ws + p.off_hist);
  a.O = reinterpret_cast<const uint32_t*>(ws + p.off_O);
  a.split = reinterpret_cast<const uint32_t*>(ws + p.off_split);
  a.n = p.n;
  a.min_u = p.min_u;
  a.R = p.R;
  a.T = p.T;
  a.out_head = p.out_head;
  a.chunk = p.chunk;
  a.nchunks = p.nchunks;
  a.body_lo = p.out_head < p.n ? p.out_head : p.n;
  a.body_hi = a.body_lo + 4 * ((p.n - a.body_lo) / 4);
  switch (p.items) {
    case 4: hipLaunchKernelGGL(k_fill<1>, dim3(p.fill_grid), dim3(kFillBlock), 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_fill<2>, dim3(p.fill_grid), dim3(kFillBlock), 0, s, a); break;
    default: hipLaunchKernelGGL(k_fill<4>, dim3(p.fill_grid), dim3(kFillBlock), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace rtcdf
