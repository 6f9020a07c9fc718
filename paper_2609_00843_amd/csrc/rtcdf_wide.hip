// rtcdf_wide.hip -- sorts of n >= 2^32 keys: per-value counts in 64 bits.
//
// The plain sort keeps every count and output position in 32 bits (a tile
// histogram entry, the local CDF C_t, the tile offset O_t of Alg. 4-7), which
// holds for n < 2^32.  A larger sort is cut in two directions so that every
// stage of the plain sort still sees fewer than 2^32 keys or positions, and
// only the per-value totals are 64-bit:
//
//   1. Counting.  The input is cut into pieces of kWidePiece keys; each piece
//      is counted by the plain histogram and reduction (Alg. 5, the counts
//      H_s of that piece) and k_acc64 adds H_s into H64[R].
//   2. Cumulative counts.  H64 is scanned in place into the inclusive
//      cumulative counts E(x) = #keys <= minVal + x (Alg. 4 over the whole
//      range in one tile, in 64 bits): k_scan64_local scans blocks of
//      kScan64Chunk values and leaves the block totals, k_scan64_top turns
//      those into exclusive block prefixes; E(x) is the block prefix plus the
//      local value and is formed where it is read.
//   3. Output.  Output window w holds positions [B, B + L), B = w kWidePiece.
//      Value x occupies positions [E(x - 1), E(x)) of the whole output, so
//      the window holds |[E(x - 1), E(x)) intersected with [B, B + L)| copies
//      of it: k_window64 writes these 32-bit counts and their 128-bin block
//      totals where the reduction leaves H and its block totals, and the
//      plain local-CDF and output stages (Alg. 4, 6, 7) of a plan for L keys
//      write the window as the sorted output of those counts.
//
// Every stage of every piece and window is enqueued on one stream in this
// order, so the workspace regions of the plain plans are reused from piece to
// piece and window to window; only H64 and the block prefixes are kept across
// the stages.  The input is read only in step 1, so keys_out may equal keys_in.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rtcdf_device.h"
#include "rtcdf_internal.h"

namespace rtcdf {
namespace {

constexpr uint32_t kScan64Block = 256;   // threads of the 64-bit scan workgroups
constexpr uint32_t kScan64Per = 16;      // values per thread
constexpr uint32_t kScan64Chunk = kScan64Block * kScan64Per;   // values per block (4096)
constexpr uint32_t kWindowBins = 1024;   // values per k_window64 workgroup (8 blocks of 128)

// LDS index with one spare 8-byte entry per 16: a thread's run of 16 values
// then starts 34 words after its neighbour's (2-way bank conflicts, not 64).
__host__ __device__ constexpr uint32_t pad16(uint32_t i) { return i + (i >> 4); }

// Inclusive scan of a 64-bit value over the wave.
__device__ __forceinline__ uint64_t wave_scan64(uint64_t x) {
  const uint32_t lane = dev::lane_id();
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// H64[x] = (first ? 0 : H64[x]) + H[x] for x < R.
__global__ __launch_bounds__(256) void k_acc64(const uint32_t* __restrict__ H, uint64_t* __restrict__ H64,
                                               uint32_t R, uint32_t first) {
  const uint32_t stride = gridDim.x * 256u;
  for (uint32_t x = blockIdx.x * 256u + threadIdx.x; x < R; x += stride)
    H64[x] = (first ? 0ull : H64[x]) + H[x];
}

// Block b of kScan64Chunk values: in-place inclusive scan of H64 over the
// block; tot[b] = the block's total.
__global__ __launch_bounds__(kScan64Block) void k_scan64_local(uint64_t* __restrict__ H64, uint32_t R,
                                                               uint64_t* __restrict__ tot) {
  __shared__ uint64_t s[pad16(kScan64Chunk)];
  __shared__ uint64_t wt[kScan64Block / 64];
  const uint32_t tid = threadIdx.x, lane = dev::lane_id(), wave = tid >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kScan64Chunk;
  for (uint32_t j = tid; j < kScan64Chunk; j += kScan64Block)
    s[pad16(j)] = base + j < R ? H64[base + j] : 0ull;
  __syncthreads();
  uint64_t run = 0;
#pragma unroll
  for (uint32_t k = 0; k < kScan64Per; ++k) {
    run += s[pad16(tid * kScan64Per + k)];
    s[pad16(tid * kScan64Per + k)] = run;
  }
  const uint64_t inc = wave_scan64(run);
  if (lane == 63) wt[wave] = inc;
  __syncthreads();
  uint64_t before = 0, total = 0;
  for (uint32_t w = 0; w < kScan64Block / 64; ++w) {
    if (w < wave) before += wt[w];
    total += wt[w];
  }
  const uint64_t excl = before + inc - run;
#pragma unroll
  for (uint32_t k = 0; k < kScan64Per; ++k) s[pad16(tid * kScan64Per + k)] += excl;
  __syncthreads();
  for (uint32_t j = tid; j < kScan64Chunk; j += kScan64Block)
    if (base + j < R) H64[base + j] = s[pad16(j)];
  if (tid == 0) tot[blockIdx.x] = total;
}

// One workgroup: tot[0, nb) becomes its exclusive prefix sums, in place.
__global__ __launch_bounds__(1024) void k_scan64_top(uint64_t* __restrict__ tot, uint32_t nb) {
  __shared__ uint64_t wt[16];
  const uint32_t tid = threadIdx.x, lane = dev::lane_id(), wave = tid >> 6;
  uint64_t carry = 0;
  for (uint32_t c0 = 0; c0 < nb; c0 += 1024) {
    const uint32_t i = c0 + tid;
    const uint64_t v = i < nb ? tot[i] : 0ull;
    const uint64_t inc = wave_scan64(v);
    if (lane == 63) wt[wave] = inc;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t w = 0; w < 16; ++w) {
      if (w < wave) before += wt[w];
      total += wt[w];
    }
    if (i < nb) tot[i] = carry + before + inc - v;
    carry += total;
    __syncthreads();   // wt is rewritten by the next batch
  }
}

__device__ __forceinline__ uint64_t clamp64(uint64_t e, uint64_t lo, uint64_t hi) {
  return e < lo ? lo : (e > hi ? hi : e);
}

// Window [B, B + L) of the output: H[x] = copies of value x inside the window,
// from the cumulative counts E(x) = pre[x / kScan64Chunk] + H64[x] (H64
// scanned per block, pre the exclusive block prefixes); rsum[k] = the total of
// bins [128k, 128k + 128), as the reduction leaves them; flags[0] = 0 (no
// output chunk flagged sparse yet).  Thread t of a workgroup takes four
// consecutive values, so 32 threads (half a wave) hold one 128-bin block.
__global__ __launch_bounds__(256) void k_window64(const uint64_t* __restrict__ H64, const uint64_t* __restrict__ pre,
                                                  uint32_t R, uint64_t B, uint64_t L, uint32_t* __restrict__ H,
                                                  uint32_t* __restrict__ rsum, uint32_t nred,
                                                  uint32_t* __restrict__ flags) {
  const uint32_t tid = threadIdx.x;
  const uint32_t x0 = blockIdx.x * kWindowBins + 4 * tid;
  const uint64_t hi = B + L;
  uint32_t sum = 0;
  if (x0 < R) {
    // E(x0 - 1): 0 below the first value, the block prefix at a block start
    uint64_t prev;
    if (x0 == 0) prev = 0;
    else if (x0 % kScan64Chunk == 0) prev = pre[x0 / kScan64Chunk];
    else prev = pre[(x0 - 1) / kScan64Chunk] + H64[x0 - 1];
    prev = clamp64(prev, B, hi);
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint32_t x = x0 + k;
      if (x < R) {
        const uint64_t e = clamp64(pre[x / kScan64Chunk] + H64[x], B, hi);
        const uint32_t c = (uint32_t)(e - prev);
        H[x] = c;
        sum += c;
        prev = e;
      }
    }
  }
  // sum over the 32 threads of the 128-bin block
#pragma unroll
  for (uint32_t off = 16; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 32);
  const uint32_t k = blockIdx.x * (kWindowBins / kReduceBins) + tid / 32;
  if ((tid & 31u) == 0 && k < nred) rsum[k] = sum;
  if (blockIdx.x == 0 && tid == 0) flags[0] = 0u;
}

hipError_t launch_acc64(const uint32_t* H, uint64_t* H64, uint32_t R, bool first, int cus, hipStream_t s) {
  const uint32_t grid = (uint32_t)std::min<uint64_t>(((uint64_t)R + 255) / 256, (uint64_t)cus * 8);
  hipLaunchKernelGGL(k_acc64, dim3(grid), dim3(256), 0, s, H, H64, R, first ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_scan64(uint64_t* H64, uint32_t R, uint64_t* tot, hipStream_t s) {
  const uint32_t nb = (R + kScan64Chunk - 1) / kScan64Chunk;
  hipLaunchKernelGGL(k_scan64_local, dim3(nb), dim3(kScan64Block), 0, s, H64, R, tot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan64_top, dim3(1), dim3(1024), 0, s, tot, nb);
  return hipGetLastError();
}

hipError_t launch_window64(const uint64_t* H64, const uint64_t* pre, uint64_t B, uint64_t L, const Plan& p,
                           uint8_t* ws, hipStream_t s) {
  // the window plan's bins are counted in 128-bin blocks, 8 per workgroup
  static_assert(kWindowBins % kReduceBins == 0 && kWindowBins == 4 * 256, "k_window64 geometry");
  const uint32_t grid = (p.R + kWindowBins - 1) / kWindowBins;
  hipLaunchKernelGGL(k_window64, dim3(grid), dim3(256), 0, s, H64, pre, p.R, B, L,
                     reinterpret_cast<uint32_t*>(ws + p.off_hist), reinterpret_cast<uint32_t*>(ws + p.off_rsum),
                     p.nred, reinterpret_cast<uint32_t*>(ws + p.off_flags));
  return hipGetLastError();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

void make_wide_plan(size_t n, int64_t minVal, int64_t maxVal, const rtcdf_config_t& cfg, const void* in,
                    const void* out, const DeviceInfo& dev, WidePlan* w, uint32_t kb, uint32_t flip) {
  *w = WidePlan{};
  w->n = n;
  w->kb = kb;
  w->R = (uint32_t)(maxVal - minVal);
  w->cus = dev.cus;
  w->piece = kWidePiece;
  w->pieces = (n + kWidePiece - 1) / kWidePiece;
  const uint64_t last = n - (w->pieces - 1) * kWidePiece;
  // Pieces and windows start at multiples of kWidePiece keys (a multiple of
  // 16 bytes), so all but the last share the alignment, and the plan, of the
  // first.
  const uint8_t* in_last = static_cast<const uint8_t*>(in) + (w->pieces - 1) * kWidePiece * kb;
  const uint8_t* out_last = static_cast<const uint8_t*>(out) + (w->pieces - 1) * kWidePiece * kb;
  make_plan(kWidePiece, minVal, maxVal, cfg, in, out, dev, &w->hist_full, kb, flip, PlanRole::kPiece);
  make_plan(last, minVal, maxVal, cfg, in_last, out_last, dev, &w->hist_last, kb, flip, PlanRole::kPiece);
  make_plan(kWidePiece, minVal, maxVal, cfg, in, out, dev, &w->win_full, kb, flip, PlanRole::kWindow);
  make_plan(last, minVal, maxVal, cfg, in_last, out_last, dev, &w->win_last, kb, flip, PlanRole::kWindow);
  size_t off = std::max(std::max(w->hist_full.ws_bytes, w->hist_last.ws_bytes),
                        std::max(w->win_full.ws_bytes, w->win_last.ws_bytes));
  off = align256(off);
  w->off_h64 = off;
  off = align256(off + (size_t)w->R * 8);
  w->off_pre = off;
  off = align256(off + (size_t)((w->R + kScan64Chunk - 1) / kScan64Chunk) * 8);
  w->carry_words = std::max(w->hist_full.carry_words, w->hist_last.carry_words);
  w->off_carry = off;   // used by the caller-workspace form only
  off = align256(off + w->carry_words * 4);
  w->ws_bytes = off;
}

hipError_t enqueue_wide(const WidePlan& w, const void* in, void* out, uint8_t* ws, uint32_t* carry,
                        hipStream_t s) {
  uint64_t* h64 = reinterpret_cast<uint64_t*>(ws + w.off_h64);
  uint64_t* pre = reinterpret_cast<uint64_t*>(ws + w.off_pre);
  hipError_t e = hipSuccess;
  for (uint64_t i = 0; i < w.pieces; ++i) {
    const Plan& p = i + 1 < w.pieces ? w.hist_full : w.hist_last;
    const int32_t* keys = reinterpret_cast<const int32_t*>(static_cast<const uint8_t*>(in) + i * w.piece * w.kb);
    if (p.part) {
      e = launch_partition(p, keys, ws, s);
      if (e != hipSuccess) return e;
    }
    e = launch_hist(p, keys, ws, carry, s);
    if (e != hipSuccess) return e;
    e = launch_reduce(p, ws, carry, nullptr, s);
    if (e != hipSuccess) return e;
    e = launch_acc64(reinterpret_cast<const uint32_t*>(ws + p.off_hist), h64, w.R, i == 0, w.cus, s);
    if (e != hipSuccess) return e;
  }
  e = launch_scan64(h64, w.R, pre, s);
  if (e != hipSuccess) return e;
  for (uint64_t i = 0; i < w.pieces; ++i) {
    const Plan& p = i + 1 < w.pieces ? w.win_full : w.win_last;
    const uint64_t B = i * w.piece;
    e = launch_window64(h64, pre, B, p.n, p, ws, s);
    if (e != hipSuccess) return e;
    e = launch_tilescan(p, ws, nullptr, s);
    if (e != hipSuccess) return e;
    e = launch_fill(p, reinterpret_cast<int32_t*>(static_cast<uint8_t*>(out) + B * w.kb), ws, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rtcdf
