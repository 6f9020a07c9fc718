// rtcdf_internal.h -- internal plan and kernel launchers of the RT-CDF library.
// Not part of the public ABI (include/rtcdf.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rtcdf.h"

namespace rtcdf {

constexpr uint32_t kLdsBytes = 163840;      // LDS per workgroup/CU on gfx950
constexpr uint32_t kReduceBins = 128;       // bins per workgroup of the partial-row reduction
constexpr uint32_t kFillWindow = 4096;      // cumulative counts held in LDS by one output chunk
constexpr uint32_t kFillBlock = 256;        // threads per output workgroup
constexpr uint32_t kScanBlock = 1024;       // threads per local-CDF workgroup
constexpr uint32_t kReduceBlock = 1024;     // threads per reduction workgroup
constexpr uint32_t kWrapSlots = 64;         // least slots of the narrow histogram's LDS wrap table
constexpr uint32_t kWrapSlotsMax = 4096;    // most slots (the LDS left by the counters permitting)

// Single-tile fast path (one tile, one pass of 32-bit counters, R <= 2048).
// Its accumulation area holds two regions of kFastRegionWords and two parity
// words.  Between sorts, region par[...] and region 1 - par are zero.  The
// histogram adds into region `par`, its workgroup 0 zeroes the other region
// and stores cur = par; the output stage reads region `cur` and its
// workgroup 0 stores par = cur ^ 1.  No word is written while the other
// kernel's workgroups read it, and all state is on the device, so a captured
// graph replays correctly.
constexpr uint32_t kFastMaxRange = 2048;
// ... and fewer than kFastMaxBytes bytes of keys (2^26 int32 keys).  The fast
// path saves the reduction and local-CDF launches (~13 us), but its output
// stage writes more slowly than the staged k_fill at large sizes (measured on
// MI355X, int32 keys, R = 2^7 and 2^11: fast path 7-11 % faster at
// n = 3 x 10^7, staged path 4-5 % faster at 10^8 and 10 % at 3 x 10^8).
constexpr uint64_t kFastMaxBytes = 1ull << 28;
constexpr uint32_t kFastRegionWords = 4096;
constexpr uint32_t kFastPar = 2 * kFastRegionWords;        // word read by the histogram
constexpr uint32_t kFastCur = 2 * kFastRegionWords + 32;   // word read by the output stage
constexpr uint32_t kFastAreaWords = 2 * kFastRegionWords + 64;

// Prefix-maximum output method (Alg. 3): output positions per chunk (one wave
// each): short chunks while n <= kPmaxSmallN (more waves in flight), long ones
// above (fewer chunk carries).
constexpr uint32_t kPmaxChunkSmall = 2048;
constexpr uint32_t kPmaxChunkLarge = 8192;
constexpr uint64_t kPmaxSmallN = 1ull << 21;

// Partition of the keys by LDS pass (rtcdf_part.hip), for ranges that need
// several passes: at most kPartMaxBuckets passes; keys per partition tile.
constexpr uint32_t kPartMaxBuckets = 8192;
constexpr uint32_t kPartTileKeys = 8192;
// The library partitions from kPartMinPasses passes on when n x passes is at
// least kPartMinWork (measured on MI355X: at n = 10^8 the multi-pass
// histogram grows ~0.05 ms a pass against a nearly constant partition cost,
// crossing near 9 passes; smaller n cross later).
constexpr uint32_t kPartMinPasses = 9;
constexpr uint64_t kPartMinWork = 1ull << 26;

// Learned picker: sketch and MLP sizes (see include/rtcdf.h).
constexpr int kSketchBins = 32;
constexpr uint32_t kSketchSamples = 4096;
constexpr int kMlpIn = 2 + kSketchBins;      // log2 n, log2 R, bin fractions
constexpr int kMlpHidden = 64;
constexpr int kMlpOut = RTCDF_GRID_SIZE;     // the configuration grid
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpOut * kMlpHidden + kMlpOut;

// Everything one plain sort needs, derived on the host from (n, range, config,
// pointer alignment, device).  Workspace offsets are in bytes from the base.
struct Plan {
  // problem
  uint64_t n;
  uint32_t kb;           // key bytes: 4 (int32), 2 or 1 (16- and 8-bit keys), 8 (int64)
  uint32_t flip;         // narrow keys: bits XORed with each key (its sign bit if signed)
  uint32_t min_u;        // (uint32)minVal; normalised value x = (uint32)key - min_u
                         // (narrow keys: in the flipped, zero-extended domain; int64
                         // keys: 0, the kernels normalising with min64)
  int64_t min64;         // minVal (int64 keys: x = key - min64, exact in 64 bits)
  uint32_t R;            // range size
  // tile geometry (Sec. 3): m = ceil(R/T), tile t = [tT, tT + w_t)
  uint32_t T, m;
  // config knobs
  uint32_t items, bpt;
  // histogram passes
  uint32_t bits;         // LDS counter width: 32, 16 (two per word) or 8 (four per word)
  bool dedupe;           // wave-level aggregation of a frequent value before the LDS atomics
  uint32_t W;            // bins per LDS pass (multiple of 128, or R rounded up when one pass)
  uint32_t passes;       // ceil(R / W)
  uint32_t G;            // workgroups (input chunks) per pass, multiple of 8
  uint32_t row_words;    // 32-bit words per partial row (W * bits / 32)
  uint32_t wrap_slots;   // narrow counters: slots of the histogram's LDS wrap table
  uint32_t sub_log;      // 32-bit counters: 2^sub_log LDS copies of each bin (0: one)
  uint32_t hist_block;   // threads per histogram workgroup
  uint32_t hist_interleave;  // 1: tiles dealt round-robin to chunks; 0: contiguous chunks
  uint32_t in_head;      // keys before the 16-byte aligned input body
  uint64_t in_n4;        // int4 vectors in the input body
  uint64_t in_per;       // int4 vectors per input chunk
  // reduction
  uint32_t nred;         // ceil(R / kReduceBins)
  // output
  uint32_t out_head;     // output positions before the 16-byte aligned body
  uint32_t chunk;        // output positions per chunk (multiple of 4 * kFillBlock)
  uint32_t nchunks;
  uint32_t fill_grid;
  uint32_t fill_sparse_keys;   // the sparse output form below this many keys per value
  // Single-tile fast path: the histogram accumulates into fast_rows rows of
  // fast_stride words of the fast-path area and the output stage scans them
  // itself; no reduction or local-CDF launch.
  bool fast;
  uint32_t fast_rows, fast_stride;
  // Output by step writes and a prefix maximum (Alg. 3) instead of Alg. 7:
  // pm_chunks chunks of pm_chunk positions (after the min(out_head, n)
  // head), their maxima / carries at off_pm.
  bool pmax;
  uint32_t pm_chunk, pm_chunks, pm_init_grid;
  // Partition by pass (part): part_grid workgroups of part_per keys sort the
  // keys by bucket (= pass) into off_pkeys; the histogram of pass b reads
  // bucket b, whose padded bounds are at off_pbound.
  bool part;
  uint32_t part_grid, part_per, part_buckets;
  uint32_t scan_parts;   // workgroups per tile in the local-CDF stage (fixed split)
  uint32_t scan_grid;    // workgroups of the local-CDF stage; > m: split by chunk counts
  // workspace layout
  size_t off_partial, off_hist, off_cdf, off_rsum, off_O, off_split, off_flags, off_pm, ws_bytes;
  size_t off_pkeys, off_pcnt, off_ptot, off_pbound, off_prow;
  size_t off_carry;      // carry array inside a caller-owned workspace (rtcdf_sort_ws)
  size_t carry_words;    // 0 for 32-bit counters; the fast-path area on the fast path
};

struct DeviceInfo {
  int device = -1;
  int cus = 0;
  bool gfx950 = false;
};

// Kernel launchers (rtcdf_kernels.hip).  All enqueue on `stream` and return the
// hipError_t of the launch.
hipError_t launch_clear(uint32_t* p, size_t words, hipStream_t stream);
// Checked mode: *count (zeroed first) = number of keys[0, n) with
// (uint32)key - min_u >= R.
hipError_t launch_count_out_of_range(const int32_t* keys, uint64_t n, uint32_t min_u, uint32_t R,
                                     uint64_t* count, int cus, hipStream_t stream);
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int cus, hipStream_t stream);
// With p.part the histogram reads the partitioned keys of the workspace and
// `keys` is not read.
hipError_t launch_hist(const Plan& p, const int32_t* keys, uint8_t* ws, uint32_t* carry,
                       hipStream_t stream);
// Partition by pass (rtcdf_part.hip): three launches, before the histogram.
hipError_t launch_partition(const Plan& p, const int32_t* keys, uint8_t* ws, hipStream_t stream);
size_t partition_lds_bytes(uint32_t buckets);
// pm_out: the output B when the plan uses the prefix-maximum output (the
// reduction then also writes the initial B and the local-CDF stage the steps
// of Alg. 3), else null.
hipError_t launch_reduce(const Plan& p, uint8_t* ws, uint32_t* carry, int32_t* pm_out,
                         hipStream_t stream);
hipError_t launch_tilescan(const Plan& p, uint8_t* ws, int32_t* pm_out, hipStream_t stream);
hipError_t launch_fill(const Plan& p, int32_t* out, const uint8_t* ws, hipStream_t stream);
// Prefix-maximum output (rtcdf_pmax.hip): after the steps of Alg. 3 are in B
// and the chunk maxima in the workspace, the prefix maximum of B in place (one
// launch, two with more than 1024 chunks).
uint32_t pmax_chunks(uint64_t n, uint32_t head, uint32_t chunk);
hipError_t launch_output_pmax(const Plan& p, int32_t* out, uint8_t* ws, hipStream_t stream);
// Single-tile fast path: output stage from the counts the histogram left in the
// fast-path area `area` (kFastAreaWords, whose state the launch advances).
hipError_t launch_fill_fast(const Plan& p, int32_t* out, uint32_t* area, hipStream_t stream);

// Batched sort (rtcdf_batched.hip).  batched_plan sizes the workspace from
// the host-side bounds: order_words words of work-item list, slot_words words
// of chunked-tile state, park_words words of park slots for the items that
// sort both range tiles of an in-place segment (counters: 3 words).
struct BatchPlan {
  uint32_t K;            // keys (and output positions) per chunk of a chunked segment
  uint32_t max_slots;    // chunked tiles the workspace holds
  uint32_t max_chunks;   // count items (and fill items) it holds
  uint32_t max_range;    // the bounds' largest range (wider segments are skipped)
  uint64_t items_max;    // work items it holds
  uint64_t order_words;
  uint64_t slot_words;
  uint64_t park_words;
};
BatchPlan batched_plan(uint32_t nseg, uint64_t total_keys, uint32_t cus, uint32_t max_range);
hipError_t launch_batched(const rtcdf_segment_t* segs, uint32_t nseg, const BatchPlan& plan, uint32_t* order,
                          uint32_t* counters, uint32_t* slots, uint32_t* park, uint32_t grid,
                          hipStream_t stream);

// Learned picker (rtcdf_mlp.hip).
hipError_t launch_sketch(const int32_t* keys, uint64_t n, int64_t minVal, uint64_t R, uint32_t samples,
                         float* feat, hipStream_t s);
hipError_t launch_mlp_forward(const float* P, const float* X, uint32_t B, float* Z1, float* Z2, float* Y,
                              hipStream_t s);
hipError_t launch_mlp_grad(const float* P, const float* X, const float* T, const float* M, uint32_t B,
                           float inv_count, float* G, float* loss_dev, float* scratch, hipStream_t s);
size_t mlp_grad_scratch_floats(uint32_t B);
hipError_t launch_adam(float* P, const float* G, float* Mo, float* Vo, float lr, float b1, float b2,
                       float eps, uint32_t t, hipStream_t s);
// out_pred (kMlpOut predictions), out_zmax (the largest |normalised
// feature|) and out_feat (the kMlpIn raw sketch features) may be null.  With
// acc (kPickAccWords device words, zero, returned to zero by the kernel) the
// sampling is spread over kPickGroups workgroups; without it one workgroup
// samples (the same features and outputs either way).
constexpr uint32_t kPickGroups = 16;
constexpr uint32_t kPickAccWords = kSketchBins + 1;
hipError_t launch_pick(const int32_t* keys, uint64_t n, int64_t minVal, uint64_t R, uint32_t samples,
                       const float* P, const float* norm, const uint8_t* valid, uint32_t* out_index,
                       float* out_pred, float* out_zmax, float* out_feat, hipStream_t s,
                       uint32_t* acc = nullptr);

// Host helpers shared by the C ABI translation units (rtcdf_api.hip).
rtcdf_status_t device_info(DeviceInfo* out);
// Raises kernel fn's dynamic LDS limit to `bytes` on the current device, once
// per (kernel, device): each caller passes the largest size any of its
// launches uses, so the attribute is not set again on every launch.
hipError_t ensure_dynamic_lds(const void* fn, int bytes);
rtcdf_status_t hip_fail(hipError_t e);
bool config_valid(const rtcdf_config_t& c);
// What a plan is for: a whole sort; the histogram and reduction of one piece
// of a sort of n >= 2^32 keys (no single-tile fast path, no prefix-maximum
// output: the reduction must leave H); or one output window of such a sort
// (the local-CDF and output stages only: neither of those, and no partition
// by pass, whose key copy the window never uses).
enum class PlanRole { kSort, kPiece, kWindow };

// kb / flip: key width in bytes and the sign-bit flip of narrow signed keys
// (4 / 0 for int32 keys).  `in` and `out` are only inspected for alignment.
void make_plan(size_t n, int64_t minVal, int64_t maxVal, const rtcdf_config_t& cfg,
               const void* in, const void* out, const DeviceInfo& dev, Plan* p, uint32_t kb = 4,
               uint32_t flip = 0, PlanRole role = PlanRole::kSort);

// Sorts of n >= 2^32 keys (rtcdf_wide.hip): the input is counted in pieces
// of kWidePiece keys into 64-bit per-value counts, and the output written in
// windows of kWidePiece positions, each by the plain local-CDF and output
// stages.  Sorts of up to kWideMaxN keys are accepted.
constexpr uint64_t kWidePiece = 1ull << 31;
constexpr uint64_t kWideMaxN = 1ull << 40;
struct WidePlan {
  uint64_t n;
  uint32_t kb, R;
  int cus;
  uint64_t piece;         // keys per piece = positions per window
  uint64_t pieces;        // pieces = windows = ceil(n / piece)
  Plan hist_full, hist_last;   // histogram + reduction of a whole piece / of the last one
  Plan win_full, win_last;     // local-CDF + output stages of a whole window / of the last one
  // workspace: the plain plans' regions (shared, used one stage at a time),
  // then the 64-bit counts H64[R] and the block prefixes of their scan
  size_t off_h64, off_pre, off_carry, carry_words, ws_bytes;
};
void make_wide_plan(size_t n, int64_t minVal, int64_t maxVal, const rtcdf_config_t& cfg, const void* in,
                    const void* out, const DeviceInfo& dev, WidePlan* w, uint32_t kb = 4, uint32_t flip = 0);
// `carry` points at a zeroed array of w.carry_words (narrow counters), which
// the reductions return to zero.
hipError_t enqueue_wide(const WidePlan& w, const void* in, void* out, uint8_t* ws, uint32_t* carry,
                        hipStream_t s);

// Argument checks of the plain sort (n, range, pointers, overlap).
rtcdf_status_t check_problem(const int32_t* keys_in, const int32_t* keys_out, size_t n, int64_t minVal,
                             int64_t maxVal);
// The sort in a device workspace of ws_bytes at d_ws (256-byte aligned),
// after check_problem: no allocation, no host synchronisation.
rtcdf_status_t sort_in_workspace(const int32_t* keys_in, int32_t* keys_out, size_t n, int64_t minVal,
                                 int64_t maxVal, const rtcdf_config_t* cfg, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream);

// The full configuration of a plain sort from the caller's cfg (null or
// zeroed: the library's choice for the config mode, with the learned pick only
// when keys_in is given; partial: the static table's knobs with cfg's flags).
rtcdf_status_t complete_config(const rtcdf_config_t* cfg, const int32_t* keys_in, size_t n, int64_t minVal,
                               int64_t maxVal, hipStream_t stream, rtcdf_config_t* out);
// The static default table's configuration for (n, R) (flags 0).
rtcdf_config_t static_config_for(size_t n, uint32_t R);

// Configuration source (rtcdf_config.hip): the choice rtcdf_sort makes when the
// caller gives no config, under the current config mode.
// With keys_in in LEARNED mode, wait false never waits for the network's pick
// (the first sort of a buffer enqueues it and gets the static choice), wait
// true waits for it.
rtcdf_status_t pick_config(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                           hipStream_t stream, rtcdf_config_t* out, bool wait = false);

}  // namespace rtcdf
