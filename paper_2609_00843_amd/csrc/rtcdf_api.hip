// rtcdf_api.hip -- host side of the RT-CDF library: argument checks, planning,
// workspace management and the C ABI declared in include/rtcdf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/rtcdf.h"
#include "rtcdf_internal.h"

namespace rtcdf {

thread_local int g_last_hip_error = 0;

rtcdf_status_t hip_fail(hipError_t e) {
  g_last_hip_error = (int)e;
  return RTCDF_ERROR_HIP;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ devices

static std::mutex g_dev_mu;
static std::map<int, DeviceInfo> g_devs;

rtcdf_status_t device_info(DeviceInfo* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_devs.find(dev);
  if (it == g_devs.end()) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e);
    DeviceInfo d;
    d.device = dev;
    d.cus = prop.multiProcessorCount;
    d.gfx950 = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    it = g_devs.emplace(dev, d).first;
  }
  *out = it->second;
  if (!out->gfx950) return RTCDF_ERROR_NOT_SUPPORTED;
  return RTCDF_SUCCESS;
}

static std::mutex g_attr_mu;
static std::map<std::pair<const void*, int>, int> g_attr_done;

hipError_t ensure_dynamic_lds(const void* fn, int bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_attr_mu);
  auto key = std::make_pair(fn, dev);
  auto it = g_attr_done.find(key);
  if (it != g_attr_done.end() && it->second >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) g_attr_done[key] = bytes;
  return e;
}

// --------------------------------------------------------------- validation

rtcdf_status_t check_problem(const int32_t* keys_in, const int32_t* keys_out, size_t n,
                             int64_t minVal, int64_t maxVal) {
  if (maxVal <= minVal) return RTCDF_ERROR_INVALID_VALUE;
  if (minVal < (int64_t)INT32_MIN || maxVal > (int64_t)INT32_MAX + 1) return RTCDF_ERROR_INVALID_VALUE;
  if ((uint64_t)(maxVal - minVal) > (uint64_t)RTCDF_MAX_RANGE) return RTCDF_ERROR_RANGE_TOO_LARGE;
  if ((uint64_t)n > kWideMaxN) return RTCDF_ERROR_SIZE_TOO_LARGE;
  if (n == 0) return RTCDF_SUCCESS;
  if (keys_in == nullptr || keys_out == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  if ((reinterpret_cast<uintptr_t>(keys_in) & 3u) || (reinterpret_cast<uintptr_t>(keys_out) & 3u))
    return RTCDF_ERROR_INVALID_VALUE;
  if (keys_in != keys_out) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(keys_in), b = reinterpret_cast<uintptr_t>(keys_out);
    const uintptr_t bytes = (uintptr_t)n * 4;
    if (a < b + bytes && b < a + bytes) return RTCDF_ERROR_OVERLAP;
  }
  return RTCDF_SUCCESS;
}

static bool flags_valid(uint32_t f) {
  constexpr uint32_t known = RTCDF_FLAG_OUTPUT_PREFIX_MAX | RTCDF_FLAG_COUNTERS_MASK | RTCDF_FLAG_WAVE_DEDUPE |
                             RTCDF_FLAG_CHUNK_4096;
  if ((f & ~known) != 0) return false;
  const uint32_t cw = f & RTCDF_FLAG_COUNTERS_MASK;
  if ((cw & (cw - 1)) != 0) return false;   // more than one width
  return true;
}

// (T, items, blocks) all zero: the static table's for the problem (see
// complete_config); the flags alone are then the configuration.
static bool config_is_partial(const rtcdf_config_t& c) {
  return c.tile_width == 0 && c.items_per_thread == 0 && c.blocks_per_tile == 0 && c.flags != 0;
}

bool config_valid(const rtcdf_config_t& c) {
  if (!flags_valid(c.flags)) return false;
  if (config_is_partial(c)) return true;
  if (c.tile_width < 128 || c.tile_width > 32768 || (c.tile_width % 128) != 0) return false;
  if (c.items_per_thread != 4 && c.items_per_thread != 8 && c.items_per_thread != 16) return false;
  if (c.blocks_per_tile != 1 && c.blocks_per_tile != 2 && c.blocks_per_tile != 4) return false;
  if ((uint64_t)c.tile_width * 4 * c.blocks_per_tile > kLdsBytes) return false;
  return true;
}

static bool config_is_zero(const rtcdf_config_t* c) {
  return c == nullptr ||
         (c->tile_width == 0 && c->items_per_thread == 0 && c->blocks_per_tile == 0 && c->flags == 0);
}

// The full configuration of a plain sort: the library's choice for a null or
// zeroed cfg (keys_in may be null: no learned pick then), the static table's
// (T, items, blocks) with cfg's flags for a partial cfg, else cfg itself.
rtcdf_status_t complete_config(const rtcdf_config_t* cfg, const int32_t* keys_in, size_t n, int64_t minVal,
                               int64_t maxVal, hipStream_t stream, rtcdf_config_t* out) {
  if (config_is_zero(cfg)) return pick_config(keys_in, n, minVal, maxVal, stream, out);
  if (!config_valid(*cfg)) return RTCDF_ERROR_INVALID_VALUE;
  if (config_is_partial(*cfg)) {
    *out = static_config_for(n, (uint32_t)(maxVal - minVal));
    out->flags = cfg->flags;
    return RTCDF_SUCCESS;
  }
  *out = *cfg;
  return RTCDF_SUCCESS;
}

// ----------------------------------------------------------------- planning

// Developer overrides of launch shapes (RTCDF_DEV_*), read at every plan so a
// measurement script can sweep them; unset means the planner's choice.
static int64_t env_int(const char* name, int64_t dflt) {
  const char* v = std::getenv(name);
  if (v == nullptr || *v == 0) return dflt;
  return std::strtoll(v, nullptr, 10);
}

// Derives every launch parameter and the workspace layout.  `out` is only
// inspected for its alignment.
void make_plan(size_t n, int64_t minVal, int64_t maxVal, const rtcdf_config_t& cfg,
               const void* in, const void* out, const DeviceInfo& dev, Plan* p, uint32_t kb,
               uint32_t flip, PlanRole role) {
  std::memset(p, 0, sizeof(*p));
  const uint32_t R = (uint32_t)(maxVal - minVal);
  p->n = n;
  p->kb = kb;
  p->flip = flip;
  p->min_u = kb == 8 ? 0u : (uint32_t)(uint64_t)(minVal + (int64_t)flip);
  p->min64 = minVal;
  p->R = R;
  // 8- and 16-bit keys: one 16-byte vector of keys per thread per step;
  // int64 keys: two (four keys)
  p->items = kb == 4 ? cfg.items_per_thread : (kb == 8 ? 8u : 4u);
  p->bpt = cfg.blocks_per_tile;
  // Tile geometry (Sec. 3): tiles never need to be wider than the range.
  const uint32_t Rr = (R + 127) & ~127u;
  p->T = std::min<uint32_t>(cfg.tile_width, Rr);
  p->m = (R + p->T - 1) / p->T;

  // Histogram passes: as many whole tiles per workgroup LDS as fit, with 32-bit
  // counters, or with four 8-bit counters per word when that needs fewer
  // passes over the input.
  const uint32_t lds = kLdsBytes / p->bpt;
  const uint32_t k32 = std::max<uint32_t>(1, lds / (4 * p->T));
  // narrow counters leave room for a wrap table of at least 64 slots and its
  // mask word (516 B)
  const uint32_t k16 = std::max<uint32_t>(1, (lds - 516) / (2 * p->T));
  const uint32_t k8 = std::max<uint32_t>(1, (lds - 516) / p->T);
  const uint32_t k4 = std::max<uint32_t>(1, 2 * (lds - 516) / p->T);
  const uint32_t passes32 = (p->m + k32 - 1) / k32;
  const uint32_t passes8 = (p->m + k8 - 1) / k8;
  // 32-bit counters where they need no more passes (no wraps, no returning
  // atomics); otherwise four 8-bit counters per word (measured faster than
  // two 16-bit ones at equal passes: half the partial-row traffic, wraps of hot
  // bins gathered in LDS).  16-bit counters stay selectable for measurement.
  p->bits = passes32 <= passes8 ? 32 : 8;
  const uint32_t cw = cfg.flags & RTCDF_FLAG_COUNTERS_MASK;
  if (cw == RTCDF_FLAG_COUNTERS_16) p->bits = 16;
  else if (cw == RTCDF_FLAG_COUNTERS_32) p->bits = 32;
  else if (cw == RTCDF_FLAG_COUNTERS_4 && kb == 4) p->bits = 4;
  p->dedupe = (cfg.flags & RTCDF_FLAG_WAVE_DEDUPE) != 0 && kb == 4;
  const int force_bits = env_int("RTCDF_DEV_COUNTER_BITS", 0);
  if (force_bits == 8 || force_bits == 16 || force_bits == 32 || (force_bits == 4 && kb == 4))
    p->bits = (uint32_t)force_bits;
  const uint32_t k = p->bits == 4 ? k4 : (p->bits == 8 ? k8 : (p->bits == 16 ? k16 : k32));
  p->passes = (p->m + k - 1) / k;
  // Passes of equal width (whole tiles): no more passes than k tiles a pass
  // needs, and the LDS the counters leave goes to the wrap table.
  p->W = p->passes == 1 ? std::min<uint32_t>(Rr, k * p->T) : (p->m + p->passes - 1) / p->passes * p->T;
  p->row_words = p->W / (32 / p->bits);
  // The wrap table takes the LDS the counters leave, up to kWrapSlotsMax slots:
  // a pass with few bins (R = 2^16 in one pass of 8-bit counters) gives every
  // warm bin of skewed keys a slot of its own.
  p->wrap_slots = kWrapSlots;
  if (p->bits < 32) {
    const uint32_t free_words = lds / 4 > p->row_words + 1 ? lds / 4 - p->row_words - 1 : 0;
    while (p->wrap_slots < kWrapSlotsMax && 4 * p->wrap_slots <= free_words) p->wrap_slots *= 2;
  }
  p->hist_block = 1024 / p->bpt;
  p->hist_interleave = (uint32_t)env_int("RTCDF_DEV_HIST_INTERLEAVE", 1);

  // Input body: 16-byte aligned vectors (16 / kb keys each) between a scalar
  // head and tail.
  const uintptr_t ia = reinterpret_cast<uintptr_t>(in);
  uint64_t head = ((16 - (ia & 15)) & 15) / kb;
  if (head > n) head = n;
  p->in_head = (uint32_t)head;
  p->in_n4 = (n - head) / (16 / kb);
  // One wave of resident workgroups over all passes; chunks per pass a multiple
  // of 8 so the XCD-aware mapping is a bijection.
  const uint32_t V = p->items / 4;
  uint32_t G = (uint32_t)dev.cus * p->bpt / p->passes / 8 * 8;
  if (p->bits == 8) {
    // Bound the keys per workgroup to 10 R, so that values up to ~25 x denser
    // than uniform stay below the 256 hits at which a byte counter wraps (a
    // wrap takes the slow repair path; n = 10^9 normal keys with sd R/64 spent
    // two thirds of their histogram time there).  More workgroups mean more
    // partial rows: their traffic (written once, read once) is capped at 1/32
    // of the 8 bytes per key.
    const uint64_t want = (n + 10ull * R - 1) / (10ull * R);
    const uint64_t cap = n / (32ull * p->passes * p->row_words);
    const uint64_t g = std::min<uint64_t>(want, cap);
    if (g > G) G = (uint32_t)std::min<uint64_t>((g + 7) / 8 * 8, 1u << 16);
  } else if (p->bits == 4) {
    // The same bound for nibble counters (a wrap every 16 hits): at most R
    // keys per workgroup, about one per bin for uniform keys.
    const uint64_t want = (n + (uint64_t)R - 1) / R;
    const uint64_t cap = n / (32ull * p->passes * p->row_words);
    const uint64_t g = std::min<uint64_t>(want, cap);
    if (g > G) G = (uint32_t)std::min<uint64_t>((g + 7) / 8 * 8, 1u << 16);
  }
  const int64_t gmul = env_int("RTCDF_DEV_HIST_GMUL", 1);
  if (gmul > 1 && gmul <= 64) G *= (uint32_t)gmul;
  // The cap on G is taken from the largest body any alignment of the input
  // can have (n / keys per vector), so that G, and with it the partial-row
  // area of the workspace, does not depend on where keys_in starts (the
  // workspace size is asked for without keys_in).
  const uint64_t n4_max = n / (16 / kb);
  const uint64_t iters = (n4_max + (uint64_t)p->hist_block * V - 1) / ((uint64_t)p->hist_block * V);
  const uint64_t gcap = std::max<uint64_t>(8, (iters + 7) / 8 * 8);
  G = (uint32_t)std::min<uint64_t>(std::max<uint32_t>(G, 8), gcap);
  p->G = G;
  p->in_per = (p->in_n4 + G - 1) / G;

  // Partition by pass when the range needs kPartMinPasses or more LDS passes
  // and n x passes is at least kPartMinWork (measured crossover;
  // RTCDF_DEV_PARTITION = 0 / 1 forces it off / on wherever it applies).
  {
    const int64_t force = env_int("RTCDF_DEV_PARTITION", -1);
    // bucket bounds are uint32 positions in the padded copy (at most n + 3 per
    // bucket of padding), so the padded copy must stay below 2^32 keys
    const bool fits = p->passes >= 2 && p->passes <= kPartMaxBuckets && kb == 4 &&
                      (uint64_t)n + 4ull * p->passes + 4 <= 0xffffffffull;
    p->part = fits && role != PlanRole::kWindow &&
              (force == 1 || (force != 0 && p->passes >= kPartMinPasses && (uint64_t)n * p->passes >= kPartMinWork));
    if (p->part) {
      p->part_buckets = p->passes;
      const uint64_t tiles = (n + kPartTileKeys - 1) / kPartTileKeys;
      const uint64_t per_cu = (uint64_t)std::max<int64_t>(1, env_int("RTCDF_DEV_PART_WGS_PER_CU", 4));
      p->part_grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(tiles, (uint64_t)dev.cus * per_cu));
      p->part_per = (uint32_t)((n + p->part_grid - 1) / p->part_grid);
    }
  }

  // LDS copies of 32-bit counters (2^sub_log, at most 16, as many as the LDS
  // holds; not with the partition by pass or wave aggregation).  8-bit keys
  // take 8: their 256 bins put many of a wave's 64 x 16 keys on one word per
  // atomic (measured on MI355X at n = 10^8: uint8 uniform 8 % and concentrated
  // 18 % faster, int8 4 %); wider keys lose 0-11 % to the copies.
  {
    const int64_t want = env_int("RTCDF_DEV_HIST_SPREAD", kb == 1 ? 3 : 0);
    p->sub_log = 0;
    if (p->bits == 32 && !p->dedupe && !p->part && want > 0)
      while (p->sub_log < (uint32_t)std::min<int64_t>(want, 4) &&
             ((size_t)p->row_words << (p->sub_log + 1)) * 4 <= lds)
        ++p->sub_log;
  }

  p->nred = (R + kReduceBins - 1) / kReduceBins;

  // Output chunks: s(0) = 0, s(k) = out_head + k * chunk; the output body
  // starts on a 16-byte boundary (keys_out is aligned to the key size).
  const uintptr_t oa = reinterpret_cast<uintptr_t>(out);
  p->out_head = (uint32_t)(((16 - (oa & 15)) & 15) / kb);
  const uint32_t gran = 4 * kFillBlock;
  const uint64_t fill_per_cu = (uint64_t)env_int("RTCDF_DEV_FILL_WGS_PER_CU", 4);
  // Chunks of 2048 positions (8 KiB of output): the workgroups interleave
  // chunk by chunk, so the whole chip writes one narrow moving window.
  uint64_t want = 2048;
  // 16- and 8-bit keys: the dense output step covers 8 or 16 keys a lane, so
  // 8192-position chunks (16 or 8 KiB) keep every wave busy and repay the
  // per-chunk work over as many bytes (measured 21-26 % faster at n = 10^8);
  // from 4 keys per value on, so that a chunk's values fit the LDS window.
  if (kb < 4 && n >= 4ull * R) want = 8192;
  if (kb == 4 && (cfg.flags & RTCDF_FLAG_CHUNK_4096)) want = 4096;
  const int64_t force_chunk = env_int("RTCDF_DEV_FILL_CHUNK", 0);
  if (force_chunk > 0) want = (uint64_t)force_chunk;
  p->chunk = (uint32_t)((want + gran - 1) / gran * gran);
  p->nchunks = 1 + ((n >= 1 && n - 1 >= p->out_head) ? (uint32_t)((n - 1 - p->out_head) / p->chunk) : 0);
  p->fill_grid = (uint32_t)std::min<uint64_t>(p->nchunks, (uint64_t)dev.cus * fill_per_cu);
  p->fill_sparse_keys = (uint32_t)std::max<int64_t>(0, env_int("RTCDF_DEV_FILL_SPARSE_KEYS", 64));
  // Local-CDF stage: enough workgroups to spread the splitters over the chip,
  // but no more than one per 256 chunk starts.  With at most kScanBlock tiles
  // and 8 * kScanBlock block totals the kernel assigns the workgroups to tiles
  // by their share of chunk starts (it sees the counts); otherwise every tile
  // gets the same number of workgroups.
  const uint32_t by_work = std::max<uint32_t>(1, p->nchunks / 256);
  if (p->m <= kScanBlock && p->nred <= 8 * kScanBlock) {
    p->scan_parts = 1;
    // one per tile plus up to 64 spares (all-equal keys: ~760 splitters each at n = 10^8)
    p->scan_grid = p->m + std::min<uint32_t>(64u, by_work);
  } else {
    const uint32_t want_parts = std::max<uint32_t>(1, (uint32_t)dev.cus / p->m);
    p->scan_parts = std::min<uint32_t>(want_parts, std::max<uint32_t>(1, by_work / p->m));
    p->scan_grid = p->m * p->scan_parts;
  }

  // Single-tile fast path: one tile, one pass of 32-bit counters, at most
  // kFastMaxRange bins and fewer than kFastMaxBytes bytes of keys.  The histogram adds into accumulation rows of the
  // fast-path area and the output stage sums and scans them itself.  Rows
  // spread the atomics of the histogram workgroups over more addresses; every
  // output workgroup reads rows * stride <= kFastRegionWords words.
  // Prefix-maximum output (Alg. 3) in place of Alg. 7: runs after the staged
  // local-CDF stage, so it never takes the fast path.
  p->pmax = (cfg.flags & RTCDF_FLAG_OUTPUT_PREFIX_MAX) != 0 && kb == 4 && role == PlanRole::kSort;
  if (p->pmax) {
    const uint32_t h = (uint32_t)std::min<uint64_t>(p->out_head, n);
    p->pm_chunk = n <= kPmaxSmallN ? kPmaxChunkSmall : kPmaxChunkLarge;
    p->pm_chunks = pmax_chunks(n, h, p->pm_chunk);
    const uint64_t n4 = (n - h) / 4;
    p->pm_init_grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n4 + 255) / 256,
                                                                         (uint64_t)dev.cus * 8));
  }
  p->fast = p->m == 1 && p->bits == 32 && p->passes == 1 && R <= kFastMaxRange && (uint64_t)n * kb < kFastMaxBytes &&
            !p->pmax && role == PlanRole::kSort && env_int("RTCDF_DEV_FAST", 1) != 0;
  if (p->fast) {
    p->fast_stride = Rr;
    const int64_t force_rows = env_int("RTCDF_DEV_FAST_ROWS", 0);
    const uint32_t max_rows = std::max<uint32_t>(1u, kFastRegionWords / Rr);
    p->fast_rows = force_rows > 0 ? (uint32_t)std::min<int64_t>(force_rows, max_rows)
                                  : std::min<uint32_t>(16u, max_rows);
  }

  // Workspace layout.
  size_t off = 0;
  // Partial rows: one per histogram workgroup; with the partition by pass
  // one per piece of a bucket in a workgroup's range, numbered workgroup +
  // bucket (at most passes more).
  p->off_partial = off;
  off = align256(off + ((size_t)p->passes * p->G + (p->part ? p->passes : 0)) * p->row_words * 4);
  p->off_hist = off;
  off = align256(off + (size_t)R * 4);
  p->off_cdf = off;
  off = align256(off + (size_t)R * 4);
  p->off_rsum = off;
  off = align256(off + (size_t)p->nred * 4);
  p->off_O = off;
  off = align256(off + (size_t)p->m * 4);
  p->off_split = off;
  off = align256(off + ((size_t)p->nchunks + 1) * 4);
  p->off_flags = off;                       // [0]: some output chunk is sparse
  off = align256(off + 4);
  p->off_pm = off;                          // prefix-maximum output: chunk maxima / carries
  off = align256(off + (size_t)p->pm_chunks * 4);
  // partition by pass: keys (each bucket padded to 4), counts, totals, bounds
  const size_t P = p->part ? p->part_buckets : 0;
  p->off_pkeys = off;
  off = align256(off + (p->part ? ((size_t)n + 4 * P + 4) * 4 : 0));
  p->off_pcnt = off;
  off = align256(off + P * p->part_grid * 4);
  p->off_ptot = off;
  off = align256(off + P * 4);
  p->off_pbound = off;
  off = align256(off + (p->part ? (P + 1) * 4 : 0));
  p->off_prow = off;                        // each bucket's first partial row and their number
  off = align256(off + P * 8);
  // Carry entries cover every bin of every pass (plus the partner of the last
  // bin), so even keys outside the declared range stay in bounds.
  p->carry_words = p->bits < 32 ? (size_t)p->passes * p->W + 4 : 0;
  if (p->fast) p->carry_words = kFastAreaWords;   // the fast-path area
  p->off_carry = off;                       // used by the caller-workspace form only
  off = align256(off + p->carry_words * 4);
  p->ws_bytes = off;
}

// ------------------------------------------------------------ workspaces

// The library's own workspace for rtcdf_sort: one per (device, stream), so
// sorts on different streams never share scratch memory.  The carry array of
// the 16-bit counters lives in its own buffer that is zero between sorts
// (zeroed when allocated, re-zeroed by the reduction after every use).
struct Workspace {
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t* carry = nullptr;
  size_t carry_words = 0;
  // The single-tile fast path's accumulation area (zeroed when allocated; the
  // kernels keep its state consistent from sort to sort).  Set dirty when a
  // sort could not enqueue all its stages, which re-zeroes it before the next.
  uint32_t* fast = nullptr;
  bool fast_dirty = false;
  uint64_t* check = nullptr;   // checked mode: the out-of-range count
  // A sort captured into a HIP graph keeps raw pointers to these buffers, and
  // the graph may be replayed at any time: once a capture has used them they
  // are never freed (growth moves them to g_retired instead).
  bool captured = false;
};

static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
static std::vector<void*> g_retired;   // buffers of captured workspaces, kept until exit

// Frees a buffer of workspace w, or keeps it alive if a capture used it.
// `s` is the workspace's stream: its work is the only work that reads the
// buffer, so waiting for it (not for the whole device) makes the free safe.
static hipError_t drop_buffer(Workspace& w, void* ptr, hipStream_t s) {
  if (ptr == nullptr) return hipSuccess;
  if (w.captured) {
    g_retired.push_back(ptr);
    return hipSuccess;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  return hipFree(ptr);
}

static rtcdf_status_t grow(Workspace& w, const Plan& p, hipStream_t s) {
  if (w.ws_bytes < p.ws_bytes) {
    hipError_t e = drop_buffer(w, w.ws, s);
    if (e != hipSuccess) return hip_fail(e);
    w.ws = nullptr;
    w.ws_bytes = 0;
    const size_t bytes = std::max<size_t>(p.ws_bytes, (size_t)1 << 20);
    e = hipMalloc(&w.ws, bytes);
    if (e != hipSuccess) {
      w.ws = nullptr;
      (void)hipGetLastError();
      return RTCDF_ERROR_OUT_OF_MEMORY;
    }
    w.ws_bytes = bytes;
  }
  if (p.fast && w.fast == nullptr) {
    hipError_t e = hipMalloc(&w.fast, (size_t)kFastAreaWords * 4);
    if (e != hipSuccess) {
      w.fast = nullptr;
      (void)hipGetLastError();
      return RTCDF_ERROR_OUT_OF_MEMORY;
    }
    // cleared on the sort's stream: a hipMemset runs on the null stream,
    // which a non-blocking stream's kernels do not wait for
    e = launch_clear(w.fast, kFastAreaWords, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (!p.fast && w.carry_words < p.carry_words) {
    hipError_t e = drop_buffer(w, w.carry, s);
    if (e != hipSuccess) return hip_fail(e);
    w.carry = nullptr;
    w.carry_words = 0;
    const size_t words = std::max<size_t>(p.carry_words, 1 << 16);
    e = hipMalloc(&w.carry, words * 4);
    if (e != hipSuccess) {
      w.carry = nullptr;
      (void)hipGetLastError();
      return RTCDF_ERROR_OUT_OF_MEMORY;
    }
    e = launch_clear(w.carry, words, s);   // on the sort's stream, as above
    if (e != hipSuccess) return hip_fail(e);
    w.carry_words = words;
  }
  return RTCDF_SUCCESS;
}

// Whether work enqueued on `s` now is being captured into a graph.
static rtcdf_status_t capturing(hipStream_t s, bool* out) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return hip_fail(e);
  *out = cs != hipStreamCaptureStatusNone;
  return RTCDF_SUCCESS;
}

// True when the cached workspace already holds everything plan p needs.
static bool fits_cached(const Workspace& w, const Plan& p) {
  if (w.ws_bytes < p.ws_bytes) return false;
  if (p.fast) return w.fast != nullptr;
  return w.carry_words >= p.carry_words;
}

// ------------------------------------------------------------- profiling

// Optional per-stage timing: when enabled, every sort records HIP events on
// its own stream before the histogram and after each stage.  rtcdf_profile_collect
// waits for them and sums the elapsed time per stage.
static std::atomic<bool> g_prof{false};
static std::mutex g_prof_mu;
struct StageMarks {
  hipEvent_t ev[5];
};
static std::vector<StageMarks> g_prof_pending;
static std::vector<hipEvent_t> g_prof_pool;

static hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Enqueue the four stages (two on the fast path).  `carry` points at a zeroed
// array of p.carry_words, or at the fast-path area on the fast path.
static rtcdf_status_t enqueue(const Plan& p, const int32_t* in, int32_t* out, uint8_t* ws,
                              uint32_t* carry, hipStream_t s, uint32_t* dbg_hist = nullptr,
                              uint32_t* dbg_cdf = nullptr, uint32_t* dbg_O = nullptr) {
  const Plan& q = p;
  StageMarks marks;
  bool prof = g_prof.load() && out != nullptr;
  if (prof) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& ev : marks.ev) {
      ev = prof_event();
      if (ev == nullptr) prof = false;
    }
  }
  auto mark = [&](int i) {
    if (prof) (void)hipEventRecord(marks.ev[i], s);
  };
  mark(0);
  hipError_t e = hipSuccess;
  if (q.part) {
    e = launch_partition(q, in, ws, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  e = launch_hist(q, in, ws, carry, s);
  if (e != hipSuccess) return hip_fail(e);
  mark(1);
  if (q.fast) {   // the output stage does the reduction and the scan
    mark(2);
    mark(3);
    e = launch_fill_fast(q, out, carry, s);
    if (e != hipSuccess) return hip_fail(e);
    mark(4);
    if (prof) {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_prof_pending.push_back(marks);
    }
    return RTCDF_SUCCESS;
  }
  int32_t* pm_out = q.pmax ? out : nullptr;   // null on the debug path (no output)
  e = launch_reduce(q, ws, carry, pm_out, s);
  if (e != hipSuccess) return hip_fail(e);
  mark(2);
  if (dbg_hist) {
    e = hipMemcpyAsync(dbg_hist, ws + q.off_hist, (size_t)q.R * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  e = launch_tilescan(q, ws, pm_out, s);
  if (e != hipSuccess) return hip_fail(e);
  mark(3);
  if (dbg_cdf) {
    e = hipMemcpyAsync(dbg_cdf, ws + q.off_cdf, (size_t)q.R * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (dbg_O) {
    e = hipMemcpyAsync(dbg_O, ws + q.off_O, (size_t)q.m * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (out) {
    e = q.pmax ? launch_output_pmax(q, out, ws, s) : launch_fill(q, out, ws, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  mark(4);
  if (prof) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back(marks);
  }
  return RTCDF_SUCCESS;
}

// A sort of n >= 2^32 keys in the library's workspace (see rtcdf_wide.hip).
// The configuration is the caller's, or the static choice for a piece of
// kWidePiece keys (the learned pick is not consulted); the prefix-maximum
// output is never taken.
static rtcdf_status_t sort_wide_cached(const int32_t* in, int32_t* out, size_t n, int64_t minVal,
                                       int64_t maxVal, const rtcdf_config_t* cfg, hipStream_t s, bool cap,
                                       const DeviceInfo& dev, uint32_t kb, uint32_t flip) {
  rtcdf_config_t c;
  rtcdf_status_t st = complete_config(cfg, nullptr, kWidePiece, minVal, maxVal, s, &c);
  if (st != RTCDF_SUCCESS) return st;
  if (kb != 4) c.flags = 0;
  WidePlan wp;
  make_wide_plan(n, minVal, maxVal, c, in, out, dev, &wp, kb, flip);
  Plan need;   // what the cached workspace must hold
  std::memset(&need, 0, sizeof(need));
  need.ws_bytes = wp.ws_bytes;
  need.carry_words = wp.carry_words;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  Workspace& w = g_ws[std::make_pair(dev.device, s)];
  if (cap) {
    if (!fits_cached(w, need)) return RTCDF_ERROR_CAPTURE_NEEDS_WORKSPACE;
    w.captured = true;
  }
  st = grow(w, need, s);
  if (st != RTCDF_SUCCESS) return st;
  const hipError_t e = enqueue_wide(wp, in, out, static_cast<uint8_t*>(w.ws), w.carry, s);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

// kb / flip: 8- and 16-bit keys (see make_plan); their configuration never
// takes the prefix-maximum output, and the learned picker (whose sketch
// reads int32 keys) is not consulted for them.
static rtcdf_status_t sort_cached(const int32_t* in, int32_t* out, size_t n, int64_t minVal,
                                  int64_t maxVal, const rtcdf_config_t* cfg, hipStream_t s,
                                  uint32_t* dbg_hist, uint32_t* dbg_cdf, uint32_t* dbg_O,
                                  uint32_t kb = 4, uint32_t flip = 0) {
  DeviceInfo dev;
  rtcdf_status_t st = device_info(&dev);
  if (st != RTCDF_SUCCESS) return st;
  // Under stream capture nothing may allocate, free or wait on the host: the
  // learned pick (which reads its result back) is skipped, and the cached
  // workspace must already be large enough (a sort of the same or a larger
  // problem on this stream before the capture allocates it).
  bool cap = false;
  st = capturing(s, &cap);
  if (st != RTCDF_SUCCESS) return st;
  if (n > 0xffffffffull) {
    if (out == nullptr) return RTCDF_ERROR_SIZE_TOO_LARGE;   // intermediates: n < 2^32 only
    return sort_wide_cached(in, out, n, minVal, maxVal, cfg, s, cap, dev, kb, flip);
  }
  rtcdf_config_t c;
  st = complete_config(cfg, (kb == 4 && !cap) ? in : nullptr, n, minVal, maxVal, s, &c);
  if (st != RTCDF_SUCCESS) return st;
  if (kb != 4) c.flags = 0;
  Plan p;
  make_plan(n, minVal, maxVal, c, in, out ? out : in, dev, &p, kb, flip);
  // The intermediates are only materialised by the staged path.
  if (out == nullptr) p.fast = false;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  Workspace& w = g_ws[std::make_pair(dev.device, s)];
  if (cap) {
    if (!fits_cached(w, p)) return RTCDF_ERROR_CAPTURE_NEEDS_WORKSPACE;
    w.captured = true;
  }
  st = grow(w, p, s);
  if (st != RTCDF_SUCCESS) return st;
  if (!p.fast)
    return enqueue(p, in, out, static_cast<uint8_t*>(w.ws), w.carry, s, dbg_hist, dbg_cdf, dbg_O);
  if (w.fast_dirty) {
    hipError_t e = launch_clear(w.fast, kFastAreaWords, s);
    if (e != hipSuccess) return hip_fail(e);
    w.fast_dirty = false;
  }
  st = enqueue(p, in, out, static_cast<uint8_t*>(w.ws), w.fast, s);
  if (st != RTCDF_SUCCESS) w.fast_dirty = true;
  return st;
}

// The sort in a workspace the caller provides (rtcdf_sort_ws) or the
// library's fixed device array (rtcdf_sort_noalloc): no allocation, no host
// synchronisation.  Arguments are checked by the caller; d_ws is 256-byte
// aligned.  The configuration never comes from the learned pick (which reads
// its result back to the host): the TUNED/DEFAULT choice is used.
rtcdf_status_t sort_in_workspace(const int32_t* keys_in, int32_t* keys_out, size_t n, int64_t minVal,
                                 int64_t maxVal, const rtcdf_config_t* cfg, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream) {
  DeviceInfo dev;
  rtcdf_status_t st = device_info(&dev);
  if (st != RTCDF_SUCCESS) return st;
  rtcdf_config_t c;
  if (n > 0xffffffffull) {   // n >= 2^32: counts in 64 bits (rtcdf_wide.hip)
    st = complete_config(cfg, nullptr, kWidePiece, minVal, maxVal, nullptr, &c);
    if (st != RTCDF_SUCCESS) return st;
    WidePlan wp;
    make_wide_plan(n, minVal, maxVal, c, keys_in, keys_out, dev, &wp);
    if (ws_bytes < wp.ws_bytes) return RTCDF_ERROR_WORKSPACE_TOO_SMALL;
    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    uint32_t* carry = reinterpret_cast<uint32_t*>(ws + wp.off_carry);
    hipError_t e = wp.carry_words ? launch_clear(carry, wp.carry_words, stream) : hipSuccess;
    if (e == hipSuccess) e = enqueue_wide(wp, keys_in, keys_out, ws, carry, stream);
    return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
  }
  st = complete_config(cfg, nullptr, n, minVal, maxVal, nullptr, &c);
  if (st != RTCDF_SUCCESS) return st;
  Plan p;
  make_plan(n, minVal, maxVal, c, keys_in, keys_out, dev, &p);
  if (ws_bytes < p.ws_bytes) return RTCDF_ERROR_WORKSPACE_TOO_SMALL;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  uint32_t* carry = reinterpret_cast<uint32_t*>(ws + p.off_carry);
  // The carry array (or the fast path's accumulation area) must start at
  // zero: cleared by a kernel, so no memset node enters a captured graph.
  if (p.carry_words) {
    hipError_t e = launch_clear(carry, p.carry_words, stream);
    if (e != hipSuccess) return hip_fail(e);
  }
  return enqueue(p, keys_in, keys_out, ws, carry, stream);
}

}  // namespace rtcdf

using namespace rtcdf;

extern "C" {

rtcdf_status_t rtcdf_sort(const int32_t* keys_in, int32_t* keys_out, size_t n, int64_t minVal,
                          int64_t maxVal, hipStream_t stream) {
  return rtcdf_sort_with_config(keys_in, keys_out, n, minVal, maxVal, nullptr, stream);
}

rtcdf_status_t rtcdf_sort_with_config(const int32_t* keys_in, int32_t* keys_out, size_t n,
                                      int64_t minVal, int64_t maxVal, const rtcdf_config_t* cfg,
                                      hipStream_t stream) {
  rtcdf_status_t st = check_problem(keys_in, keys_out, n, minVal, maxVal);
  if (st != RTCDF_SUCCESS || n == 0) return st;
  if (!config_is_zero(cfg) && !config_valid(*cfg)) return RTCDF_ERROR_INVALID_VALUE;
  return sort_cached(keys_in, keys_out, n, minVal, maxVal, cfg, stream, nullptr, nullptr, nullptr);
}

rtcdf_status_t rtcdf_sort_keys(const void* keys_in, void* keys_out, size_t n, int key_type,
                               int64_t minVal, int64_t maxVal, const rtcdf_config_t* cfg,
                               hipStream_t stream) {
  uint32_t kb, flip;
  int64_t lo, hi;   // the key type's values, [lo, hi)
  switch (key_type) {
    case RTCDF_KEY_INT32:
      return rtcdf_sort_with_config(static_cast<const int32_t*>(keys_in), static_cast<int32_t*>(keys_out),
                                    n, minVal, maxVal, cfg, stream);
    case RTCDF_KEY_INT16: kb = 2; flip = 0x8000u; lo = -32768; hi = 32768; break;
    case RTCDF_KEY_UINT16: kb = 2; flip = 0u; lo = 0; hi = 65536; break;
    case RTCDF_KEY_INT8: kb = 1; flip = 0x80u; lo = -128; hi = 128; break;
    case RTCDF_KEY_UINT8: kb = 1; flip = 0u; lo = 0; hi = 256; break;
    case RTCDF_KEY_INT64: kb = 8; flip = 0u; lo = INT64_MIN; hi = INT64_MAX; break;
    default: return RTCDF_ERROR_INVALID_VALUE;
  }
  if (maxVal <= minVal || minVal < lo || maxVal > hi) return RTCDF_ERROR_INVALID_VALUE;
  if ((uint64_t)maxVal - (uint64_t)minVal > RTCDF_MAX_RANGE) return RTCDF_ERROR_RANGE_TOO_LARGE;
  if ((uint64_t)n > kWideMaxN) return RTCDF_ERROR_SIZE_TOO_LARGE;
  if (n == 0) return RTCDF_SUCCESS;
  if (keys_in == nullptr || keys_out == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  const uintptr_t a = reinterpret_cast<uintptr_t>(keys_in), b = reinterpret_cast<uintptr_t>(keys_out);
  if ((a % kb) != 0 || (b % kb) != 0) return RTCDF_ERROR_INVALID_VALUE;
  const uintptr_t bytes = (uintptr_t)n * kb;
  if (a != b && a < b + bytes && b < a + bytes) return RTCDF_ERROR_OVERLAP;
  if (!config_is_zero(cfg) && (!config_valid(*cfg) || cfg->flags != 0)) return RTCDF_ERROR_INVALID_VALUE;
  return sort_cached(static_cast<const int32_t*>(keys_in), static_cast<int32_t*>(keys_out), n, minVal, maxVal,
                     cfg, stream, nullptr, nullptr, nullptr, kb, flip);
}

rtcdf_status_t rtcdf_count_out_of_range(const int32_t* keys, size_t n, int64_t minVal, int64_t maxVal,
                                        uint64_t* d_count, hipStream_t stream) {
  if (d_count == nullptr || (reinterpret_cast<uintptr_t>(d_count) & 7u)) return RTCDF_ERROR_INVALID_VALUE;
  rtcdf_status_t st = check_problem(keys, keys, n, minVal, maxVal);
  if (st != RTCDF_SUCCESS) return st;
  DeviceInfo dev;
  st = device_info(&dev);
  if (st != RTCDF_SUCCESS) return st;
  const hipError_t e = launch_count_out_of_range(keys, n, (uint32_t)(int32_t)minVal,
                                                 (uint32_t)(maxVal - minVal), d_count, dev.cus, stream);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

rtcdf_status_t rtcdf_sort_checked(const int32_t* keys_in, int32_t* keys_out, size_t n, int64_t minVal,
                                  int64_t maxVal, const rtcdf_config_t* cfg, hipStream_t stream) {
  rtcdf_status_t st = check_problem(keys_in, keys_out, n, minVal, maxVal);
  if (st != RTCDF_SUCCESS || n == 0) return st;
  if (!config_is_zero(cfg) && !config_valid(*cfg)) return RTCDF_ERROR_INVALID_VALUE;
  DeviceInfo dev;
  st = device_info(&dev);
  if (st != RTCDF_SUCCESS) return st;
  uint64_t bad = 0;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace& w = g_ws[std::make_pair(dev.device, stream)];
    if (w.check == nullptr) {
      hipError_t e = hipMalloc(&w.check, 256);
      if (e != hipSuccess) {
        w.check = nullptr;
        (void)hipGetLastError();
        return RTCDF_ERROR_OUT_OF_MEMORY;
      }
    }
    hipError_t e = launch_count_out_of_range(keys_in, n, (uint32_t)(int32_t)minVal,
                                             (uint32_t)(maxVal - minVal), w.check, dev.cus, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, w.check, sizeof(bad), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (bad != 0) return RTCDF_ERROR_KEY_OUT_OF_RANGE;
  return sort_cached(keys_in, keys_out, n, minVal, maxVal, cfg, stream, nullptr, nullptr, nullptr);
}

rtcdf_status_t rtcdf_workspace_bytes(size_t n, int64_t minVal, int64_t maxVal,
                                     const rtcdf_config_t* cfg, const int32_t* keys_out,
                                     size_t* bytes) {
  if (bytes == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  const int32_t* probe = keys_out ? keys_out : reinterpret_cast<const int32_t*>((uintptr_t)256);
  rtcdf_status_t st = check_problem(probe, probe, n, minVal, maxVal);
  if (st != RTCDF_SUCCESS) return st;
  if (n == 0) {
    *bytes = 0;
    return RTCDF_SUCCESS;
  }
  DeviceInfo dev;
  st = device_info(&dev);
  if (st != RTCDF_SUCCESS) return st;
  rtcdf_config_t c;
  const bool wide = n > 0xffffffffull;
  st = complete_config(cfg, nullptr, wide ? kWidePiece : n, minVal, maxVal, nullptr, &c);
  if (st != RTCDF_SUCCESS) return st;
  if (wide) {
    WidePlan wp;
    make_wide_plan(n, minVal, maxVal, c, probe, probe, dev, &wp);
    *bytes = wp.ws_bytes;
    return RTCDF_SUCCESS;
  }
  Plan p;
  // The layout depends on n, R, the config and keys_out's alignment (output
  // chunk starts); keys_in's alignment changes only the histogram's head and
  // tail, never the number of its workgroups (see make_plan).
  make_plan(n, minVal, maxVal, c, probe, probe, dev, &p);
  *bytes = p.ws_bytes;
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_sort_ws(const int32_t* keys_in, int32_t* keys_out, size_t n, int64_t minVal,
                             int64_t maxVal, const rtcdf_config_t* cfg, void* d_ws, size_t ws_bytes,
                             hipStream_t stream) {
  rtcdf_status_t st = check_problem(keys_in, keys_out, n, minVal, maxVal);
  if (st != RTCDF_SUCCESS || n == 0) return st;
  if (d_ws == nullptr || (reinterpret_cast<uintptr_t>(d_ws) & 255u)) return RTCDF_ERROR_INVALID_VALUE;
  return sort_in_workspace(keys_in, keys_out, n, minVal, maxVal, cfg, d_ws, ws_bytes, stream);
}

rtcdf_status_t rtcdf_debug_intermediates(const int32_t* keys_in, size_t n, int64_t minVal,
                                         int64_t maxVal, const rtcdf_config_t* cfg,
                                         uint32_t* d_hist, uint32_t* d_cdf, uint32_t* d_offsets,
                                         hipStream_t stream) {
  rtcdf_status_t st = check_problem(keys_in, keys_in, n, minVal, maxVal);
  if (st != RTCDF_SUCCESS) return st;
  if (n == 0) return RTCDF_ERROR_INVALID_VALUE;
  if (n > 0xffffffffull) return RTCDF_ERROR_SIZE_TOO_LARGE;
  if (config_is_zero(cfg) || !config_valid(*cfg)) return RTCDF_ERROR_INVALID_VALUE;
  return sort_cached(keys_in, nullptr, n, minVal, maxVal, cfg, stream, d_hist, d_cdf, d_offsets);
}

// ---- batched

struct BatchLayout {
  size_t off_counters, off_order, off_slots, off_park, bytes;
  uint32_t grid;
  BatchPlan plan;
};

static rtcdf_status_t batch_layout(uint32_t nseg, const rtcdf_batch_bounds_t* bounds, BatchLayout* L) {
  if (bounds == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  if (bounds->max_range > RTCDF_BATCH_MAX_RANGE) return RTCDF_ERROR_RANGE_TOO_LARGE;
  DeviceInfo dev;
  rtcdf_status_t st = device_info(&dev);
  if (st != RTCDF_SUCCESS) return st;
  L->plan = batched_plan(nseg, bounds->total_keys, dev.cus, bounds->max_range);
  // one persistent workgroup per compute unit, or one per work item
  L->grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)dev.cus, L->plan.items_max));
  L->off_counters = 0;
  L->off_order = 256;
  L->off_slots = align256(L->off_order + L->plan.order_words * 4);
  L->off_park = align256(L->off_slots + L->plan.slot_words * 4);
  L->bytes = align256(L->off_park + L->plan.park_words * 4);
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_batched_workspace_bytes(uint32_t num_segments, const rtcdf_batch_bounds_t* bounds,
                                             size_t* bytes) {
  if (bytes == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  BatchLayout L;
  rtcdf_status_t st = batch_layout(num_segments, bounds, &L);
  if (st != RTCDF_SUCCESS) return st;
  *bytes = L.bytes;
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_sort_batched(const rtcdf_segment_t* d_segments, uint32_t num_segments,
                                  const rtcdf_batch_bounds_t* bounds, void* d_ws, size_t ws_bytes,
                                  hipStream_t stream) {
  if (bounds == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  if (num_segments == 0) return RTCDF_SUCCESS;
  if (d_segments == nullptr || d_ws == nullptr || (reinterpret_cast<uintptr_t>(d_ws) & 255u) ||
      (reinterpret_cast<uintptr_t>(d_segments) & 7u))
    return RTCDF_ERROR_INVALID_VALUE;
  BatchLayout L;
  rtcdf_status_t st = batch_layout(num_segments, bounds, &L);
  if (st != RTCDF_SUCCESS) return st;
  if (ws_bytes < L.bytes) return RTCDF_ERROR_WORKSPACE_TOO_SMALL;
  uint8_t* ws = static_cast<uint8_t*>(d_ws);
  hipError_t e = launch_batched(d_segments, num_segments, L.plan, reinterpret_cast<uint32_t*>(ws + L.off_order),
                                reinterpret_cast<uint32_t*>(ws + L.off_counters),
                                reinterpret_cast<uint32_t*>(ws + L.off_slots),
                                reinterpret_cast<uint32_t*>(ws + L.off_park), L.grid, stream);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

const char* rtcdf_status_string(rtcdf_status_t s) {
  switch (s) {
    case RTCDF_SUCCESS: return "success";
    case RTCDF_ERROR_INVALID_VALUE: return "invalid value";
    case RTCDF_ERROR_SIZE_TOO_LARGE: return "n too large (sorts: n <= 2^40; plan and intermediates: n < 2^32)";
    case RTCDF_ERROR_RANGE_TOO_LARGE: return "range too large";
    case RTCDF_ERROR_OVERLAP: return "input and output overlap partially";
    case RTCDF_ERROR_OUT_OF_MEMORY: return "out of device memory";
    case RTCDF_ERROR_HIP: return "HIP error";
    case RTCDF_ERROR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case RTCDF_ERROR_NOT_SUPPORTED: return "not supported on this device";
    case RTCDF_ERROR_NO_MODEL: return "no model loaded";
    case RTCDF_ERROR_KEY_OUT_OF_RANGE: return "a key lies outside [minVal, maxVal)";
    case RTCDF_ERROR_CAPTURE_NEEDS_WORKSPACE:
      return "the stream is being captured and the library's workspace would have to grow";
  }
  return "unknown status";
}

int rtcdf_last_hip_error(void) { return g_last_hip_error; }

rtcdf_status_t rtcdf_profile_enable(int on) {
  g_prof.store(on != 0);
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_profile_collect(rtcdf_stage_stats_t* out) {
  if (out == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  std::memset(out, 0, sizeof(*out));
  std::lock_guard<std::mutex> lk(g_prof_mu);
  rtcdf_status_t st = RTCDF_SUCCESS;
  for (StageMarks& m : g_prof_pending) {
    hipError_t e = hipEventSynchronize(m.ev[4]);
    if (e != hipSuccess) st = hip_fail(e);
    for (int i = 0; i < 4 && e == hipSuccess; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, m.ev[i], m.ev[i + 1]) == hipSuccess) out->ms[i] += ms;
    }
    out->sorts += 1;
    for (auto& ev : m.ev) g_prof_pool.push_back(ev);
  }
  g_prof_pending.clear();
  return st;
}

int rtcdf_version(void) { return 100; }

static_assert(sizeof(rtcdf_plan_info_t) == 72, "rtcdf_plan_info_t layout (the Python binding mirrors it)");

rtcdf_status_t rtcdf_plan_info(size_t n, int64_t minVal, int64_t maxVal, const rtcdf_config_t* cfg,
                               const int32_t* keys_in, const int32_t* keys_out, rtcdf_plan_info_t* out) {
  if (out == nullptr || n == 0) return RTCDF_ERROR_INVALID_VALUE;
  const int32_t* probe = reinterpret_cast<const int32_t*>((uintptr_t)256);
  rtcdf_status_t st = check_problem(probe, probe, n, minVal, maxVal);
  if (st != RTCDF_SUCCESS) return st;
  if (n > 0xffffffffull) return RTCDF_ERROR_SIZE_TOO_LARGE;   // one plan describes n < 2^32 only
  DeviceInfo dev;
  st = device_info(&dev);
  if (st != RTCDF_SUCCESS) return st;
  rtcdf_config_t c;
  st = complete_config(cfg, nullptr, n, minVal, maxVal, nullptr, &c);
  if (st != RTCDF_SUCCESS) return st;
  Plan p;
  make_plan(n, minVal, maxVal, c, keys_in ? keys_in : probe, keys_out ? keys_out : probe, dev, &p);
  out->tile_width = p.T;
  out->tiles = p.m;
  out->counter_bits = p.bits;
  out->passes = p.passes;
  out->pass_bins = p.W;
  out->hist_workgroups = p.passes * p.G;
  out->hist_threads = p.hist_block;
  out->items_per_thread = p.items;
  out->scan_workgroups = p.fast ? 0 : p.scan_grid;
  out->out_chunk = p.pmax ? p.pm_chunk : p.chunk;
  out->out_chunks = p.pmax ? p.pm_chunks : p.nchunks;
  out->fill_workgroups = p.pmax ? (p.pm_chunks + 3) / 4 : p.fill_grid;
  out->workspace_bytes = p.ws_bytes;
  out->output_flags = p.pmax ? RTCDF_FLAG_OUTPUT_PREFIX_MAX : 0u;
  out->partition_buckets = p.part ? p.part_buckets : 0u;
  out->hist_dedupe = p.dedupe ? 1u : 0u;
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_stream_copy(const void* d_src, void* d_dst, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return RTCDF_SUCCESS;
  if (d_src == nullptr || d_dst == nullptr || (bytes & 15u) ||
      (reinterpret_cast<uintptr_t>(d_src) & 15u) || (reinterpret_cast<uintptr_t>(d_dst) & 15u))
    return RTCDF_ERROR_INVALID_VALUE;
  DeviceInfo dev;
  rtcdf_status_t st = device_info(&dev);
  if (st != RTCDF_SUCCESS) return st;
  hipError_t e = launch_stream_copy(d_src, d_dst, bytes, dev.cus, stream);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

rtcdf_status_t rtcdf_release_workspaces(void) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  hipError_t e = hipDeviceSynchronize();
  for (auto it = g_ws.begin(); it != g_ws.end();) {
    Workspace& w = it->second;
    if (w.captured) {   // a captured graph may still replay with these buffers
      ++it;
      continue;
    }
    if (w.ws) (void)hipFree(w.ws);
    if (w.carry) (void)hipFree(w.carry);
    if (w.fast) (void)hipFree(w.fast);
    if (w.check) (void)hipFree(w.check);
    it = g_ws.erase(it);
  }
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

}  // extern "C"
