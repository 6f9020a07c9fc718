// rtcdf_config.hip -- where rtcdf_sort gets its kernel configuration from when
// the caller passes none (DEFAULT: static per-range table; TUNED: nearest
// entry of a loaded tuning table; LEARNED: the MLP picker, with exhaustive
// autotuning where the network is not trusted), the configuration grid, the
// exhaustive autotuner, and the C ABI of the picker's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/rtcdf.h"
#include "rtcdf_default_table.h"
#include "rtcdf_internal.h"

namespace rtcdf {

static std::atomic<int> g_mode{RTCDF_CONFIG_DEFAULT};

// ------------------------------------------------------------------ grid

// The tuning grid: kPlainPoints (T, items, blocks) points with no option flags
// (the search output and the library's counter width; index 9 log2(T/1024) +
// 3 log2(items/4) + log2(blocks)), then the option points: the static table's
// (T, items, blocks) for the problem with one set of option flags.
constexpr int kPlainPoints = 54;
constexpr uint32_t kGridOptions[RTCDF_GRID_SIZE - kPlainPoints] = {
    RTCDF_FLAG_OUTPUT_PREFIX_MAX,
    RTCDF_FLAG_COUNTERS_16,
    RTCDF_FLAG_COUNTERS_16 | RTCDF_FLAG_WAVE_DEDUPE,
    RTCDF_FLAG_WAVE_DEDUPE,
    RTCDF_FLAG_CHUNK_4096,
    RTCDF_FLAG_COUNTERS_16 | RTCDF_FLAG_CHUNK_4096,
    RTCDF_FLAG_COUNTERS_32,
    RTCDF_FLAG_COUNTERS_4,
};
static_assert(RTCDF_GRID_SIZE == kMlpOut, "one network output per grid point");

rtcdf_config_t grid_config(int i) {
  rtcdf_config_t c;
  if (i >= kPlainPoints) {
    c.tile_width = c.items_per_thread = c.blocks_per_tile = 0;
    c.flags = kGridOptions[i - kPlainPoints];
    return c;
  }
  c.tile_width = 1024u << (i / 9);
  c.items_per_thread = 4u << ((i / 3) % 3);
  c.blocks_per_tile = 1u << (i % 3);
  c.flags = 0;
  return c;
}

bool grid_valid(int i) { return config_valid(grid_config(i)); }

// ------------------------------------------------------------ default table

static rtcdf_config_t default_config(size_t n, uint32_t R) {
  (void)n;
  for (const DefaultRow& row : kDefaultTable)
    if (R <= row.max_range) return row.cfg;
  return kDefaultTable[sizeof(kDefaultTable) / sizeof(kDefaultTable[0]) - 1].cfg;
}

rtcdf_config_t static_config_for(size_t n, uint32_t R) { return default_config(n, R); }

// Grid point i as a full configuration for (n, R): option points take the
// static table's (T, items, blocks).
static rtcdf_config_t resolve_grid_point(int i, size_t n, uint32_t R) {
  rtcdf_config_t c = grid_config(i);
  if (i >= kPlainPoints) {
    const rtcdf_config_t b = default_config(n, R);
    c.tile_width = b.tile_width;
    c.items_per_thread = b.items_per_thread;
    c.blocks_per_tile = b.blocks_per_tile;
  }
  return c;
}

// -------------------------------------------------------------- tuned table

struct TunedRow {
  double log2n, log2r;
  rtcdf_config_t cfg;   // may be an option point (T, items, blocks 0)
};
static std::mutex g_cfg_mu;
static std::vector<TunedRow> g_tuned;

static bool tuned_config(size_t n, uint32_t R, rtcdf_config_t* out) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  if (g_tuned.empty() || n == 0) return false;
  const double a = std::log2((double)n), b = std::log2((double)R);
  double best = 1e300;
  for (const TunedRow& r : g_tuned) {
    const double d = (r.log2n - a) * (r.log2n - a) + (r.log2r - b) * (r.log2r - b);
    if (d < best) {
      best = d;
      *out = r.cfg;
    }
  }
  if (out->tile_width == 0) {   // an option point: the static table's knobs with its flags
    const uint32_t f = out->flags;
    *out = default_config(n, R);
    out->flags = f;
  }
  return true;
}

// ------------------------------------------------------------ output method

// Output method (the adaptive selection between Alg. 7 and Alg. 3 that the
// paper leaves as future work in Sec. 4.1): the prefix maximum when the range
// is at least kPmaxMinRange and at least n.  There the search path spends its
// output stage walking many sparse values per output chunk, while the
// prefix-maximum steps are written one value per thread by the local-CDF
// stage; measured on MI355X over n in [10^3, 10^7] and R in [2^8, 2^24] with
// uniform, normal and all-equal keys.  RTCDF_DEV_OUTPUT_RULE=0 keeps the
// search everywhere (for measurement).  The learned picker can choose the
// prefix maximum elsewhere (a grid point) from the keys' sketch.
constexpr uint32_t kPmaxMinRange = 1u << 14;

static uint32_t output_method_flags(size_t n, uint32_t R) {
  const char* v = std::getenv("RTCDF_DEV_OUTPUT_RULE");
  if (v != nullptr && v[0] == '0' && v[1] == 0) return 0u;
  return (R >= kPmaxMinRange && (uint64_t)R >= (uint64_t)n) ? RTCDF_FLAG_OUTPUT_PREFIX_MAX : 0u;
}

// The choice without the network: the TUNED row (unless mode is DEFAULT) or
// the static table's (T, items, blocks), with the output-method rule's flags
// (a tuned row that is an option point keeps its own flags).
static rtcdf_config_t static_choice(size_t n, uint32_t R, int mode) {
  rtcdf_config_t c;
  if (mode == RTCDF_CONFIG_DEFAULT || !tuned_config(n, R, &c)) c = default_config(n, R);
  if (c.flags == 0) c.flags = output_method_flags(n, R);
  return c;
}

// Grid index of a full configuration for (n, R): a plain point, or an option
// point whose knobs are the static table's; -1 if it is neither.
static int grid_index(const rtcdf_config_t& c, size_t n, uint32_t R) {
  if (c.flags == 0) {
    for (int i = 0; i < kPlainPoints; ++i) {
      const rtcdf_config_t g = grid_config(i);
      if (g.tile_width == c.tile_width && g.items_per_thread == c.items_per_thread &&
          g.blocks_per_tile == c.blocks_per_tile)
        return i;
    }
    return -1;
  }
  const rtcdf_config_t b = default_config(n, R);
  if (b.tile_width != c.tile_width || b.items_per_thread != c.items_per_thread ||
      b.blocks_per_tile != c.blocks_per_tile)
    return -1;
  for (int i = kPlainPoints; i < RTCDF_GRID_SIZE; ++i)
    if (kGridOptions[i - kPlainPoints] == c.flags) return i;
  return -1;
}

// ------------------------------------------------------------- learned model

struct Model {
  bool loaded = false;
  std::vector<float> params, norm;      // norm: mean[34] then sd[34]
  std::vector<uint8_t> valid;           // per grid point
  float log2n_lo = 0, log2n_hi = 0, log2r_lo = 0, log2r_hi = 0;   // training ranges
  float margin = 0;                     // least predicted log-time gain that is acted on
  float zmax = 0;                       // feature range trusted (0: no limit)
};
// The pick kernel writes its result into a slot of pinned host memory: word 0
// the argmin index, words kPickPred.. the predictions, kPickZ the largest
// |normalised feature|, kPickFeat.. the raw sketch features.  Each slot has an
// event recorded after its kernel, so a sort can ask whether the result is
// there without waiting.
constexpr int kPickPred = 1, kPickZ = 1 + kMlpOut, kPickFeat = 2 + kMlpOut;
constexpr int kPickWords = 2 + kMlpOut + kMlpIn;
constexpr int kPickSlots = 64;          // picks in flight per device
struct DeviceModel {
  float* params = nullptr;
  float* norm = nullptr;
  uint8_t* valid = nullptr;
  uint32_t* host = nullptr;             // pinned, kPickSlots x kPickWords
  uint32_t* dev = nullptr;              // its device address
  uint32_t* acc = nullptr;              // device, kPickSlots x 64 words: the spread sketch's bins (zero)
  hipEvent_t ev[kPickSlots] = {};
  std::vector<int> free_slots;
  std::vector<int> draining;            // slots of dropped entries whose pick may still run
  uint64_t generation = 0;
};
static Model g_model;
static uint64_t g_model_generation = 0;
static std::map<int, DeviceModel> g_dev_models;
static std::atomic<bool> g_fallback{true};

// Decisions of LEARNED mode per (device, keys_in, n, minVal, maxVal, model
// generation): an entry is pending while its pick runs, then resolved, so a
// buffer sorted again costs no pick.  Exhaustive autotuning results are kept
// per shape class (fallback_class).
using PickKey = std::tuple<int, uintptr_t, uint64_t, int64_t, int64_t, uint64_t>;
using ClassKey = std::tuple<int, int, int, int, int, uint64_t>;
struct Decision {
  rtcdf_config_t cfg;
  int index;    // grid index, -1 if none
  int source;   // RTCDF_PICK_* of the decision
};
struct PickEntry {
  bool resolved = false;
  int dev = -1, slot = -1;              // pending: where its pick writes
  Decision d;
};
static std::map<PickKey, PickEntry> g_pick_cache;
static std::map<ClassKey, int> g_class_best;
constexpr size_t kPickCacheMax = 4096;

thread_local int t_last_index = -1;
thread_local int t_last_source = RTCDF_PICK_STATIC;

static rtcdf_status_t upload_model(int dev, DeviceModel** out) {
  DeviceModel& d = g_dev_models[dev];
  if (d.host == nullptr) {
    hipError_t e = hipMalloc(&d.params, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&d.norm, sizeof(float) * 2 * kMlpIn);
    if (e == hipSuccess) e = hipMalloc(&d.valid, kMlpOut);
    // the picks' results go straight to pinned host memory (no copy launch)
    if (e == hipSuccess)
      e = hipHostMalloc(&d.host, sizeof(uint32_t) * kPickWords * kPickSlots, hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&d.dev), d.host, 0);
    if (e == hipSuccess) e = hipMalloc(&d.acc, sizeof(uint32_t) * 64 * kPickSlots);
    if (e == hipSuccess) e = hipMemset(d.acc, 0, sizeof(uint32_t) * 64 * kPickSlots);
    // the memset runs on the null stream, which the picks' (possibly
    // non-blocking) streams do not wait for: wait for it here, once
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    for (int k = 0; k < kPickSlots && e == hipSuccess; ++k) {
      e = hipEventCreateWithFlags(&d.ev[k], hipEventDisableTiming);
      if (e == hipSuccess) d.free_slots.push_back(k);
    }
    if (e != hipSuccess) {
      d.host = nullptr;
      d.free_slots.clear();
      return hip_fail(e);
    }
  }
  if (d.generation != g_model_generation) {
    hipError_t e = hipMemcpy(d.params, g_model.params.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(d.norm, g_model.norm.data(), sizeof(float) * 2 * kMlpIn, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.valid, g_model.valid.data(), kMlpOut, hipMemcpyHostToDevice);
    // a copy from pageable memory may return before its transfer lands, and
    // it runs on the null stream: wait for it before a pick reads the weights
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) return hip_fail(e);
    d.generation = g_model_generation;
  }
  *out = &d;
  return RTCDF_SUCCESS;
}

// A free result slot (slots of dropped entries are reused once their pick
// has finished), or -1.
static int acquire_slot(DeviceModel& d) {
  for (auto it = d.draining.begin(); it != d.draining.end();) {
    if (hipEventQuery(d.ev[*it]) == hipSuccess) {
      d.free_slots.push_back(*it);
      it = d.draining.erase(it);
    } else {
      ++it;
    }
  }
  if (d.free_slots.empty()) return -1;
  const int s = d.free_slots.back();
  d.free_slots.pop_back();
  return s;
}

// Forgets every decision (g_cfg_mu held); pending picks keep their slots
// until they have finished.
static void drop_picks() {
  for (auto& kv : g_pick_cache) {
    const PickEntry& en = kv.second;
    if (!en.resolved && en.slot >= 0) g_dev_models[en.dev].draining.push_back(en.slot);
  }
  g_pick_cache.clear();
}

// Shape class of an array for the exhaustive fallback's cache: n and R to
// half an octave, and the sketch's largest bin fraction (in quarters) and the
// eighth of the range its largest bin lies in.
static ClassKey fallback_class(int dev, size_t n, uint32_t R, const float* feat) {
  int arg = 0;
  float mx = -1.f;
  for (int b = 0; b < kSketchBins; ++b)
    if (feat[2 + b] > mx) {
      mx = feat[2 + b];
      arg = b;
    }
  return ClassKey(dev, (int)std::lround(2.0 * std::log2((double)n)), (int)std::lround(2.0 * std::log2((double)R)),
                  std::min(3, (int)(4.f * mx)), arg / (kSketchBins / 8), g_model_generation);
}

// Exhaustive autotuning of the grid on this array (into a scratch output, so
// the caller's buffers are untouched): the index of the fastest point.
static rtcdf_status_t autotune_index(const int32_t* keys, size_t n, int64_t minVal, int64_t maxVal,
                                     hipStream_t stream, int* best) {
  int32_t* tmp = nullptr;
  hipError_t e = hipMalloc(&tmp, n * sizeof(int32_t));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return RTCDF_ERROR_OUT_OF_MEMORY;
  }
  std::vector<float> t(RTCDF_GRID_SIZE);
  rtcdf_status_t st = rtcdf_autotune(keys, tmp, n, minVal, maxVal, 1, 3, t.data(), nullptr, stream);
  e = hipStreamSynchronize(stream);
  (void)hipFree(tmp);
  if (st != RTCDF_SUCCESS) return st;
  if (e != hipSuccess) return hip_fail(e);
  int bi = -1;
  for (int i = 0; i < RTCDF_GRID_SIZE; ++i)
    if (t[i] > 0.f && (bi < 0 || t[i] < t[bi])) bi = i;
  *best = bi;
  return RTCDF_SUCCESS;
}

// LEARNED mode.  The first call for a buffer enqueues the pick kernel on
// `stream` (sketch of keys -> network -> argmin, into a pinned slot) and, with
// wait false, returns the static choice (source PENDING) without waiting; a
// later call whose pick has finished decides: the network's point where it
// predicts at least the model's margin less than for the static choice, else
// the static choice; where the network is not trusted (n or R outside its
// training ranges, or a sketch farther than zmax from its training
// features) the grid is timed exhaustively (once per shape class).  With
// wait true the call waits for the pick and decides at once.
static rtcdf_status_t learned_decision(const int32_t* keys, size_t n, int64_t minVal, int64_t maxVal,
                                       hipStream_t stream, bool wait, Decision* out) {
  const uint32_t R = (uint32_t)(maxVal - minVal);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  const rtcdf_config_t stat = static_choice(n, R, RTCDF_CONFIG_TUNED);
  out->cfg = stat;
  out->index = grid_index(stat, n, R);
  out->source = RTCDF_PICK_STATIC;
  std::unique_lock<std::mutex> lk(g_cfg_mu);
  if (!g_model.loaded || keys == nullptr || n == 0) return RTCDF_SUCCESS;
  const PickKey key(dev, reinterpret_cast<uintptr_t>(keys), (uint64_t)n, minVal, maxVal, g_model_generation);
  auto it = g_pick_cache.find(key);
  if (it == g_pick_cache.end()) {
    DeviceModel* d = nullptr;
    rtcdf_status_t st = upload_model(dev, &d);
    if (st != RTCDF_SUCCESS) return st;
    const int slot = acquire_slot(*d);
    if (slot < 0) return RTCDF_SUCCESS;   // every slot in flight: the static choice this time
    uint32_t* res = d->dev + (size_t)slot * kPickWords;
    e = launch_pick(keys, n, minVal, (uint64_t)R, kSketchSamples, d->params, d->norm, d->valid, res,
                    reinterpret_cast<float*>(res + kPickPred), reinterpret_cast<float*>(res + kPickZ),
                    reinterpret_cast<float*>(res + kPickFeat), stream, d->acc + (size_t)slot * 64);
    if (e == hipSuccess) e = hipEventRecord(d->ev[slot], stream);
    if (e != hipSuccess) {
      d->draining.push_back(slot);
      return hip_fail(e);
    }
    if (g_pick_cache.size() >= kPickCacheMax) drop_picks();
    PickEntry en;
    en.dev = dev;
    en.slot = slot;
    it = g_pick_cache.emplace(key, en).first;
  }
  if (it->second.resolved) {
    *out = it->second.d;
    if (out->source != RTCDF_PICK_STATIC) out->source = RTCDF_PICK_CACHED;
    return RTCDF_SUCCESS;
  }
  DeviceModel& d = g_dev_models[it->second.dev];
  const int slot = it->second.slot;
  if (slot < 0) {   // another thread is deciding (its exhaustive timing runs unlocked)
    out->source = RTCDF_PICK_PENDING;
    return RTCDF_SUCCESS;
  }
  if (wait) {
    e = hipEventSynchronize(d.ev[slot]);
    if (e != hipSuccess) return hip_fail(e);
  } else if (hipEventQuery(d.ev[slot]) != hipSuccess) {
    out->source = RTCDF_PICK_PENDING;
    return RTCDF_SUCCESS;
  }
  uint32_t res[kPickWords];
  std::memcpy(res, d.host + (size_t)slot * kPickWords, sizeof(res));
  d.free_slots.push_back(slot);
  it->second.slot = -1;
  const uint32_t idx = res[0];
  const float* pred = reinterpret_cast<const float*>(res + kPickPred);
  float z;
  std::memcpy(&z, res + kPickZ, sizeof(float));
  const float* feat = reinterpret_cast<const float*>(res + kPickFeat);
  const double a = std::log2((double)n), b = std::log2((double)R);
  const bool in_range = a >= g_model.log2n_lo - 0.5 && a <= g_model.log2n_hi + 0.5 &&
                        b >= g_model.log2r_lo - 0.5 && b <= g_model.log2r_hi + 0.5;
  const bool trusted = in_range && (g_model.zmax <= 0.f || z <= g_model.zmax) && idx < (uint32_t)kMlpOut &&
                       grid_valid((int)idx);
  if (trusted) {
    const int si = out->index;
    if (si >= 0 && g_model.valid[si] && pred[si] - pred[idx] < g_model.margin) {
      out->source = RTCDF_PICK_NETWORK_KEPT_STATIC;
    } else {
      out->cfg = resolve_grid_point((int)idx, n, R);
      out->index = (int)idx;
      out->source = RTCDF_PICK_NETWORK;
    }
  } else if (g_fallback.load()) {
    const ClassKey ck = fallback_class(dev, n, R, feat);
    auto cb = g_class_best.find(ck);
    int bi = -1;
    if (cb != g_class_best.end()) {
      bi = cb->second;
    } else {
      lk.unlock();   // the autotuner sorts through the public entry points
      rtcdf_status_t st = autotune_index(keys, n, minVal, maxVal, stream, &bi);
      lk.lock();
      if (st != RTCDF_SUCCESS) {
        g_pick_cache.erase(key);
        return st;
      }
      g_class_best[ck] = bi;
    }
    if (bi >= 0) {
      out->cfg = resolve_grid_point(bi, n, R);
      out->index = bi;
      out->source = RTCDF_PICK_AUTOTUNED;
    }
  }
  auto again = g_pick_cache.find(key);   // the map may have changed while unlocked
  if (again != g_pick_cache.end()) {
    again->second.resolved = true;
    again->second.slot = -1;
    again->second.d = *out;
  }
  return RTCDF_SUCCESS;
}

rtcdf_status_t pick_config(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                           hipStream_t stream, rtcdf_config_t* out, bool wait) {
  const int mode = g_mode.load();
  const uint32_t R = (uint32_t)(maxVal - minVal);
  if (mode == RTCDF_CONFIG_LEARNED && keys_in != nullptr) {
    Decision d;
    rtcdf_status_t st = learned_decision(keys_in, n, minVal, maxVal, stream, wait, &d);
    if (st != RTCDF_SUCCESS) return st;
    *out = d.cfg;
    t_last_index = d.index;
    t_last_source = d.source;
    return RTCDF_SUCCESS;
  }
  *out = static_choice(n, R, mode);
  t_last_index = grid_index(*out, n, R);
  t_last_source = RTCDF_PICK_STATIC;
  return RTCDF_SUCCESS;
}

}  // namespace rtcdf

using namespace rtcdf;

extern "C" {

rtcdf_status_t rtcdf_set_config_mode(int mode) {
  if (mode != RTCDF_CONFIG_DEFAULT && mode != RTCDF_CONFIG_TUNED && mode != RTCDF_CONFIG_LEARNED)
    return RTCDF_ERROR_INVALID_VALUE;
  g_mode.store(mode);
  return RTCDF_SUCCESS;
}

int rtcdf_get_config_mode(void) { return g_mode.load(); }

rtcdf_status_t rtcdf_set_learned_fallback(int on) {
  g_fallback.store(on != 0);
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  drop_picks();
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_clear_pick_cache(void) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  drop_picks();
  g_class_best.clear();
  return RTCDF_SUCCESS;
}

int rtcdf_last_pick_index(void) { return t_last_index; }
int rtcdf_last_pick_source(void) { return t_last_source; }

rtcdf_status_t rtcdf_pick_config(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                                 hipStream_t stream, rtcdf_config_t* cfg) {
  if (cfg == nullptr || maxVal <= minVal) return RTCDF_ERROR_INVALID_VALUE;
  if ((uint64_t)(maxVal - minVal) > (uint64_t)RTCDF_MAX_RANGE) return RTCDF_ERROR_RANGE_TOO_LARGE;
  return pick_config(keys_in, n, minVal, maxVal, stream, cfg, true);
}

rtcdf_status_t rtcdf_config_grid(rtcdf_config_t* configs, uint8_t* valid) {
  for (int i = 0; i < RTCDF_GRID_SIZE; ++i) {
    if (configs) configs[i] = grid_config(i);
    if (valid) valid[i] = grid_valid(i) ? 1 : 0;
  }
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_load_tuned_table(const char* path) {
  if (path == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  std::vector<TunedRow> rows;
  char line[512];
  bool bad = false;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    TunedRow r;
    unsigned t, it, b, fl = 0;
    const int got = std::sscanf(line, "%lf %lf %u %u %u %u", &r.log2n, &r.log2r, &t, &it, &b, &fl);
    if (got != 5 && got != 6) {
      bad = true;
      break;
    }
    r.cfg = {t, it, b, fl};
    if (!config_valid(r.cfg)) {
      bad = true;
      break;
    }
    rows.push_back(r);
  }
  std::fclose(f);
  if (bad || rows.empty()) return RTCDF_ERROR_INVALID_VALUE;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_tuned.swap(rows);
  return RTCDF_SUCCESS;
}

// Model file: "RTCDFMLP" | u32 version (1 to 4) | u32 inputs, hidden,
// outputs, params | f32 log2n_lo, log2n_hi, log2r_lo, log2r_hi | versions 2
// and up: f32 margin, f32 zmax | f32 mean[inputs] | f32 sd[inputs] |
// f32 params[params] | u8 valid[outputs].  The outputs must match this
// library's grid (version 4: RTCDF_GRID_SIZE points, the option points with
// 4-bit counters; files of other grids are refused).
rtcdf_status_t rtcdf_load_model(const char* path) {
  if (path == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  FILE* f = std::fopen(path, "rb");
  if (f == nullptr) return RTCDF_ERROR_NO_MODEL;
  Model m;
  char magic[8];
  uint32_t hdr[5];
  float ranges[4];
  float gate[2] = {0.f, 0.f};   // margin, zmax
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "RTCDFMLP", 8) == 0 &&
            std::fread(hdr, 4, 5, f) == 5 && hdr[0] >= 1 && hdr[0] <= 4 && hdr[1] == (uint32_t)kMlpIn &&
            hdr[2] == (uint32_t)kMlpHidden && hdr[3] == (uint32_t)kMlpOut && hdr[4] == (uint32_t)kMlpParams &&
            std::fread(ranges, 4, 4, f) == 4 && (hdr[0] == 1 || std::fread(gate, 4, 2, f) == 2);
  ok = ok && std::isfinite(gate[0]) && gate[0] >= 0.f && std::isfinite(gate[1]) && gate[1] >= 0.f;
  if (ok) {
    m.norm.resize(2 * kMlpIn);
    m.params.resize(kMlpParams);
    m.valid.resize(kMlpOut);
    ok = std::fread(m.norm.data(), 4, 2 * kMlpIn, f) == (size_t)(2 * kMlpIn) &&
         std::fread(m.params.data(), 4, kMlpParams, f) == (size_t)kMlpParams &&
         std::fread(m.valid.data(), 1, kMlpOut, f) == (size_t)kMlpOut;
  }
  std::fclose(f);
  if (!ok) return RTCDF_ERROR_INVALID_VALUE;
  for (int i = 0; i < kMlpIn; ++i)
    if (!(m.norm[kMlpIn + i] > 0.f) || !std::isfinite(m.norm[i])) return RTCDF_ERROR_INVALID_VALUE;
  for (float p : m.params)
    if (!std::isfinite(p)) return RTCDF_ERROR_INVALID_VALUE;
  for (int i = 0; i < kMlpOut; ++i)
    if (m.valid[i] && !grid_valid(i)) return RTCDF_ERROR_INVALID_VALUE;
  m.log2n_lo = ranges[0];
  m.log2n_hi = ranges[1];
  m.log2r_lo = ranges[2];
  m.log2r_hi = ranges[3];
  m.margin = gate[0];
  m.zmax = gate[1];
  m.loaded = true;
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_model = m;
  ++g_model_generation;
  drop_picks();
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_unload_model(void) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_model = Model();
  ++g_model_generation;
  drop_picks();
  return RTCDF_SUCCESS;
}

// ---- autotuner

rtcdf_status_t rtcdf_autotune(const int32_t* keys_in, int32_t* keys_out, size_t n, int64_t minVal,
                              int64_t maxVal, uint32_t warmup, uint32_t reps, float* times_ms,
                              rtcdf_config_t* best, hipStream_t stream) {
  if (times_ms == nullptr || reps == 0 || n == 0) return RTCDF_ERROR_INVALID_VALUE;
  std::vector<hipEvent_t> ev(2 * reps, nullptr);
  for (auto& e : ev) {
    hipError_t he = hipEventCreate(&e);
    if (he != hipSuccess) return hip_fail(he);
  }
  rtcdf_status_t st = RTCDF_SUCCESS;
  float best_t = 0.f;
  int best_i = -1;
  std::vector<float> samples(reps);
  for (int i = 0; i < RTCDF_GRID_SIZE && st == RTCDF_SUCCESS; ++i) {
    times_ms[i] = -1.f;
    if (!grid_valid(i)) continue;
    const rtcdf_config_t c = grid_config(i);
    for (uint32_t w = 0; w < warmup && st == RTCDF_SUCCESS; ++w)
      st = rtcdf_sort_with_config(keys_in, keys_out, n, minVal, maxVal, &c, stream);
    for (uint32_t r = 0; r < reps && st == RTCDF_SUCCESS; ++r) {
      (void)hipEventRecord(ev[2 * r], stream);
      st = rtcdf_sort_with_config(keys_in, keys_out, n, minVal, maxVal, &c, stream);
      (void)hipEventRecord(ev[2 * r + 1], stream);
    }
    if (st != RTCDF_SUCCESS) break;
    hipError_t he = hipEventSynchronize(ev[2 * reps - 1]);
    if (he != hipSuccess) {
      st = hip_fail(he);
      break;
    }
    for (uint32_t r = 0; r < reps; ++r) (void)hipEventElapsedTime(&samples[r], ev[2 * r], ev[2 * r + 1]);
    std::sort(samples.begin(), samples.end());
    const float med = reps % 2 ? samples[reps / 2] : 0.5f * (samples[reps / 2 - 1] + samples[reps / 2]);
    times_ms[i] = med;
    if (best_i < 0 || med < best_t) {
      best_t = med;
      best_i = i;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (st == RTCDF_SUCCESS && best) *best = grid_config(best_i);
  return st;
}

// ---- picker kernels

rtcdf_status_t rtcdf_sketch(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                            float* d_features, hipStream_t stream) {
  if (d_features == nullptr || maxVal <= minVal || (n > 0 && keys_in == nullptr)) return RTCDF_ERROR_INVALID_VALUE;
  hipError_t e = launch_sketch(keys_in, n, minVal, (uint64_t)(maxVal - minVal), kSketchSamples, d_features, stream);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

rtcdf_status_t rtcdf_mlp_forward(const float* d_params, const float* d_X, uint32_t batch, float* d_Y,
                                 hipStream_t stream) {
  if (batch == 0) return RTCDF_SUCCESS;
  if (d_params == nullptr || d_X == nullptr || d_Y == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  hipError_t e = launch_mlp_forward(d_params, d_X, batch, nullptr, nullptr, d_Y, stream);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

rtcdf_status_t rtcdf_mlp_workspace_bytes(uint32_t batch, size_t* bytes) {
  if (bytes == nullptr) return RTCDF_ERROR_INVALID_VALUE;
  *bytes = (mlp_grad_scratch_floats(batch) + kMlpParams + 64) * sizeof(float);
  return RTCDF_SUCCESS;
}

static uint32_t mask_count_host(const float* d_M, uint32_t batch, hipStream_t stream, rtcdf_status_t* st) {
  std::vector<float> h((size_t)batch * kMlpOut);
  hipError_t e = hipMemcpyAsync(h.data(), d_M, h.size() * sizeof(float), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    *st = hip_fail(e);
    return 0;
  }
  double c = 0;
  for (float v : h) c += v;
  *st = c > 0 ? RTCDF_SUCCESS : RTCDF_ERROR_INVALID_VALUE;
  return (uint32_t)c;
}

rtcdf_status_t rtcdf_mlp_gradient(const float* d_params, const float* d_X, const float* d_T, const float* d_M,
                                  uint32_t batch, float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes,
                                  hipStream_t stream) {
  if (batch == 0 || !d_params || !d_X || !d_T || !d_M || !d_grad || !d_ws) return RTCDF_ERROR_INVALID_VALUE;
  size_t need;
  rtcdf_mlp_workspace_bytes(batch, &need);
  if (ws_bytes < need) return RTCDF_ERROR_WORKSPACE_TOO_SMALL;
  rtcdf_status_t st;
  const uint32_t count = mask_count_host(d_M, batch, stream, &st);
  if (st != RTCDF_SUCCESS) return st;
  hipError_t e = launch_mlp_grad(d_params, d_X, d_T, d_M, batch, 1.f / (float)count, d_grad, d_loss,
                                 static_cast<float*>(d_ws), stream);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

rtcdf_status_t rtcdf_mlp_adam_step(float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t t,
                                   float lr, float beta1, float beta2, float eps, hipStream_t stream) {
  if (!d_params || !d_grad || !d_m || !d_v || t == 0) return RTCDF_ERROR_INVALID_VALUE;
  hipError_t e = launch_adam(d_params, d_grad, d_m, d_v, lr, beta1, beta2, eps, t, stream);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

rtcdf_status_t rtcdf_mlp_train(float* d_params, float* d_m, float* d_v, uint32_t t0, const float* d_X,
                               const float* d_T, const float* d_M, uint32_t batch, uint32_t steps, float lr,
                               void* d_ws, size_t ws_bytes, float* d_loss_history, hipStream_t stream) {
  if (!d_params || !d_m || !d_v || batch == 0 || !d_ws) return RTCDF_ERROR_INVALID_VALUE;
  size_t need;
  rtcdf_mlp_workspace_bytes(batch, &need);
  if (ws_bytes < need) return RTCDF_ERROR_WORKSPACE_TOO_SMALL;
  rtcdf_status_t st;
  const uint32_t count = mask_count_host(d_M, batch, stream, &st);
  if (st != RTCDF_SUCCESS) return st;
  float* scratch = static_cast<float*>(d_ws);
  float* grad = scratch + mlp_grad_scratch_floats(batch);
  for (uint32_t k = 0; k < steps; ++k) {
    hipError_t e = launch_mlp_grad(d_params, d_X, d_T, d_M, batch, 1.f / (float)count, grad,
                                   d_loss_history ? d_loss_history + k : nullptr, scratch, stream);
    if (e == hipSuccess) e = launch_adam(d_params, grad, d_m, d_v, lr, 0.9f, 0.999f, 1e-8f, t0 + k + 1, stream);
    if (e != hipSuccess) return hip_fail(e);
  }
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_mlp_pick(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                              const float* d_params, const float* d_norm, const uint8_t* d_valid,
                              uint32_t* d_index, float* d_pred, hipStream_t stream) {
  if (!keys_in || n == 0 || maxVal <= minVal || !d_params || !d_norm || !d_valid || !d_index ||
      (reinterpret_cast<uintptr_t>(d_params) & 15u))
    return RTCDF_ERROR_INVALID_VALUE;
  hipError_t e = launch_pick(keys_in, n, minVal, (uint64_t)(maxVal - minVal), kSketchSamples, d_params, d_norm,
                             d_valid, d_index, d_pred, nullptr, nullptr, stream);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

}  // extern "C"
