// rtcdf_config.hip -- where rtcdf_sort gets its kernel configuration from when
// the caller passes none (DEFAULT: static per-range table; TUNED: nearest
// entry of a loaded tuning table; LEARNED: the MLP picker), the configuration
// grid, the exhaustive autotuner, and the C ABI of the picker's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/rtcdf.h"
#include "rtcdf_default_table.h"
#include "rtcdf_internal.h"

namespace rtcdf {

static std::atomic<int> g_mode{RTCDF_CONFIG_DEFAULT};

// ------------------------------------------------------------------ grid

rtcdf_config_t grid_config(int i) {
  rtcdf_config_t c;
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

// -------------------------------------------------------------- tuned table

struct TunedRow {
  double log2n, log2r;
  rtcdf_config_t cfg;
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
  return true;
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
// Pick results: word 0 the argmin index, words 1..kMlpOut the predictions,
// then the largest |normalised feature|.
constexpr int kPickWords = 2 + kMlpOut;
struct DeviceModel {
  float* params = nullptr;
  float* norm = nullptr;
  uint8_t* valid = nullptr;
  uint32_t* out = nullptr;              // kPickWords
  uint32_t* host_out = nullptr;         // pinned, kPickWords
  uint64_t generation = 0;
};
static Model g_model;
static uint64_t g_model_generation = 0;
static std::map<int, DeviceModel> g_dev_models;

static rtcdf_status_t upload_model(int dev, DeviceModel** out) {
  DeviceModel& d = g_dev_models[dev];
  if (d.out == nullptr) {
    hipError_t e = hipMalloc(&d.params, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&d.norm, sizeof(float) * 2 * kMlpIn);
    if (e == hipSuccess) e = hipMalloc(&d.valid, kMlpOut);
    if (e == hipSuccess) e = hipMalloc(&d.out, sizeof(uint32_t) * kPickWords);
    if (e == hipSuccess) e = hipHostMalloc(&d.host_out, sizeof(uint32_t) * kPickWords);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (d.generation != g_model_generation) {
    hipError_t e = hipMemcpy(d.params, g_model.params.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(d.norm, g_model.norm.data(), sizeof(float) * 2 * kMlpIn, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.valid, g_model.valid.data(), kMlpOut, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    d.generation = g_model_generation;
  }
  *out = &d;
  return RTCDF_SUCCESS;
}

static int grid_index(const rtcdf_config_t& c) {
  for (int i = 0; i < kMlpOut; ++i) {
    const rtcdf_config_t g = grid_config(i);
    if (g.tile_width == c.tile_width && g.items_per_thread == c.items_per_thread &&
        g.blocks_per_tile == c.blocks_per_tile)
      return i;
  }
  return -1;
}

// The configuration used when the learned model does not decide.
static rtcdf_config_t static_config(size_t n, uint32_t R, int mode) {
  rtcdf_config_t c;
  if (mode != RTCDF_CONFIG_DEFAULT && tuned_config(n, R, &c)) return c;
  return default_config(n, R);
}

static rtcdf_status_t learned_config(const int32_t* keys, size_t n, int64_t minVal, int64_t maxVal,
                                     hipStream_t stream, rtcdf_config_t* out, bool* used) {
  *used = false;
  const rtcdf_config_t fallback = static_config(n, (uint32_t)(maxVal - minVal), RTCDF_CONFIG_TUNED);
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  if (!g_model.loaded || keys == nullptr || n == 0) return RTCDF_SUCCESS;
  const double a = std::log2((double)n), b = std::log2((double)(maxVal - minVal));
  // Outside the ranges the network was trained on it is not consulted.
  if (a < g_model.log2n_lo - 0.5 || a > g_model.log2n_hi + 0.5 || b < g_model.log2r_lo - 0.5 ||
      b > g_model.log2r_hi + 0.5)
    return RTCDF_SUCCESS;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  DeviceModel* d = nullptr;
  rtcdf_status_t st = upload_model(dev, &d);
  if (st != RTCDF_SUCCESS) return st;
  e = launch_pick(keys, n, minVal, (uint64_t)(maxVal - minVal), kSketchSamples, d->params, d->norm, d->valid,
                  d->out, reinterpret_cast<float*>(d->out + 1),
                  reinterpret_cast<float*>(d->out + 1 + kMlpOut), stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d->host_out, d->out, sizeof(uint32_t) * kPickWords, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e);
  const uint32_t idx = d->host_out[0];
  if (idx >= (uint32_t)kMlpOut || !grid_valid((int)idx)) return RTCDF_SUCCESS;
  // Keys whose sketch lies outside the features the network was trained on
  // (farther than zmax sd from the training mean in some feature) are left to
  // the static configuration, like arrays outside the trained n and R ranges.
  float z;
  std::memcpy(&z, d->host_out + 1 + kMlpOut, sizeof(float));
  if (g_model.zmax > 0.f && !(z <= g_model.zmax)) return RTCDF_SUCCESS;
  // Act on the prediction only where it promises at least the margin over
  // the configuration that would be used otherwise.
  const float* pred = reinterpret_cast<const float*>(d->host_out + 1);
  const int si = grid_index(fallback);
  if (si >= 0 && g_model.valid[si] && pred[si] - pred[idx] < g_model.margin) return RTCDF_SUCCESS;
  *out = grid_config((int)idx);
  *used = true;
  return RTCDF_SUCCESS;
}

// Output method (the adaptive selection between Alg. 7 and Alg. 3 that the
// paper leaves as future work in Sec. 4.1): the prefix maximum when the range
// is at least kPmaxMinRange and at least n.  There the search path spends its
// output stage walking many sparse values per output chunk, while the
// prefix-maximum steps are written one value per thread by the local-CDF
// stage; measured on MI355X over n in [10^3, 10^7] and R in [2^8, 2^24] with
// uniform, normal and all-equal keys.  RTCDF_DEV_OUTPUT_RULE=0 keeps the
// search everywhere (for measurement).
constexpr uint32_t kPmaxMinRange = 1u << 14;

static uint32_t output_method_flags(size_t n, uint32_t R) {
  const char* v = std::getenv("RTCDF_DEV_OUTPUT_RULE");
  if (v != nullptr && v[0] == '0' && v[1] == 0) return 0u;
  return (R >= kPmaxMinRange && (uint64_t)R >= (uint64_t)n) ? RTCDF_FLAG_OUTPUT_PREFIX_MAX : 0u;
}

static rtcdf_status_t pick_kernel_config(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                                         hipStream_t stream, rtcdf_config_t* out) {
  const int mode = g_mode.load();
  const uint32_t R = (uint32_t)(maxVal - minVal);
  if (mode == RTCDF_CONFIG_LEARNED) {
    bool used = false;
    rtcdf_status_t st = learned_config(keys_in, n, minVal, maxVal, stream, out, &used);
    if (st != RTCDF_SUCCESS) return st;
    if (used) return RTCDF_SUCCESS;
  }
  if (mode != RTCDF_CONFIG_DEFAULT && tuned_config(n, R, out)) return RTCDF_SUCCESS;
  *out = default_config(n, R);
  return RTCDF_SUCCESS;
}

rtcdf_status_t pick_config(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                           hipStream_t stream, rtcdf_config_t* out) {
  rtcdf_status_t st = pick_kernel_config(keys_in, n, minVal, maxVal, stream, out);
  if (st == RTCDF_SUCCESS) out->flags = output_method_flags(n, (uint32_t)(maxVal - minVal));
  return st;
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

rtcdf_status_t rtcdf_pick_config(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                                 hipStream_t stream, rtcdf_config_t* cfg) {
  if (cfg == nullptr || maxVal <= minVal) return RTCDF_ERROR_INVALID_VALUE;
  if ((uint64_t)(maxVal - minVal) > (uint64_t)RTCDF_MAX_RANGE) return RTCDF_ERROR_RANGE_TOO_LARGE;
  return pick_config(keys_in, n, minVal, maxVal, stream, cfg);
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
    unsigned t, it, b;
    if (std::sscanf(line, "%lf %lf %u %u %u", &r.log2n, &r.log2r, &t, &it, &b) != 5) {
      bad = true;
      break;
    }
    r.cfg = {t, it, b, 0};
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

// Model file: "RTCDFMLP" | u32 version (1 or 2) | u32 inputs, hidden, outputs,
// params | f32 log2n_lo, log2n_hi, log2r_lo, log2r_hi | version 2: f32 margin,
// f32 zmax | f32 mean[inputs] | f32 sd[inputs] | f32 params[params] |
// u8 valid[outputs].
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
            std::fread(hdr, 4, 5, f) == 5 && (hdr[0] == 1 || hdr[0] == 2) && hdr[1] == (uint32_t)kMlpIn &&
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
  return RTCDF_SUCCESS;
}

rtcdf_status_t rtcdf_unload_model(void) {
  std::lock_guard<std::mutex> lk(g_cfg_mu);
  g_model = Model();
  ++g_model_generation;
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
  if (!keys_in || n == 0 || maxVal <= minVal || !d_params || !d_norm || !d_valid || !d_index)
    return RTCDF_ERROR_INVALID_VALUE;
  hipError_t e = launch_pick(keys_in, n, minVal, (uint64_t)(maxVal - minVal), kSketchSamples, d_params, d_norm,
                             d_valid, d_index, d_pred, nullptr, stream);
  return e == hipSuccess ? RTCDF_SUCCESS : hip_fail(e);
}

}  // extern "C"
