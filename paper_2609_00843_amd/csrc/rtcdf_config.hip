// rtcdf_config.hip -- where rtcdf_sort gets its kernel configuration from when
// the caller passes none: a static per-range table (DEFAULT), a tuning
// database (TUNED) or the learned picker (LEARNED).
#include <hip/hip_runtime.h>

#include <atomic>

#include "../../include/rtcdf.h"
#include "rtcdf_internal.h"

namespace rtcdf {

static std::atomic<int> g_mode{RTCDF_CONFIG_DEFAULT};

// Static default: one row per range class (upper bound on R, inclusive).
struct DefaultRow {
  uint32_t max_range;
  rtcdf_config_t cfg;
};
static const DefaultRow kDefaultTable[] = {
    {1u << 28, {2048, 16, 1, 0}},
};

rtcdf_config_t default_config(size_t n, uint32_t R) {
  (void)n;
  for (const DefaultRow& row : kDefaultTable)
    if (R <= row.max_range) return row.cfg;
  return kDefaultTable[sizeof(kDefaultTable) / sizeof(kDefaultTable[0]) - 1].cfg;
}

rtcdf_status_t pick_config(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                           hipStream_t stream, rtcdf_config_t* out) {
  (void)keys_in;
  (void)stream;
  *out = default_config(n, (uint32_t)(maxVal - minVal));
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

rtcdf_status_t rtcdf_pick_config(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                                 hipStream_t stream, rtcdf_config_t* cfg) {
  if (cfg == nullptr || maxVal <= minVal) return RTCDF_ERROR_INVALID_VALUE;
  if ((uint64_t)(maxVal - minVal) > (uint64_t)RTCDF_MAX_RANGE) return RTCDF_ERROR_RANGE_TOO_LARGE;
  return pick_config(keys_in, n, minVal, maxVal, stream, cfg);
}

}  // extern "C"
