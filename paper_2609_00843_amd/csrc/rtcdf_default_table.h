// rtcdf_default_table.h -- static default configuration per range class.
// Written by paper_2609_00843_amd/tune.py from measured tuning rows (the
// geometric mean of relative times per range, as in Sec. 4.1 of the paper);
// rows are ordered by max_range and the first row with R <= max_range applies.
#pragma once

#include "../../include/rtcdf.h"

namespace rtcdf {

struct DefaultRow {
  uint32_t max_range;
  rtcdf_config_t cfg;
};

static const DefaultRow kDefaultTable[] = {
    {1u << 28, {2048, 16, 1, 0}},
};

}  // namespace rtcdf
