// rtcdf_default_table.h -- static default configuration per range class.
// Written by paper_2609_00843_amd/tune.py from measured tuning rows (the
// geometric mean of relative times per range, as in Sec. 4.1 of the paper);
// rows are ordered by max_range and the first row with R <= max_range applies.
// Source: tune_train.jsonl, 2000 arrays
#pragma once

#include "../../include/rtcdf.h"

namespace rtcdf {

struct DefaultRow {
  uint32_t max_range;
  rtcdf_config_t cfg;
};

static const DefaultRow kDefaultTable[] = {
    {181u, {2048, 8, 2, 0}},   // log2 R ~ 7
    {362u, {1024, 8, 2, 0}},   // log2 R ~ 8
    {724u, {1024, 8, 2, 0}},   // log2 R ~ 9
    {1448u, {32768, 8, 1, 0}},   // log2 R ~ 10
    {2896u, {8192, 8, 1, 0}},   // log2 R ~ 11
    {5792u, {1024, 8, 1, 0}},   // log2 R ~ 12
    {11585u, {1024, 8, 1, 0}},   // log2 R ~ 13
    {23170u, {1024, 8, 1, 0}},   // log2 R ~ 14
    {46340u, {1024, 16, 1, 0}},   // log2 R ~ 15
    {92681u, {1024, 16, 1, 0}},   // log2 R ~ 16
    {185363u, {1024, 16, 1, 0}},   // log2 R ~ 17
    {370727u, {1024, 8, 1, 0}},   // log2 R ~ 18
    {1u << 28, {8192, 8, 1, 0}},   // wider than the tuning rows
};

}  // namespace rtcdf
