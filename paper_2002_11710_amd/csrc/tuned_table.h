// tuned_table.h -- default launch shape of the one-workgroup-per-solve schedule
// by move slots per iteration (M*(M+V) + M*(M-1)/2).  Rows are tried in order;
// the first row whose max_slots exceeds the solve's slots applies.
// Written by paper_2002_11710_amd/autotune.py from timings on gfx950.
#pragma once
#include <cstdint>

namespace at {
struct TunedRow { int64_t max_slots; int block; int chunk; };
static const TunedRow kTuned[] = {
    {4000, 256, 8},
    {12000, 256, 32},
    {30000, 256, 32},
    {60000, 512, 32},
    {100000, 1024, 32},
    {INT64_MAX, 1024, 32},
};
}  // namespace at
