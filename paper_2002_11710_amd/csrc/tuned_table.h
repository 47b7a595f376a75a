// tuned_table.h -- default schedule and launch shape of small solves by move
// slots per iteration (M*(M+V) + M*(M-1)/2).  Rows are tried in order; the
// first row whose max_slots exceeds the solve's slots applies: wave = 1 gives
// such solves one wavefront each (the wave schedule), else one workgroup of
// `block` threads with swap units of `chunk` columns.
// Written by paper_2002_11710_amd/autotune.py from timings on gfx950.
#pragma once
#include <cstdint>

namespace at {
struct TunedRow { int64_t max_slots; int wave; int block; int chunk; };
static const TunedRow kTuned[] = {
    {2000, 0, 256, 8},
    {4000, 0, 256, 8},
    {12000, 0, 256, 32},
    {30000, 0, 256, 32},
    {60000, 0, 512, 32},
    {100000, 0, 1024, 32},
    {INT64_MAX, 0, 1024, 32},
};
}  // namespace at
